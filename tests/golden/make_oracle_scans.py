"""Expected outputs of the full-size scans, written by the CPU oracle alone.

Each configuration is a seeded sample of one of the scan workloads (the whole
grid for the 64 x 64 scan).  For every sampled orbit the oracle runs five
times: on the state as generated, and with r0 or p0 moved up or down by one
ulp.  The spread of the five FLIs is the oracle's own rounding sensitivity
at that orbit and end time (a one-ulp change of the initial state changes
every rounding that follows); the GPU parity tests take their per-orbit FLI
tolerance from it.

Run from the repository root:  python tests/golden/make_oracle_scans.py [name ...]
It imports only the oracle and the seeded input generators, and writes
tests/golden/oracle_scan_<name>.txt (one row per sampled orbit):

    index status label steps fli fli_r0_up fli_r0_down fli_p0_up fli_p0_down

`load(name)` reads a file back as a dict of arrays.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1802_00147_amd import workloads as W  # noqa: E402  (seeded inputs only)


def _grid314(beta, qm):
    return W.grid314(beta=beta, quad_mono=qm)


# name -> (workload factory, sample size (None = every orbit), sample seed, model)
CONFIGS = {
    "grid64": (W.grid64, None, 0, {}),
    "grid314_b1_qm1": (lambda: _grid314(1.0, 1), 986, 101, dict(quad_mono=1)),
    "grid314_b1_qm0": (lambda: _grid314(1.0, 0), 200, 102, dict(quad_mono=0)),
    "grid314_b0.5_qm1": (lambda: _grid314(0.5, 1), 200, 103, dict(quad_mono=1)),
    "grid314_b0.5_qm0": (lambda: _grid314(0.5, 0), 200, 104, dict(quad_mono=0)),
    "batch1M": (W.batch, 1000, 105, {}),
    "fig7_phys": (W.fig7, 986, 106, dict(spin_units=0)),
    "fig7_eq8": (W.fig7, 986, 107, dict(spin_units=1)),
    "grid4096": (W.grid4096, 1000, 108, {}),
}


TWINS = ("fli_r", "fli_rm", "fli_p", "fli_pm")
COLUMNS = ("index", "status", "label", "steps", "fli") + TWINS


def sample(name):
    """(workload, sample indices) of a configuration."""
    make, k, seed, _ = CONFIGS[name]
    wl = make()
    idx = np.arange(wl.n) if k is None else W.strided_sample(wl.n, k, seed=seed)
    return wl, idx


def path(name):
    return os.path.join(HERE, f"oracle_scan_{name}.txt")


def oracle_rows(name, idx_subset=None, nthreads=None):
    """Run the oracle on a configuration's sample (or on the given subset of
    its indices); returns the rows as a dict of arrays."""
    import oracle as O
    wl, idx = sample(name)
    model = CONFIGS[name][3]
    if idx_subset is not None:
        idx = np.asarray(idx_subset)
    sub = wl.subset(idx)
    nthreads = nthreads or os.cpu_count() or 1
    y0 = O.init_state(sub.r0, sub.p0, sub.th1, sub.ph1, sub.th2, sub.ph2, sub.beta, sub.chi1, sub.chi2,
                      model=model)
    runs = []
    # As generated; r_x one ulp up and down; p_y one ulp up and down.
    for comp, to in ((None, 0.0), (0, np.inf), (0, -np.inf), (4, np.inf), (4, -np.inf)):
        y = y0.copy()
        if comp is not None:
            y[:, comp] = np.nextafter(y[:, comp], to)
        runs.append(O.fli_scan(y, sub.t_end, sub.beta, sub.chi1, sub.chi2, model=model, nthreads=nthreads))
    base = runs[0]
    rows = dict(index=idx.astype(np.int64), status=base["status"].astype(np.int64),
                label=base["label"].astype(np.int64), steps=base["steps"].astype(np.int64), fli=base["fli"])
    for k, key in enumerate(TWINS):
        rows[key] = runs[1 + k]["fli"]
    return rows


def write(name, rows, seconds):
    wl, _ = sample(name)
    make, k, seed, model = CONFIGS[name]
    with open(path(name), "w") as f:
        f.write(f"# oracle scan expectations: {name} ({wl.n} orbits; "
                f"{'all' if k is None else f'{k} sampled with seed {seed}'}), model {model}, "
                f"t_end {'per orbit' if isinstance(wl.t_end, np.ndarray) else wl.t_end:}, RK4 h=1, "
                f"six-integral correction\n")
        f.write(f"# written by tests/golden/make_oracle_scans.py in {seconds:.0f} s\n")
        f.write("# index status label steps fli fli_r0_up fli_r0_down fli_p0_up fli_p0_down\n")
        for i in range(len(rows["index"])):
            f.write(f"{rows['index'][i]} {rows['status'][i]} {rows['label'][i]} {rows['steps'][i]} " +
                    " ".join(repr(float(rows[k][i])) for k in ("fli",) + TWINS) + "\n")


def load(name):
    data = np.loadtxt(path(name), comments="#", ndmin=2)
    out = {c: data[:, k] for k, c in enumerate(COLUMNS)}
    for c in ("index", "status", "label", "steps"):
        out[c] = out[c].astype(np.int64)
    return out


if __name__ == "__main__":
    names = sys.argv[1:] or list(CONFIGS)
    for name in names:
        t0 = time.perf_counter()
        rows = oracle_rows(name)
        dt = time.perf_counter() - t0
        write(name, rows, dt)
        ok = rows["status"] == 0
        print(f"{name}: {len(rows['index'])} orbits, {int(np.sum(rows['label'] == 1))} chaotic, "
              f"{int(np.sum(~ok))} removed, {dt:.0f} s", flush=True)
