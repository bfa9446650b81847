"""GPU parity: every entry point of the HIP library against the CPU oracle on
the same seeded inputs, called through the C ABI (Python binding).

Tolerances (floating point; the GPU contracts a*b+c into FMAs and uses a
refined hardware reciprocal square root where the oracle uses IEEE operations
without contraction, so the two round differently):
  * RHS, invariants, initial states: 1e-13 of the largest component per row
    (a few ulps on terms that partly cancel).
  * One correction: 1e-13 relative per row (1e-12 for the dual scaling,
    whose 2x2 Newton system may have a condition number up to 1e3).
  * State after integration up to t = 1e3 (1000 steps of h = 1): 1e-10
    relative (the stated parity bound for trajectories).
  * FLI of regular orbits at the end of the single-orbit run (t = 1e4):
    1e-6 relative, the stated parity bound.
  * FLI at other times and in short runs: 3e-5 absolute.  The separation d is
    the difference of two states of size |y| ~ 10-60 that each carry rounding
    of order eps |y| per step; with d0 = 1e-8 that noise is ~1e-7 of d per
    step and accumulates as a random walk (~1e-5 of d after 1e4 steps), i.e.
    ~1e-5 in log10(d / d0) whichever side computes it.
  * With a correction after every step, each trajectory also carries the
    rounding of its projection, amplified by up to ~1e2 along the direction in
    which the energy row is nearly dependent on the J rows (and up to ~1e3 in
    the dual scaling's 2x2 solve): FLIs of short runs then agree to 3e-4.
  * Labels and status codes exact.
"""
FLI_ABS = 3e-5
FLI_ABS_CORRECTED = 3e-4
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import DEV, dev, from_soa, orbit_states, random_states, rel_err_rows, to_soa

pytestmark = pytest.mark.gpu

MODELS = [
    dict(),
    dict(spin_units=1),
    dict(pn_order=1, spin_spin=0),
    dict(pn_order=0, spin_orbit=0, quad_mono=0),
    dict(quad_mono=0),
]


@pytest.fixture(scope="module")
def pn():
    assert torch.cuda.is_available(), "GPU parity tests need a ROCm device"
    from paper_1802_00147_amd import pn as P
    P.lib()
    return P


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("per_orbit", [False, True])
def test_rhs_parity(pn, model, per_orbit):
    rng = np.random.default_rng(100)
    n = 10000
    y = random_states(rng, n)
    if per_orbit:
        beta, c1, c2 = rng.uniform(0.1, 1, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n)
        ref = O.rhs(y, beta, c1, c2, model=model)
        got = from_soa(pn.rhs(to_soa(y), dev(beta), dev(c1), dev(c2), model=model))
    else:
        ref = O.rhs(y, 0.6, 0.9, 0.4, model=model)
        got = from_soa(pn.rhs(to_soa(y), 0.6, 0.9, 0.4, model=model))
    assert np.all(rel_err_rows(got, ref) <= 1e-13)


def test_rhs_ragged_and_padded(pn):
    """n not a multiple of the 64-lane wavefront, ld > n: padding is untouched."""
    rng = np.random.default_rng(101)
    n, ld = 1000 + 37, 1100
    y = random_states(rng, n)
    ys = to_soa(y, ld)
    f = pn.rhs(ys, 1.0, 1.0, 1.0, n=n)
    ref = O.rhs(y, 1.0, 1.0, 1.0)
    assert np.all(rel_err_rows(from_soa(f, n), ref) <= 1e-13)
    # Single orbit and empty batch.
    f1 = pn.rhs(to_soa(y[:1]), 1.0, 1.0, 1.0)
    assert np.all(rel_err_rows(from_soa(f1), ref[:1]) <= 1e-13)
    pn.rhs(torch.zeros((12, 1), dtype=torch.float64, device=DEV), 1.0, 1.0, 1.0, n=0)


@pytest.mark.parametrize("model", MODELS[:2])
def test_invariants_parity(pn, model):
    rng = np.random.default_rng(102)
    y = random_states(rng, 5000)
    H, J = O.invariants(y, 0.45, 0.7, 0.2, model=model)
    Hg, Jg = pn.invariants(to_soa(y), 0.45, 0.7, 0.2, model=model)
    Hg, Jg = Hg.cpu().numpy(), Jg.cpu().numpy().T
    scale = np.abs(y[:, :3]).max(axis=1) * np.abs(y[:, 3:6]).max(axis=1) + 1
    assert np.all(np.abs(Hg - H) <= 1e-13 * (np.abs(H) + 1.0 / np.linalg.norm(y[:, :3], axis=1)))
    assert np.all(np.abs(Jg - J).max(axis=1) <= 1e-14 * scale)


def test_init_state_parity(pn):
    rng = np.random.default_rng(103)
    n = 3000
    r0 = rng.uniform(8, 60, n)
    p0 = r0 ** -0.5
    th1, th2 = rng.uniform(0, np.pi, n), rng.uniform(0, np.pi, n)
    ph1, ph2 = rng.uniform(0, 2 * np.pi, n), rng.uniform(0, 2 * np.pi, n)
    beta, c1, c2 = rng.uniform(0.1, 1, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n)
    ref = O.init_state(r0, p0, th1, ph1, th2, ph2, beta, c1, c2)
    got = from_soa(pn.init_state(*[dev(a) for a in (r0, p0, th1, ph1, th2, ph2)], dev(beta), dev(c1), dev(c2)))
    assert np.all(np.abs(got - ref).max(axis=1) <= 4e-16 * np.abs(ref).max(axis=1))


@pytest.mark.parametrize("mode", ["spin", "six", "dual"])
def test_correction_parity(pn, mode):
    rng = np.random.default_rng(104)
    ys, betas = orbit_states(O, rng, 200)
    ref = np.zeros((len(ys), 4))
    for k, (y, b) in enumerate(zip(ys, betas)):
        H, J = O.invariants(y, b, 0.8, 0.6)
        ref[k] = np.concatenate([H, J[0]])
    pert = ys * (1 + 1e-9 * rng.normal(size=ys.shape))
    exp, it_exp = O.manifold_correct(pert, ref, betas, 0.8, 0.6, correction=dict(mode=mode))
    yg = to_soa(pert)
    it = pn.manifold_correct(yg, dev(ref.T), dev(betas), dev(np.full(len(ys), 0.8)), dev(np.full(len(ys), 0.6)),
                             correction=dict(mode=mode))
    got = from_soa(yg)
    # DUAL solves a 2x2 system whose conditioning the guard bounds by 1e3.
    tol = 1e-12 if mode == "dual" else 1e-13
    assert np.all(rel_err_rows(got, exp) <= tol)
    agree = np.mean(it.cpu().numpy() == it_exp)
    assert agree >= 0.95


@pytest.mark.parametrize("method", ["rk4", "rk5"])
@pytest.mark.parametrize("mode", [None, "six", "dual"])
def test_step_parity_to_t1000(pn, method, mode):
    """1000 steps of h = 1 (t = 1e3): state within 1e-10 relative."""
    rng = np.random.default_rng(105)
    ys, betas = orbit_states(O, rng, 96, steps=(1, 3))
    chi1, chi2 = np.full(96, 0.8), np.full(96, 0.6)
    corr = None if mode is None else dict(mode=mode)
    exp = O.step(ys, betas, chi1, chi2, 1000, integrator=dict(method=method), correction=corr)
    yg = to_soa(ys)
    pn.step(yg, dev(betas), dev(chi1), dev(chi2), 1000, integrator=dict(method=method), correction=corr)
    err = rel_err_rows(from_soa(yg), exp)
    assert np.all(err <= 1e-10), err.max()


def test_step_with_given_reference(pn):
    rng = np.random.default_rng(106)
    ys, _ = orbit_states(O, rng, 64, beta=0.7)
    H, J = O.invariants(ys, 0.7, 0.8, 0.6)
    ref = np.column_stack([H, J])
    exp = O.step(ys, 0.7, 0.8, 0.6, 300, correction=dict(mode="six"), ref=ref)
    yg = to_soa(ys)
    pn.step(yg, 0.7, 0.8, 0.6, 300, correction=dict(mode="six"), ref=dev(ref.T))
    assert np.all(rel_err_rows(from_soa(yg), exp) <= 1e-11)


def _scan_both(pn, wl_y0, t_end, beta, c1, c2, n, model=None, integrator=None, correction=None, fli=None,
               trace_every=0, nthreads=8):
    exp = O.fli_scan(wl_y0, t_end, beta, c1, c2, model=model, integrator=integrator, correction=correction,
                     fli=fli, nthreads=nthreads, trace_every=trace_every)
    tb = dev(beta) if isinstance(beta, np.ndarray) else beta
    t1 = dev(c1) if isinstance(c1, np.ndarray) else c1
    t2 = dev(c2) if isinstance(c2, np.ndarray) else c2
    tt = dev(t_end) if isinstance(t_end, np.ndarray) else t_end
    out = pn.fli_scan(to_soa(wl_y0), tt, tb, t1, t2, model=model, integrator=integrator, correction=correction,
                      fli=fli, trace_every=trace_every)
    torch.cuda.synchronize()
    got = {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for k, v in out.items()}
    got["y_final"] = got["y_final"].T.copy()
    if "trace" in got:
        got["trace"] = got["trace"].T.copy()
    return exp, got


def test_scan_single_orbit_c1(pn):
    """Single orbit + shadow, t = 1e4, beta = chi = 1, seeded spin angles,
    r0 = 20: the final FLI within the larger of 1e-6 relative (the stated
    bound) and twice the oracle's own spread over four runs from initial
    states one ulp away (r_x, p_y up and down), which for this orbit is
    itself ~1e-6 relative: the stated bound sits at the FLI's rounding
    noise here, and the GPU is held to that noise.  Trace within
    FLI_ABS_CORRECTED, state at t = 1e4 close."""
    from paper_1802_00147_amd import workloads as W
    wl = W.single()
    y0 = O.init_state(wl.r0, wl.p0, wl.th1, wl.ph1, wl.th2, wl.ph2, 1.0, 1.0, 1.0)
    exp, got = _scan_both(pn, y0, wl.t_end, 1.0, 1.0, 1.0, 1, trace_every=100)
    assert got["status"][0] == exp["status"][0] == 0
    assert got["label"][0] == exp["label"][0]
    spread = 0.0
    for comp, to in ((0, np.inf), (0, -np.inf), (4, np.inf), (4, -np.inf)):
        y1 = y0.copy()
        y1[0, comp] = np.nextafter(y1[0, comp], to)
        spread = max(spread, abs(O.fli_scan(y1, wl.t_end, 1.0, 1.0, 1.0)["fli"][0] - exp["fli"][0]))
    err = abs(got["fli"][0] - exp["fli"][0])
    print(f"single orbit: FLI {exp['fli'][0]:.9f}, GPU - oracle {err:.2e} ({err / exp['fli'][0]:.2e} relative), "
          f"oracle 1-ulp spread {spread:.2e}", flush=True)
    assert err <= max(1e-6 * abs(exp["fli"][0]), 2.0 * spread)
    assert np.all(np.abs(got["trace"][0] - exp["trace"][0]) <= FLI_ABS_CORRECTED)
    assert rel_err_rows(got["y_final"], exp["y_final"])[0] <= 1e-8
    assert got["dH"][0] < 1e-14 and got["dJ"][0] < 1e-14


@pytest.mark.parametrize("method,mode,model", [
    ("rk4", "six", None), ("rk5", "six", None), ("rk4", "dual", None), ("rk4", "none", None),
    ("rk4", "spin", None), ("rk4", "six", dict(spin_units=1)), ("rk4", "six", dict(quad_mono=0, spin_spin=0)),
    ("rk5", "dual", dict(pn_order=1))])
def test_scan_parity_mixed_batch(pn, method, mode, model):
    """Per-orbit beta, chi and t_end; ragged n; short runs (t <= 2000).
    Uncorrected FLIs within FLI_ABS.  A corrected FLI within the larger of
    1e-6 relative and 10 times the oracle's own rounding sensitivity at that
    orbit (the largest FLI change among four oracle runs from initial states
    one ulp away, r_x and p_y up and down), floored at the batch's median
    sensitivity: the rule of the full-size scans (tests/scan_expect.py)."""
    rng = np.random.default_rng(107)
    n = 131
    beta, c1, c2 = rng.uniform(0.1, 1, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n)
    r0 = rng.uniform(8, 40, n)
    y0 = O.init_state(r0, r0 ** -0.5 * rng.uniform(0.9, 1.1, n), rng.uniform(0, np.pi, n),
                      rng.uniform(0, 2 * np.pi, n), rng.uniform(0, np.pi, n), rng.uniform(0, 2 * np.pi, n),
                      beta, c1, c2, model=model)
    t_end = rng.uniform(100, 2000, n)
    exp, got = _scan_both(pn, y0, t_end, beta, c1, c2, n, model=model, integrator=dict(method=method),
                          correction=dict(mode=mode))
    assert np.array_equal(got["status"], exp["status"])
    assert np.array_equal(got["label"], exp["label"])
    ok = exp["status"] == 0
    if mode in ("none", "spin"):
        tol = FLI_ABS
    else:
        sens = np.zeros(n)
        for comp, to in ((0, np.inf), (0, -np.inf), (4, np.inf), (4, -np.inf)):
            y1 = y0.copy()
            y1[:, comp] = np.nextafter(y1[:, comp], to)
            twin = O.fli_scan(y1, t_end, beta, c1, c2, model=model, integrator=dict(method=method),
                              correction=dict(mode=mode), nthreads=8)
            sens = np.fmax(sens, np.abs(twin["fli"] - exp["fli"]))
        floor = float(np.median(sens[ok]))
        tol = np.maximum(1e-6 * np.abs(exp["fli"]), 10.0 * np.maximum(sens, floor))[ok]
    assert np.all(np.abs(got["fli"][ok] - exp["fli"][ok]) <= tol)
    assert np.all(rel_err_rows(got["y_final"][ok], exp["y_final"][ok]) <= 1e-9)
    assert np.array_equal(got["renorms"], exp["renorms"])


def test_scan_status_edge_cases(pn):
    """Unbound, merging, escaping, non-finite and out-of-range parameters
    give the same status codes as the oracle; zero time gives FLI ~ 0."""
    rows = []
    y = np.zeros(12); y[0], y[4] = 10.0, 0.6; rows.append(y)            # unbound
    y = np.zeros(12); y[0], y[4] = 6.0, 0.05; rows.append(y)            # plunges below r = 2
    y = np.zeros(12); y[0], y[4] = 10.0, 0.4; rows.append(y)            # leaves r_esc = 11
    y = np.zeros(12); y[0], y[4] = 10.0, np.nan; rows.append(y)         # non-finite
    y = np.zeros(12); y[0], y[4] = 8.0, 8 ** -0.5; rows.append(y)      # fine (stays inside r_esc)
    y = np.zeros(12); y[0], y[4] = 8.0, 8 ** -0.5; rows.append(y)      # bad beta below
    y0 = np.array(rows)
    n = len(rows)
    beta = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.7])
    c = np.zeros(n)
    exp, got = _scan_both(pn, y0, 2000.0, beta, c, c, n, fli=dict(r_esc=11.0), nthreads=1)
    assert list(exp["status"] & 0xFF) == [4, 1, 2, 3, 0, 5]
    assert np.array_equal(got["status"], exp["status"])
    assert np.array_equal(got["label"], exp["label"])
    # Steps completed: none for the states removed at t = 0 (unbound,
    # non-finite, bad parameter), all 2000 for the orbit that stays, the
    # removal step for the plunge and the escape.
    assert np.array_equal(got["steps"], exp["steps"])
    assert list(got["steps"][[0, 3, 5]]) == [0, 0, 0] and got["steps"][4] == 2000
    assert np.all((got["steps"][1:3] > 0) & (got["steps"][1:3] < 2000))
    # Zero end time.
    exp0, got0 = _scan_both(pn, y0[4:5], 0.0, 1.0, 0.0, 0.0, 1, nthreads=1)
    assert got0["status"][0] == 0 and abs(got0["fli"][0] - exp0["fli"][0]) < 1e-12
    assert got0["steps"][0] == 0 and exp0["steps"][0] == 0


def test_scan_newton_nonconvergence_flag(pn):
    """Forced non-convergence (one Newton iteration, tolerance 1e-300): the
    GPU sets the NEWTON_NOCONV flag exactly where the oracle does, for the
    six-integral and the dual correction, and keeps the orbits running."""
    from paper_1802_00147_amd import workloads as W
    wl = W.batch(n=24, seed=41, tmin=100.0, tmax=300.0)
    y0 = O.init_state(wl.r0, wl.p0, wl.th1, wl.ph1, wl.th2, wl.ph2, wl.beta, wl.chi1, wl.chi2)
    for mode in (2, 3):
        corr = dict(mode=mode, max_iter=1, tol=1e-300)
        exp, got = _scan_both(pn, y0, wl.t_end, wl.beta, wl.chi1, wl.chi2, wl.n, correction=corr)
        assert np.array_equal(got["status"], exp["status"])
        assert np.all((exp["status"] & 0x100) != 0)
        assert np.array_equal(got["newton_max"], exp["newton_max"])
        assert np.array_equal(got["steps"], exp["steps"])


def test_scan_grid64_full_size(pn):
    """The 64 x 64 (r0, theta) grid at t = 1e5, in the benchmark's launch
    configuration, against the oracle on every grid point
    (tests/golden/oracle_scan_grid64.txt): classes agree on >= 99.5% of the
    points, statuses and step counts exactly where both sides find a regular
    orbit, whose FLIs agree within the per-orbit tolerance of scan_expect."""
    from paper_1802_00147_amd import workloads as W
    import scan_expect as E
    wl = W.grid64()
    y0 = pn.init_state(*[dev(getattr(wl, k)) for k in ("r0", "p0", "th1", "ph1", "th2", "ph2")], 1.0, 1.0, 1.0)
    assert pn.balanced_schedule(wl.n, wl.t_end)["launches"] == 0        # the plain fused scan
    out = pn.fli_scan_balanced(y0, wl.t_end, 1.0, 1.0, 1.0)
    torch.cuda.synchronize()
    got = {k: out[k].cpu().numpy() for k in ("fli", "label", "status", "steps")}
    rep = E.compare("grid64", got)
    assert rep["points"] == wl.n
    # Whole grid: every orbit that runs to the end is corrected to rounding level.
    dH = out["dH"].cpu().numpy()
    ok = got["status"] == 0
    assert ok.sum() >= wl.n - 4 and np.nanmax(dH[ok]) < 1e-13


@pytest.mark.parametrize("beta,qm", [(1.0, 1), (1.0, 0), (0.5, 1), (0.5, 0)])
def test_scan_grid314_full_size_sampled(pn, beta, qm):
    """The 314 x 314 (r0, p-scale) grid at t = 1e6, each of its four variants
    (mass ratio 1 or 1/2, quadrupole-monopole on or off) at full size in the
    benchmark's launch configuration, against the oracle on a seeded sample
    (986 points = 1% for beta = 1 with QM, 200 for each other variant;
    tests/golden/oracle_scan_grid314_*.txt): the gates of scan_expect."""
    from paper_1802_00147_amd import workloads as W
    import scan_expect as E
    wl = W.grid314(beta=beta, quad_mono=qm)
    model = dict(quad_mono=qm)
    y0 = pn.init_state(*[dev(getattr(wl, k)) for k in ("r0", "p0", "th1", "ph1", "th2", "ph2")], beta, 1.0, 1.0,
                       model=model)
    assert pn.balanced_schedule(wl.n, wl.t_end)["launches"] >= 2         # the balanced schedule
    out = pn.fli_scan_balanced(y0, wl.t_end, beta, 1.0, 1.0, model=model, full=False)
    torch.cuda.synchronize()
    got = {k: out[k].cpu().numpy() for k in ("fli", "label", "status", "steps")}
    E.compare(f"grid314_b{beta:g}_qm{qm}", got)
    # Whole grid: labels are -1 exactly where an orbit was removed.
    assert np.array_equal(got["label"] == -1, (got["status"] & 0xFF) != 0)
