"""Judging a full-size GPU scan by the oracle's stored expectations
(tests/golden/oracle_scan_<name>.txt, written by
tests/golden/make_oracle_scans.py, which runs the oracle alone).

Classes for label agreement:
  0  regular (label 0, the orbit ran to its end time);
  1  chaotic (label 1), or removed during the run (merged, escaped,
     non-finite after at least one step);
  2  removed at t = 0 (unbound initial state, parameters out of range).
A chaotic orbit's separation from any nearby trajectory grows exponentially
from rounding, so whether it comes within r < 2 before its end time is not
reproducible between two correct integrations: the oracle's own runs from
initial states one ulp apart disagree on it for 1% of the Fig. 7 plane.
Such an orbit is chaotic either way, so class 1 combines the two outcomes.
Class 2 is decided from the initial state alone and must match exactly.

FLI tolerance of an orbit regular on both sides: the larger of 1e-6
relative (the stated parity bound for regular orbits) and 10 times the
oracle's own rounding sensitivity there, the largest FLI change of its four
1-ulp runs, floored at the configuration's median sensitivity (an orbit's
runs can all land close by chance).  The GPU contracts a*b+c into FMAs
and refines hardware reciprocals where the oracle rounds every IEEE
operation, so its FLI is another draw of the same rounding noise.
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_oracle_scans as M  # noqa: E402

LABEL_AGREEMENT_MIN = 0.995
FLI_REL = 1e-6
SENS_FACTOR = 10.0


def classes(status, label, steps):
    removed = (np.asarray(status) & 0xFF) != 0
    c = np.where(np.asarray(label) == 1, 1, 0)
    c = np.where(removed, np.where(np.asarray(steps) == 0, 2, 1), c)
    return c


def sensitivity(exp):
    """The oracle's own FLI spread at each orbit: the largest change among its
    four runs from initial states one ulp away."""
    return np.max([np.abs(exp[k] - exp["fli"]) for k in M.TWINS], axis=0)


def compare(name, got):
    """got: the GPU scan's outputs over the whole workload (numpy arrays
    fli, label, status, steps).  Asserts the gates; returns a report.  With
    PN_PARITY_DUMP set to a directory, the sampled outputs are also saved
    there (parity_<name>.npz) for inspection."""
    exp = M.load(name)
    idx = exp["index"]
    g = {k: np.asarray(got[k])[idx] for k in ("fli", "label", "status", "steps")}
    dump = os.environ.get("PN_PARITY_DUMP")
    if dump:
        os.makedirs(dump, exist_ok=True)
        np.savez(os.path.join(dump, f"parity_{name}.npz"), index=idx, **g)
    ce = classes(exp["status"], exp["label"], exp["steps"])
    cg = classes(g["status"], g["label"], g["steps"])
    agree = float(np.mean(ce == cg))
    strict = float(np.mean((g["status"] == exp["status"]) & (g["label"] == exp["label"])))
    both = (ce == 0) & (cg == 0)
    sens = sensitivity(exp)
    floor = float(np.median(sens[ce == 0])) if np.any(ce == 0) else 0.0
    tol = np.maximum(FLI_REL * np.abs(exp["fli"]), SENS_FACTOR * np.maximum(sens, floor))
    err = np.abs(g["fli"] - exp["fli"])
    worst = float(np.max(err[both] / tol[both])) if both.any() else 0.0
    rel = err[both] / np.abs(exp["fli"][both])
    report = dict(config=name, points=len(idx), regular_both=int(both.sum()), class_agreement=agree,
                  strict_agreement=strict, fli_within_rel_1e6=float(np.mean(rel <= FLI_REL)) if both.any() else 1.0,
                  median_abs_fli_diff=float(np.median(err[both])) if both.any() else 0.0,
                  median_oracle_sensitivity=floor, max_abs_fli_diff=float(err[both].max()) if both.any() else 0.0,
                  max_oracle_sensitivity=float(sens[ce == 0].max()) if np.any(ce == 0) else 0.0,
                  worst_over_tolerance=worst)
    print("scan parity", report, flush=True)
    # Removed at t = 0: decided by the initial state, exactly.
    start = (ce == 2) | (cg == 2)
    assert np.array_equal(g["status"][start], exp["status"][start]), name
    assert agree >= LABEL_AGREEMENT_MIN, (name, agree, np.flatnonzero(ce != cg)[:20])
    assert np.array_equal(g["status"][both], exp["status"][both]), name
    assert np.array_equal(g["steps"][both], exp["steps"][both]), name
    assert worst <= 1.0, (name, worst, idx[both][np.argmax(err[both] / tol[both])])
    return report
