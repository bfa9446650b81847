"""The stored oracle expectations of the full-size scans
(tests/golden/oracle_scan_*.txt) are current: their samples are the seeded
ones, and rows recomputed now by the oracle equal the stored rows bit for
bit.  The comparison rules of scan_expect pass the oracle's own rows and
reject planted disagreements."""
import numpy as np
import pytest

import scan_expect as E

M = E.M


@pytest.mark.parametrize("name", list(M.CONFIGS))
def test_expectations_are_current(name):
    exp = M.load(name)
    wl, idx = M.sample(name)
    assert np.array_equal(exp["index"], idx)
    # Recompute the two rows with the fewest steps (the cheapest to rerun).
    pick = np.argsort(exp["steps"] + (exp["steps"] == 0) * 10**9, kind="stable")[:2]
    rows = M.oracle_rows(name, idx_subset=exp["index"][pick], nthreads=2)
    for k in ("status", "label", "steps"):
        assert np.array_equal(rows[k], exp[k][pick]), k
    for k in ("fli",) + M.TWINS:
        np.testing.assert_array_equal(rows[k], exp[k][pick], err_msg=k)    # NaN equals NaN


def _full(name):
    """The expectations spread over a whole-workload output array."""
    exp = M.load(name)
    wl, _ = M.sample(name)
    got = {k: np.zeros(wl.n, dtype=exp[k].dtype) for k in ("fli", "label", "status", "steps")}
    for k in got:
        got[k][exp["index"]] = exp[k]
    return exp, got


def test_compare_accepts_the_oracle_and_rejects_planted_disagreements():
    exp, got = _full("fig7_phys")
    rep = E.compare("fig7_phys", got)
    assert rep["class_agreement"] == 1.0 and rep["worst_over_tolerance"] == 0.0
    # A 1-ulp twin of the oracle passes: its FLIs are inside the tolerance.
    twin = {k: v.copy() for k, v in got.items()}
    ok = (exp["status"] == 0) & (exp["label"] == 0)
    twin["fli"][exp["index"][ok]] = exp["fli_r"][ok]
    E.compare("fig7_phys", twin)
    # Labels flipped on 1% of the points: rejected.
    bad = {k: v.copy() for k, v in got.items()}
    flip = exp["index"][ok][:10]
    bad["label"][flip] = 1
    with pytest.raises(AssertionError):
        E.compare("fig7_phys", bad)
    # A regular FLI off by 1e-4 relative: rejected.
    bad = {k: v.copy() for k, v in got.items()}
    i = exp["index"][ok][0]
    bad["fli"][i] *= 1.0 + 1e-4
    with pytest.raises(AssertionError):
        E.compare("fig7_phys", bad)
    # A state removed at t = 0 on one side only: rejected.
    bad = {k: v.copy() for k, v in got.items()}
    bad["status"][i], bad["steps"][i], bad["label"][i] = 4, 0, -1
    with pytest.raises(AssertionError):
        E.compare("fig7_phys", bad)


def test_classes():
    st = np.array([0, 0, 1, 4, 2, 0x100])
    lab = np.array([0, 1, -1, -1, -1, 1])
    steps = np.array([10, 10, 5, 0, 3, 10])
    assert list(E.classes(st, lab, steps)) == [0, 1, 1, 2, 1, 1]
