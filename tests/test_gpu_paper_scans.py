"""The paper's own spin-angle scans (Sec. 3C, Figs. 6-7) on the GPU against
the oracle, through the C ABI.

Fig. 6 lines (314 orbits each), oracle run live: statuses (which states are
unbound, which merge or escape) must agree exactly; labels must agree
wherever the oracle's FLI is more than 0.25 from the threshold, and on
>= 99.5% of the points overall; FLIs of regular orbits agree to 3e-4 (the
oracle's own 1-ulp sensitivity on these lines is <= 1e-5).

Fig. 7 plane (314 x 314 at full size), judged on a seeded 1% sample by the
stored oracle expectations and the gates of scan_expect.
"""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import dev
from paper_1802_00147_amd import workloads as W

pytestmark = pytest.mark.gpu

FLI_ABS_REGULAR = 3e-4
NEAR = 0.25


@pytest.fixture(scope="module")
def pn():
    assert torch.cuda.is_available(), "GPU parity tests need a ROCm device"
    from paper_1802_00147_amd import pn as P
    P.lib()
    return P


def gpu_scan(pn, wl, model):
    """The scan as the benchmark runs it: pn_fli_scan_balanced with the
    device's schedule (the plain fused scan for the 314-orbit lines, the
    balanced schedule for the 314 x 314 plane)."""
    y0 = pn.init_state(*[dev(getattr(wl, k)) for k in ("r0", "p0", "th1", "ph1", "th2", "ph2")],
                       wl.beta, wl.chi1, wl.chi2, model=model)
    launches = pn.balanced_schedule(wl.n, wl.t_end)["launches"]
    assert (launches >= 2) == (wl.n > 65536 // 2)
    out = pn.fli_scan_balanced(y0, wl.t_end, wl.beta, wl.chi1, wl.chi2, model=model, full=False)
    torch.cuda.synchronize()
    return {k: out[k].cpu().numpy()[:wl.n] for k in ("fli", "label", "status")}


def oracle_scan(wl, model):
    y0 = O.init_state(wl.r0, wl.p0, wl.th1, wl.ph1, wl.th2, wl.ph2, wl.beta, wl.chi1, wl.chi2, model=model)
    return O.fli_scan(y0, wl.t_end, wl.beta, wl.chi1, wl.chi2, model=model, nthreads=16)


def compare(got, exp, thr=5.8):
    assert np.array_equal(got["status"], exp["status"])
    valid = exp["status"] == 0
    far = valid & (np.abs(exp["fli"] - thr) > NEAR)
    assert np.array_equal(got["label"][far], exp["label"][far])
    assert np.array_equal(got["label"][~valid], exp["label"][~valid])
    mismatch = int(np.sum(got["label"] != exp["label"]))
    assert mismatch <= 0.005 * len(exp["label"]), mismatch
    reg = valid & (exp["label"] == 0) & (got["label"] == 0)
    if reg.any():
        assert np.abs(got["fli"][reg] - exp["fli"][reg]).max() <= FLI_ABS_REGULAR
    return mismatch


@pytest.mark.parametrize("units", [0, 1], ids=["phys", "paper_eq8"])
@pytest.mark.parametrize("theta1", [np.pi / 2, 0.0], ids=["fig6a", "fig6b"])
def test_fig6_line_parity(pn, theta1, units):
    """All 314 orbits of the line at t = 1e5; the unbound part is removed."""
    wl = W.fig6(theta1)
    model = dict(spin_units=units)
    got = gpu_scan(pn, wl, model)
    exp = oracle_scan(wl, model)
    compare(got, exp)
    assert np.sum(exp["status"] == O.STATUS_OK) >= 50


@pytest.mark.parametrize("units", [0, 1], ids=["phys", "paper_eq8"])
def test_fig7_plane_full_size_sampled(pn, units):
    """The 314 x 314 plane at t = 1e5 in the benchmark's launch configuration,
    against the oracle on a seeded 1% sample (986 points;
    tests/golden/oracle_scan_fig7_*.txt): the gates of scan_expect."""
    import scan_expect as E
    wl = W.fig7()
    model = dict(spin_units=units)
    y0 = pn.init_state(*[dev(getattr(wl, k)) for k in ("r0", "p0", "th1", "ph1", "th2", "ph2")],
                       wl.beta, wl.chi1, wl.chi2, model=model)
    out = pn.fli_scan_balanced(y0, wl.t_end, wl.beta, wl.chi1, wl.chi2, model=model, full=False)
    torch.cuda.synchronize()
    got = {k: out[k].cpu().numpy() for k in ("fli", "label", "status", "steps")}
    E.compare("fig7_phys" if units == 0 else "fig7_eq8", got)
    # Whole plane: every state is bound (H < 0 for the printed state), so
    # only merging or escaping can remove an orbit.
    assert not np.any(got["status"] == O.STATUS_UNBOUND_INIT)
