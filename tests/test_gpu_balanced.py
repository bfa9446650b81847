"""GPU tests of the balanced scan (pn_fli_scan_balanced, McNaughton's
wrap-around schedule of orbits of equal length): the plain fused scan's
outputs bit for bit for any slot count and launch split, bitwise independence
from the schedule, parity with the oracle, the schedule choice at full scan
size, and the workspace contract."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import DEV, dev, rel_err_rows, to_soa

pytestmark = pytest.mark.gpu

KEYS = ("fli", "label", "status", "y_final", "dH", "dJ", "newton_max", "renorms", "steps")


@pytest.fixture(scope="module")
def pn():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1802_00147_amd import pn as P
    P.lib()
    return P


def host(out):
    return {k: v.cpu().numpy() for k, v in out.items() if isinstance(v, torch.Tensor)}


def mixed_inputs(pn, n, seed):
    """Uneven parameters and radii, one end time for all; every 50th orbit
    starts unbound, every 70th plunges (r0 in [5, 12] with 0.3 of the circular
    momentum) and merges at a different time, every 90th has beta = 1.5."""
    from paper_1802_00147_amd import workloads as W
    wl = W.batch(n=n, seed=seed, tmin=50.0, tmax=100.0)
    r0, p0, beta = wl.r0.copy(), wl.p0.copy(), wl.beta.copy()
    p0[::50] *= 1.6
    k = r0[7::70].size
    r0[7::70] = np.linspace(5.0, 12.0, k)
    p0[7::70] = 0.3 * r0[7::70] ** -0.5
    beta[11::90] = 1.5
    cols = [dev(v) for v in (r0, p0, wl.th1, wl.ph1, wl.th2, wl.ph2)]
    b, c1, c2 = dev(beta), dev(wl.chi1), dev(wl.chi2)
    return pn.init_state(*cols, b, c1, c2), b, c1, c2


def assert_same_as_plain(got, plain):
    """Every output bit for bit: both kernels run the same step, correction
    and FLI code on each orbit, and a saved pair state is restored exactly."""
    for k in KEYS:
        assert np.array_equal(got[k].view(np.uint8), plain[k].view(np.uint8)), k


@pytest.mark.parametrize("slots", [1, 7, 64, 1000, 5000])
def test_balanced_equals_plain_scan(pn, slots):
    """3,001 orbits to t = 700 on 1 to 5,000 slots (more slots than orbits
    leaves the last ones empty): the plain scan's outputs bit for bit."""
    y0, b, c1, c2 = mixed_inputs(pn, 3001, seed=31)
    plain = host(pn.fli_scan(y0, 700.0, b, c1, c2))
    sch = pn.balanced_schedule(3001, 700.0, slots=slots)
    assert sch["slots"] == slots and sch["launches"] >= 2
    got = host(pn.fli_scan_balanced(y0, 700.0, b, c1, c2, slots=slots))
    torch.cuda.synchronize()
    st = plain["status"] & 0xFF
    assert {0, 1, 4, 5} <= set(st.tolist())          # running, merged, unbound, bad parameter
    assert_same_as_plain(got, plain)


def test_balanced_bitwise_independent_of_schedule(pn):
    """Every output, the FLI trace included, is the same bit for bit on 3, 17,
    256 and 4,096 slots (different cuts, carries and launch counts)."""
    y0, b, c1, c2 = mixed_inputs(pn, 2500, seed=32)
    runs = []
    for slots in (3, 17, 256, 4096):
        runs.append(host(pn.fli_scan_balanced(y0, 900.0, b, c1, c2, slots=slots, trace_every=100)))
    torch.cuda.synchronize()
    for r in runs[1:]:
        for k in KEYS + ("trace",):
            assert np.array_equal(runs[0][k].view(np.uint8), r[k].view(np.uint8)), k


def test_balanced_matches_oracle(pn):
    """60 orbits of the grid64 configuration (r0 in [10, 40], theta in [0, pi])
    to t = 1,000 on 7 slots (so most orbits are split or cut by the launch
    boundary) against the oracle, to the bars of the plain scan's parity
    tests: statuses, labels and step counts exact, final states within 1e-10
    relative, FLIs within 3e-4 (a corrected run: each trajectory carries the
    rounding of its projection, which differs between the two sides)."""
    r0 = np.repeat(np.linspace(10.0, 40.0, 6), 10)
    th = np.tile(np.linspace(0.0, np.pi, 10), 6)
    z = np.zeros_like(r0)
    y0 = O.init_state(r0, r0 ** -0.5, np.full_like(r0, np.pi / 2), z, th, z, 1.0, 1.0, 1.0)
    ref = O.fli_scan(y0, 1000.0, 1.0, 1.0, 1.0)
    yd = to_soa(y0)
    got = host(pn.fli_scan_balanced(yd, 1000.0, 1.0, 1.0, 1.0, slots=7))
    torch.cuda.synchronize()
    assert np.array_equal(got["status"], ref["status"])
    assert np.array_equal(got["label"], ref["label"])
    assert np.array_equal(got["steps"], ref["steps"])
    ok = ref["status"] == 0
    assert ok.all()
    assert np.all(np.abs(got["fli"] - ref["fli"]) <= 3e-4)
    assert np.all(rel_err_rows(got["y_final"].T, ref["y_final"]) <= 1e-10)


def test_balanced_rk5_dual(pn):
    """The RK5 + dual-scaling kernel on 13 slots: the plain scan's outputs bit
    for bit."""
    y0, b, c1, c2 = mixed_inputs(pn, 700, seed=33)
    integ, corr = dict(method=1), dict(mode=3)
    plain = host(pn.fli_scan(y0, 400.0, b, c1, c2, integrator=integ, correction=corr))
    got = host(pn.fli_scan_balanced(y0, 400.0, b, c1, c2, integrator=integ, correction=corr, slots=13))
    torch.cuda.synchronize()
    assert_same_as_plain(got, plain)


def test_full_grid_takes_the_balanced_schedule(pn):
    """The paper's 314 x 314 spin-angle plane (98,596 orbits) to t = 3,000 on
    the device's resident slots: the schedule chosen is the balanced one, and
    it gives the plain scan's results; a 4,096-orbit grid keeps the plain
    scan."""
    from paper_1802_00147_amd import workloads as W
    wl = W.fig7(t_end=3000.0)
    cols = [dev(getattr(wl, k)) for k in ("r0", "p0", "th1", "ph1", "th2", "ph2")]
    y0 = pn.init_state(*cols, wl.beta, wl.chi1, wl.chi2, model=wl.model)
    sch = pn.balanced_schedule(wl.n, 3000.0)
    assert sch["launches"] >= 2 and sch["slots"] >= 32768
    plain = host(pn.fli_scan(y0, 3000.0, wl.beta, wl.chi1, wl.chi2, model=wl.model))
    got = host(pn.fli_scan_balanced(y0, 3000.0, wl.beta, wl.chi1, wl.chi2, model=wl.model))
    torch.cuda.synchronize()
    assert_same_as_plain(got, plain)
    assert pn.balanced_schedule(4096, 1e5)["launches"] == 0


def test_balanced_workspace_contract(pn):
    y0, b, c1, c2 = mixed_inputs(pn, 100, seed=34)
    sch = pn.balanced_schedule(100, 300.0, slots=9)
    short = torch.empty(int(pn.lib().pn_fli_scan_balanced_workspace_size(9)) - 1, dtype=torch.uint8, device=DEV)
    with pytest.raises(pn.PnError):
        pn.fli_scan_balanced(y0, 300.0, b, c1, c2, slots=9, ws=short)
    assert sch["launches"] >= 2
    # A reused workspace holding another scan's records gives the same results.
    ws = pn.balanced_workspace(9, DEV)
    first = host(pn.fli_scan_balanced(y0, 300.0, b, c1, c2, slots=9, ws=ws))
    y1, *_ = mixed_inputs(pn, 100, seed=35)
    pn.fli_scan_balanced(y1, 300.0, b, c1, c2, slots=9, ws=ws)
    again = host(pn.fli_scan_balanced(y0, 300.0, b, c1, c2, slots=9, ws=ws))
    torch.cuda.synchronize()
    for k in KEYS:
        assert np.array_equal(first[k].view(np.uint8), again[k].view(np.uint8)), k
    # Errors: negative slots, per-orbit end times are not taken (uneven orbits
    # belong to the batch scan).
    with pytest.raises(pn.PnError):
        pn.fli_scan_balanced(y0, 300.0, b, c1, c2, slots=-1)


@pytest.mark.parametrize("method", [0, 1], ids=["rk4", "rk5"])
@pytest.mark.parametrize("mode", [0, 1, 2, 3], ids=["none", "spin", "six", "dual"])
def test_balanced_every_kernel_build(pn, method, mode):
    """Each of the eight builds (integrator x correction) on 11 slots gives
    the plain scan's outputs bit for bit, and the runtime reports its
    resources (at least one resident wavefront per SIMD)."""
    y0, b, c1, c2 = mixed_inputs(pn, 400, seed=40 + 4 * method + mode)
    integ, corr = dict(method=method), dict(mode=mode)
    plain = host(pn.fli_scan(y0, 250.0, b, c1, c2, integrator=integ, correction=corr))
    got = host(pn.fli_scan_balanced(y0, 250.0, b, c1, c2, integrator=integ, correction=corr, slots=11))
    torch.cuda.synchronize()
    assert_same_as_plain(got, plain)
    res = pn.balanced_kernel_resources(integ, corr)
    assert res["waves_per_simd"] >= 1 and 0 < res["vgprs"] <= 512
