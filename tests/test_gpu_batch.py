"""GPU tests of the persistent work-stealing batch scan (orbits of uneven
length and parameters): same results as the plain scan, independence from
the launch shape, exactly-once claiming, longest-first ordering, parity with
the oracle, HIP-graph replay and the autotuner."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import DEV, dev, rel_err_rows

pytestmark = pytest.mark.gpu

FLI_ABS_CORRECTED = 3e-4
KEYS = ("fli", "label", "status", "y_final", "dH", "dJ", "newton_max", "renorms", "steps")


@pytest.fixture(scope="module")
def pn():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1802_00147_amd import pn as P
    P.lib()
    return P


def mixed_batch(n, seed, tmin=50.0, tmax=3000.0):
    from paper_1802_00147_amd import workloads as W
    wl = W.batch(n=n, seed=seed, tmin=tmin, tmax=tmax)
    return wl


def device_inputs(pn, wl):
    cols = [dev(getattr(wl, k)) for k in ("r0", "p0", "th1", "ph1", "th2", "ph2")]
    b, c1, c2 = dev(wl.beta), dev(wl.chi1), dev(wl.chi2)
    y0 = pn.init_state(*cols, b, c1, c2)
    return y0, dev(wl.t_end), b, c1, c2


def host(out):
    return {k: v.cpu().numpy() for k, v in out.items() if isinstance(v, torch.Tensor)}


def test_batch_equals_plain_scan(pn):
    wl = mixed_batch(3001, seed=21)
    y0, t, b, c1, c2 = device_inputs(pn, wl)
    plain = host(pn.fli_scan(y0, t, b, c1, c2))
    batch = host(pn.batch_scan(y0, t, b, c1, c2, tuning=dict(block=256, waves_per_simd=1, chunk_steps=97)))
    torch.cuda.synchronize()
    assert np.array_equal(batch["status"], plain["status"])
    assert np.array_equal(batch["label"], plain["label"])
    assert np.array_equal(batch["renorms"], plain["renorms"])
    assert np.array_equal(batch["steps"], plain["steps"])
    ok = plain["status"] == 0
    assert np.all(np.abs(batch["fli"][ok] - plain["fli"][ok]) <= 1e-12 * np.abs(plain["fli"][ok]) + 1e-12)
    assert np.all(rel_err_rows(batch["y_final"].T[ok], plain["y_final"].T[ok]) <= 1e-13)


def test_batch_bitwise_independent_of_launch_shape(pn):
    wl = mixed_batch(2500, seed=22)
    y0, t, b, c1, c2 = device_inputs(pn, wl)
    runs = []
    for tu in (dict(block=64, waves_per_simd=1, chunk_steps=1), dict(block=256, waves_per_simd=2, chunk_steps=256),
               dict(block=128, waves_per_simd=1, chunk_steps=1000)):
        runs.append(host(pn.batch_scan(y0, t, b, c1, c2, tuning=tu)))
    torch.cuda.synchronize()
    for r in runs[1:]:
        for k in KEYS:
            a, c = runs[0][k], r[k]
            assert np.array_equal(a.view(np.uint8), c.view(np.uint8)), k


def test_every_orbit_claimed_once_in_longest_first_order(pn):
    n = 4097
    wl = mixed_batch(n, seed=23, tmin=10.0, tmax=2000.0)
    y0, t, b, c1, c2 = device_inputs(pn, wl)
    out = pn.scan_outputs(n, n, DEV, full=True)
    out["status"].fill_(0x7FFF0000)
    ws = pn.batch_workspace(n, DEV)
    pn.batch_scan(y0, t, b, c1, c2, out=out, ws=ws, tuning=dict(block=64, waves_per_simd=1, chunk_steps=64))
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert not np.any(st == 0x7FFF0000)          # every orbit's result was written
    # The queue order in the workspace is a permutation, longest first by bins.
    raw = ws.cpu().numpy()
    order = raw[256 + 2048: 256 + 2048 + 4 * n].view(np.int32)
    assert np.array_equal(np.sort(order), np.arange(n))
    steps = np.ceil(wl.t_end[order])
    bins = np.floor(8 * np.log2(steps + 1))
    assert np.all(np.diff(bins) <= 0)


def test_batch_parity_with_oracle(pn):
    wl = mixed_batch(640, seed=24, tmin=100.0, tmax=1500.0)
    y0, t, b, c1, c2 = device_inputs(pn, wl)
    got = host(pn.batch_scan(y0, t, b, c1, c2))
    torch.cuda.synchronize()
    y0o = O.init_state(wl.r0, wl.p0, wl.th1, wl.ph1, wl.th2, wl.ph2, wl.beta, wl.chi1, wl.chi2)
    exp = O.fli_scan(y0o, wl.t_end, wl.beta, wl.chi1, wl.chi2, nthreads=8)
    assert np.array_equal(got["status"], exp["status"])
    assert np.array_equal(got["label"], exp["label"])
    assert np.array_equal(got["steps"], exp["steps"])
    ok = exp["status"] == 0
    assert np.array_equal(got["steps"][ok], np.ceil(wl.t_end[ok]).astype(np.int64))
    assert np.all(rel_err_rows(got["y_final"].T[ok], exp["y_final"][ok]) <= 1e-9)
    # The FLI of short corrected runs has a noise floor of its own: the
    # oracle moves by as much when one initial momentum component changes by
    # one ulp.  The GPU must stay within twice that floor.
    y1 = y0o.copy()
    y1[:, 4] = np.nextafter(y1[:, 4], 1.0)
    exp1 = O.fli_scan(y1, wl.t_end, wl.beta, wl.chi1, wl.chi2, nthreads=8)
    floor = np.abs(exp1["fli"][ok] - exp["fli"][ok]).max()
    diff = np.abs(got["fli"][ok] - exp["fli"][ok]).max()
    assert diff <= 2.0 * floor + 1e-6 and diff <= 1e-3, (diff, floor)


def test_graph_replay_matches_eager(pn):
    wl = mixed_batch(1500, seed=25)
    y0, t, b, c1, c2 = device_inputs(pn, wl)
    eager = host(pn.batch_scan(y0, t, b, c1, c2))
    g = pn.BatchGraph(y0, t, b, c1, c2)
    try:
        for rep in range(3):
            # Eager work of the program between replays.
            pn.rhs(y0, b, c1, c2)
            torch.cuda.synchronize()
            g.out["status"].fill_(-7)
            got = host(g.replay())
            torch.cuda.synchronize()
            for k in KEYS:
                assert np.array_equal(got[k].view(np.uint8), eager[k].view(np.uint8)), (rep, k)
    finally:
        g.close()


def test_autotune_and_cached_tuning(pn):
    wl = mixed_batch(5000, seed=26, tmin=100.0, tmax=5000.0)
    y0, t, b, c1, c2 = device_inputs(pn, wl)
    best, ms = pn.autotune_batch(y0, t, b, c1, c2, step_scale=0.05)
    assert best["block"] in (64, 128, 256) and best["waves_per_simd"] in (1, 2)
    assert best["chunk_steps"] in (32, 64, 256, 1024) and ms > 0
    a = host(pn.batch_scan(y0, t, b, c1, c2))                  # uses the cached result
    c = host(pn.batch_scan(y0, t, b, c1, c2, tuning=dict(block=64, waves_per_simd=1, chunk_steps=7)))
    torch.cuda.synchronize()
    for k in KEYS:
        assert np.array_equal(a[k].view(np.uint8), c[k].view(np.uint8)), k


def _run_resumable(pn, y0, t, b, c1, c2, n, tunings, max_chunks, through_host):
    """Resumable scan to the end; returns (outputs, pending after each launch)."""
    ws = pn.batch_ckpt_workspace(n, y0.device)
    ws.fill_(0x5A)
    out = pn.scan_outputs(n, n, y0.device, full=True)
    for v in out.values():
        v.fill_(-3)
    pn.batch_scan_resumable(y0, t, b, c1, c2, ws, resume=False, max_chunks=max_chunks, out=out, tuning=tunings[0])
    pending = [pn.batch_scan_pending(ws, n)]
    while pending[-1] > 0:
        assert len(pending) < 400, pending[-8:]
        if through_host:
            # Checkpoint to host memory, wipe the device copies, restore.
            ws_h = ws.cpu()
            out_h = {k: v.cpu() for k, v in out.items()}
            ws.fill_(0xC3)
            for v in out.values():
                v.fill_(-5)
            ws.copy_(ws_h)
            for k, v in out.items():
                v.copy_(out_h[k])
        pn.batch_scan_resumable(y0, t, b, c1, c2, ws, resume=True, max_chunks=max_chunks, out=out,
                                tuning=tunings[len(pending) % len(tunings)])
        pending.append(pn.batch_scan_pending(ws, n))
    torch.cuda.synchronize()
    return host(out), pending


def test_resumable_scan_equals_uninterrupted(pn):
    """Checkpoint and resume: the batch interrupted every 3 chunks, its
    workspace and outputs copied to host memory and back between launches
    (the device copies overwritten meanwhile), resumed under changing launch
    shapes, gives the uninterrupted scan's results bit for bit."""
    wl = mixed_batch(3001, seed=31, tmin=50.0, tmax=3000.0)
    y0, t, b, c1, c2 = device_inputs(pn, wl)
    ref = host(pn.batch_scan(y0, t, b, c1, c2, tuning=dict(block=256, waves_per_simd=2, chunk_steps=64)))
    tunings = [dict(block=64, waves_per_simd=1, chunk_steps=64), dict(block=256, waves_per_simd=2, chunk_steps=100),
               dict(block=128, waves_per_simd=1, chunk_steps=37)]
    got, pending = _run_resumable(pn, y0, t, b, c1, c2, wl.n, tunings, 3, through_host=True)
    assert len(pending) > 5 and pending[0] > 0
    assert all(x >= y for x, y in zip(pending, pending[1:]))     # never loses an orbit
    for k in KEYS:
        assert np.array_equal(got[k].view(np.uint8), ref[k].view(np.uint8)), k
    # Run to the end in one launch (max_chunks = 0): same bits again.
    got0, pending0 = _run_resumable(pn, y0, t, b, c1, c2, wl.n, tunings[1:2], 0, through_host=False)
    assert pending0 == [0]
    for k in KEYS:
        assert np.array_equal(got0[k].view(np.uint8), ref[k].view(np.uint8)), k


def test_resumable_scan_carries_orbits_a_smaller_grid_cannot_take(pn):
    """40,000 orbits all in flight after a two-wave launch (more than the
    one-wave grid's resident pairs on this chip) resume on one-wave grids:
    the records no slot takes are carried to the next launch; results equal
    the uninterrupted scan bit for bit."""
    wl = mixed_batch(40000, seed=32, tmin=20.0, tmax=400.0)
    y0, t, b, c1, c2 = device_inputs(pn, wl)
    ref = host(pn.batch_scan(y0, t, b, c1, c2))
    slots1 = torch.cuda.get_device_properties(y0.device).multi_processor_count * 4 * 32
    tunings = [dict(block=256, waves_per_simd=2, chunk_steps=16), dict(block=256, waves_per_simd=1, chunk_steps=16)]
    got, pending = _run_resumable(pn, y0, t, b, c1, c2, wl.n, tunings, 1, through_host=False)
    if wl.n > slots1:
        assert pending[0] > slots1          # the second launch cannot take every saved orbit
    assert all(x >= y for x, y in zip(pending, pending[1:]))
    for k in KEYS:
        assert np.array_equal(got[k].view(np.uint8), ref[k].view(np.uint8)), k


def test_batch_errors_and_empty(pn):
    wl = mixed_batch(10, seed=27)
    y0, t, b, c1, c2 = device_inputs(pn, wl)
    small = torch.empty(8, dtype=torch.uint8, device=DEV)
    with pytest.raises(pn.PnError) as e:
        pn.batch_scan(y0, t, b, c1, c2, ws=small)
    assert e.value.status == pn.PN_ENOWS
    with pytest.raises(pn.PnError) as e:
        pn.batch_scan(y0, t, b, c1, c2, tuning=dict(block=96))
    assert e.value.status == pn.PN_EINVAL
    pn.batch_scan(y0, t, b, c1, c2, n=0)


def test_batch1m_full_size_sampled(pn):
    """The 10^6-orbit uneven batch (t_end log-uniform in [1e3, 1e6], per-orbit
    beta and spins) in one persistent launch, against the oracle on 1,000
    seeded orbits (tests/golden/oracle_scan_batch1M.txt): the gates of
    scan_expect (classes agree on >= 99.5%, regular FLIs within the
    per-orbit tolerance, statuses and step counts exact for them)."""
    from paper_1802_00147_amd import workloads as W
    import scan_expect as E
    wl = W.batch()
    y0, t, b, c1, c2 = device_inputs(pn, wl)
    out = pn.batch_scan(y0, t, b, c1, c2, full=False)
    torch.cuda.synchronize()
    got = {k: out[k].cpu().numpy() for k in ("fli", "label", "status", "steps")}
    assert np.all((got["label"] == -1) == ((got["status"] & 0xFF) != 0))
    E.compare("batch1M", got)
