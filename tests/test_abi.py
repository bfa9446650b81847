"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/pn.h declares, fills its defaults, and rejects invalid arguments on the
host before anything is launched (PN_EINVAL), as the header documents."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pn.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(pn_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def pn():
    from paper_1802_00147_amd import pn as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1802_00147_amd import build
        build.build()
    P.lib()
    return P


def test_library_exports_every_declared_symbol(pn):
    names = declared_functions()
    assert len(names) >= 13
    L = pn.lib()
    for name in names:
        assert hasattr(L, name), name
    assert sorted(names) == sorted(pn.EXPORTS)


def test_defaults_match_paper_settings(pn):
    m, i, c, f = pn.model_struct(), pn.integrator_struct(), pn.correction_struct(), pn.fli_struct()
    assert (m.pn_order, m.spin_orbit, m.spin_spin, m.quad_mono, m.spin_units) == (2, 1, 1, 1, 0)
    assert (i.method, i.h) == (0, 1.0)
    assert (c.mode, c.tol, c.max_iter, c.sweeps) == (2, 1e-10, 20, 2)
    assert (f.d0, f.d_renorm, f.thr_at_1e5, f.thr_scaling, f.r_merge, f.r_esc) == (1e-8, 0.1, 5.8, 1, 2.0, 1e3)
    assert pn.lib().pn_version() == 1
    assert pn.lib().pn_status_string(1) == b"invalid argument"


def _call_rhs(pn, model=None, beta=1.0, chi=1.0, n=4, ld=4, y=1, f=1):
    m = pn.model_struct(model)
    p = pn.Params(None, None, None, beta, chi, chi)
    return pn.lib().pn_rhs(ctypes.byref(m), p, ctypes.c_int64(n),
                           ctypes.c_void_p(y) if y else None, ctypes.c_int64(ld),
                           ctypes.c_void_p(f) if f else None, None)


def test_invalid_arguments_rejected_before_launch(pn):
    # Fake non-null "device" pointers are never dereferenced: validation fails first.
    assert _call_rhs(pn, beta=0.0) == pn.PN_EINVAL
    assert _call_rhs(pn, beta=1.5) == pn.PN_EINVAL
    assert _call_rhs(pn, chi=-0.1) == pn.PN_EINVAL
    assert _call_rhs(pn, chi=float("nan")) == pn.PN_EINVAL
    assert _call_rhs(pn, model=dict(pn_order=3)) == pn.PN_EINVAL
    assert _call_rhs(pn, model=dict(spin_units=7)) == pn.PN_EINVAL
    assert _call_rhs(pn, n=-1) == pn.PN_EINVAL
    assert _call_rhs(pn, n=8, ld=4) == pn.PN_EINVAL
    assert _call_rhs(pn, y=0) == pn.PN_EINVAL
    assert _call_rhs(pn, f=0) == pn.PN_EINVAL
    # n = 0 is a valid no-op.
    assert _call_rhs(pn, n=0, ld=0, y=0, f=0) == pn.PN_OK
    # A null model pointer.
    p = pn.Params(None, None, None, 1.0, 1.0, 1.0)
    assert pn.lib().pn_rhs(None, p, ctypes.c_int64(1), ctypes.c_void_p(1), ctypes.c_int64(1),
                           ctypes.c_void_p(1), None) == pn.PN_EINVAL
    # Per-orbit arrays must be all present or all absent.
    p = pn.Params(1, None, None, 0.0, 0.0, 0.0)
    assert pn.lib().pn_rhs(ctypes.byref(pn.model_struct()), p, ctypes.c_int64(1), ctypes.c_void_p(1),
                           ctypes.c_int64(1), ctypes.c_void_p(1), None) == pn.PN_EINVAL


def test_invalid_scan_settings_rejected(pn):
    L = pn.lib()
    m = pn.model_struct()
    p = pn.Params(None, None, None, 1.0, 1.0, 1.0)
    one = ctypes.c_void_p(8)
    so = pn.ScanOut(8, 8, 8, None, None, None, None, None, None, 0, 0)

    def scan(integ=None, corr=None, fli=None, t_all=1.0, out=so):
        return L.pn_fli_scan(ctypes.byref(m), p, ctypes.byref(pn.integrator_struct(integ)),
                             ctypes.byref(pn.correction_struct(corr)), ctypes.byref(pn.fli_struct(fli)),
                             ctypes.c_int64(4), one, ctypes.c_int64(4), None, ctypes.c_double(t_all),
                             ctypes.byref(out), None)

    assert scan(integ=dict(h=0.0)) == pn.PN_EINVAL
    assert scan(integ=dict(h=-1.0)) == pn.PN_EINVAL
    assert scan(integ=dict(method=9)) == pn.PN_EINVAL
    assert scan(corr=dict(mode=7)) == pn.PN_EINVAL
    assert scan(corr=dict(max_iter=0)) == pn.PN_EINVAL
    assert scan(corr=dict(sweeps=0)) == pn.PN_EINVAL
    assert scan(corr=dict(tol=float("nan"))) == pn.PN_EINVAL
    assert scan(fli=dict(d0=0.0)) == pn.PN_EINVAL
    assert scan(fli=dict(d_renorm=1e-9)) == pn.PN_EINVAL
    assert scan(fli=dict(shadow_axis=12)) == pn.PN_EINVAL
    assert scan(fli=dict(r_esc=1.0)) == pn.PN_EINVAL
    assert scan(t_all=-1.0) == pn.PN_EINVAL
    assert scan(t_all=float("inf")) == pn.PN_EINVAL
    bad_out = pn.ScanOut(8, None, 8, None, None, None, None, None, None, 0, 0)
    assert scan(out=bad_out) == pn.PN_EINVAL
    bad_trace = pn.ScanOut(8, 8, 8, None, None, None, None, None, None, 10, 5)
    assert scan(out=bad_trace) == pn.PN_EINVAL


def test_invalid_trajectory_and_gw_arguments_rejected(pn):
    L = pn.lib()
    m = ctypes.byref(pn.model_struct())
    p = pn.Params(None, None, None, 1.0, 1.0, 1.0)
    one = ctypes.c_void_p(8)

    def traj(every=1, traj_ptr=one, nsteps=4):
        return L.pn_trajectory(m, p, ctypes.byref(pn.integrator_struct()), None, ctypes.c_int64(4), one,
                               ctypes.c_int64(4), None, ctypes.c_int64(nsteps), ctypes.c_int64(every),
                               traj_ptr, None)

    assert traj(every=0) == pn.PN_EINVAL
    assert traj(every=-3) == pn.PN_EINVAL
    assert traj(traj_ptr=None) == pn.PN_EINVAL          # rows = 4 need a buffer

    def gw(nhat=(0, 0, 1), phat=(1, 0, 0), dist=10.0, n=4, ns=2, ld=4):
        N3 = (ctypes.c_double * 3)(*nhat)
        P3 = (ctypes.c_double * 3)(*phat)
        return L.pn_gw_polarizations(m, p, ctypes.c_int64(n), ctypes.c_int64(ns), one, ctypes.c_int64(ld),
                                     N3, P3, ctypes.c_double(dist), one, one, None)

    assert gw(nhat=(0, 0, 2)) == pn.PN_EINVAL             # not unit
    assert gw(phat=(1, 0, 0.01)) == pn.PN_EINVAL          # not unit, not transverse
    assert gw(phat=(0, 0, 1)) == pn.PN_EINVAL             # along the line of sight
    assert gw(dist=0.0) == pn.PN_EINVAL
    assert gw(dist=float("inf")) == pn.PN_EINVAL
    assert gw(n=8, ld=4) == pn.PN_EINVAL
    assert gw(ns=-1) == pn.PN_EINVAL
    assert gw(n=0, ld=0) == pn.PN_OK                      # nothing to do
    assert gw(ns=0) == pn.PN_OK


def test_invalid_surrogate_scan_arguments_rejected(pn):
    L = pn.lib()
    one = ctypes.c_void_p(8)
    mean = (ctypes.c_float * 7)(*([0.0] * 7))
    std = (ctypes.c_float * 7)(*([1.0] * 7))
    bad_std = (ctypes.c_float * 7)(*([1.0] * 6 + [0.0]))
    net = pn.Mlp(*[pn.P4(*([8] * 4)) for _ in range(7)])
    step = ctypes.c_int32(0)
    integrated = ctypes.c_int64(-1)

    def scan(cfg=None, n=4, t_all=1.0, std_=std, model=None, corr=None, ws=one, ws_bytes=1 << 40):
        c = pn.surrogate_cfg(cfg)
        return L.pn_surrogate_scan(ctypes.byref(net), ctypes.byref(step), ctypes.byref(pn.model_struct(model)),
                                   pn.Params(None, None, None, 1.0, 1.0, 1.0), ctypes.byref(pn.integrator_struct()),
                                   ctypes.byref(pn.correction_struct(corr)), ctypes.byref(pn.fli_struct()),
                                   ctypes.c_int64(n), one, one, one, one, one, one, None, ctypes.c_double(t_all),
                                   mean, std_, ctypes.byref(c), one, None, ctypes.byref(integrated), None, ws,
                                   ctypes.c_size_t(ws_bytes), None)

    assert scan(cfg=dict(margin=-1.0)) == pn.PN_EINVAL
    assert scan(cfg=dict(audit_frac=1.5)) == pn.PN_EINVAL
    assert scan(cfg=dict(refine_batch=0)) == pn.PN_EINVAL
    assert scan(cfg=dict(refine_lr=0.0)) == pn.PN_EINVAL
    assert scan(cfg=dict(audit_split=-1)) == pn.PN_EINVAL
    assert pn.surrogate_cfg().audit_split == 0
    assert L.pn_batch_resident_pairs(ctypes.byref(pn.Tuning(7, 1, 64))) == 0   # invalid tuning
    assert L.pn_batch_resident_pairs(None) >= 0
    assert scan(t_all=0.0) == pn.PN_EINVAL
    assert scan(std_=bad_std) == pn.PN_EINVAL
    assert scan(model=dict(pn_order=5)) == pn.PN_EINVAL
    assert scan(corr=dict(mode=9)) == pn.PN_EINVAL
    assert scan(n=-1) == pn.PN_EINVAL
    assert scan(ws=None) == pn.PN_ENOWS
    assert scan(ws_bytes=16) == pn.PN_ENOWS
    assert scan(n=0) == pn.PN_OK and integrated.value == 0
    assert L.pn_surrogate_scan_workspace_size(0, 2048) == 0
    assert L.pn_surrogate_scan_workspace_size(1000, 0) == 0
    assert L.pn_surrogate_scan_workspace_size(1000, 2048) > 1000 * (8 * 4 * 2 + 12 * 8)


def test_fused_inference_rejects_misaligned_features(pn):
    L = pn.lib()
    net = pn.Mlp(*[pn.P4(*([256] * 4)) for _ in range(7)])
    out = ctypes.c_void_p(256)
    assert L.pn_mlp_infer_fused(ctypes.byref(net), ctypes.c_void_p(8), ctypes.c_int64(10), out, None) == pn.PN_EINVAL
    assert L.pn_mlp_infer_fused(ctypes.byref(net), None, ctypes.c_int64(10), out, None) == pn.PN_EINVAL
    assert L.pn_mlp_infer_fused(ctypes.byref(net), ctypes.c_void_p(8), ctypes.c_int64(0), out, None) == pn.PN_OK
    assert L.pn_mlp_infer_fused(ctypes.byref(net), ctypes.c_void_p(256), ctypes.c_int64(-1), out, None) == pn.PN_EINVAL


def test_workspace_sizes_and_shutdown(pn):
    L = pn.lib()
    assert L.pn_fli_scan_workspace_size(0) == 0 and L.pn_fli_scan_workspace_size(10 ** 6) == 0
    L.pn_shutdown()          # forgets cached tunings; harmless when there are none
    L.pn_shutdown()
    step = ctypes.c_int32(0)
    net = pn.Mlp(*[pn.P4(*([8] * 4)) for _ in range(7)])
    one = ctypes.c_void_p(8)
    def train(step_p=ctypes.byref(step), nbatch=2, batch=16, order=one):
        return L.pn_mlp_train(ctypes.byref(net), step_p, one, one, one, order, ctypes.c_int64(nbatch),
                              ctypes.c_int32(batch), ctypes.c_float(1e-3), one, one, ctypes.c_size_t(1 << 30), None)
    assert train(step_p=None) == pn.PN_EINVAL
    assert train(nbatch=-1) == pn.PN_EINVAL
    assert train(batch=0) == pn.PN_EINVAL
    assert train(order=None) == pn.PN_EINVAL
    assert train(nbatch=0) == pn.PN_OK and step.value == 0


def test_resumable_batch_scan_arguments(pn):
    """The checkpointed batch scan: workspace size (queue + two record tables
    of min(n, 2^18) records of 324 bytes), and rejection of bad arguments
    before anything is launched."""
    L = pn.lib()
    base = L.pn_batch_workspace_size(1000)
    size = L.pn_batch_ckpt_workspace_size(1000)
    assert size >= base + 256 + 2 * 1000 * 324 and size < base + 256 + 2 * 1000 * 324 + 20 * 256
    assert L.pn_batch_ckpt_workspace_size(-1) == 0
    big = L.pn_batch_ckpt_workspace_size(10 ** 7) - L.pn_batch_workspace_size(10 ** 7)
    assert big < 2 * (1 << 18) * 324 + 21 * 256       # tables capped at 2^18 records
    m = pn.model_struct()
    p = pn.Params(None, None, None, 1.0, 1.0, 1.0)
    one = ctypes.c_void_p(8)
    so = pn.ScanOut(8, 8, 8, None, None, None, None, None, None, 0, 0)

    def run(resume=0, max_chunks=1, t_end=one, out=so, n=4):
        return L.pn_batch_scan_resumable(ctypes.byref(m), p, ctypes.byref(pn.integrator_struct()),
                                         ctypes.byref(pn.correction_struct()), ctypes.byref(pn.fli_struct()),
                                         ctypes.c_int64(n), one, ctypes.c_int64(4), t_end, ctypes.byref(out), None,
                                         ctypes.c_int32(resume), ctypes.c_int32(max_chunks), one,
                                         ctypes.c_size_t(1 << 30), None)
    assert run(resume=2) == pn.PN_EINVAL
    assert run(resume=-1) == pn.PN_EINVAL
    assert run(max_chunks=-1) == pn.PN_EINVAL
    assert run(t_end=None) == pn.PN_EINVAL
    assert run(out=pn.ScanOut(8, 8, 8, None, None, None, None, None, 8, 10, 5)) == pn.PN_EINVAL
    assert run(n=-1) == pn.PN_EINVAL
    pending = ctypes.c_int64(7)
    assert L.pn_batch_scan_pending(one, ctypes.c_int64(0), ctypes.byref(pending), None) == pn.PN_OK
    assert pending.value == 0
    assert L.pn_batch_scan_pending(one, ctypes.c_int64(4), None, None) == pn.PN_EINVAL
    assert L.pn_batch_scan_pending(None, ctypes.c_int64(4), ctypes.byref(pending), None) == pn.PN_EINVAL


def test_radiation_reaction_flag(pn):
    """rad_reaction must be 0 or 1; the scans refuse the dissipative model."""
    L = pn.lib()
    one = ctypes.c_void_p(8)
    p = pn.Params(None, None, None, 1.0, 1.0, 1.0)
    bad = pn.model_struct(dict(rad_reaction=2))
    assert L.pn_rhs(ctypes.byref(bad), p, ctypes.c_int64(4), one, ctypes.c_int64(4), one, None) == pn.PN_EINVAL
    rr = pn.model_struct(dict(rad_reaction=1))
    so = pn.ScanOut(8, 8, 8, None, None, None, None, None, None, 0, 0)
    assert L.pn_fli_scan(ctypes.byref(rr), p, ctypes.byref(pn.integrator_struct()),
                         ctypes.byref(pn.correction_struct()), ctypes.byref(pn.fli_struct()), ctypes.c_int64(4), one,
                         ctypes.c_int64(4), None, ctypes.c_double(1.0), ctypes.byref(so), None) == pn.PN_EINVAL
    assert L.pn_batch_scan(ctypes.byref(rr), p, ctypes.byref(pn.integrator_struct()),
                           ctypes.byref(pn.correction_struct()), ctypes.byref(pn.fli_struct()), ctypes.c_int64(4),
                           one, ctypes.c_int64(4), one, ctypes.byref(so), None, one, ctypes.c_size_t(1 << 30),
                           None) == pn.PN_EINVAL
    assert L.pn_batch_scan_resumable(ctypes.byref(rr), p, ctypes.byref(pn.integrator_struct()),
                                     ctypes.byref(pn.correction_struct()), ctypes.byref(pn.fli_struct()),
                                     ctypes.c_int64(4), one, ctypes.c_int64(4), one, ctypes.byref(so), None,
                                     ctypes.c_int32(0), ctypes.c_int32(0), one, ctypes.c_size_t(1 << 30),
                                     None) == pn.PN_EINVAL
    m = pn.model_struct()
    assert m.rad_reaction == 0


def test_scan_kernel_resources_arguments(pn):
    L = pn.lib()
    assert L.pn_scan_kernel_resources(ctypes.c_int32(7), ctypes.c_int32(2), None, None, None) == pn.PN_EINVAL
    assert L.pn_scan_kernel_resources(ctypes.c_int32(0), ctypes.c_int32(9), None, None, None) == pn.PN_EINVAL


def test_orbit_counts_beyond_the_launch_limit_rejected(pn):
    """n above 2^31 - 1 would overflow a launch grid of two lanes per orbit
    (HIP allows fewer than 2^32 work-items in x) and the 32-bit orbit indices
    of the balanced scan's records: refused before launch."""
    L = pn.lib()
    one = ctypes.c_void_p(8)
    m = pn.model_struct()
    p = pn.Params(None, None, None, 1.0, 1.0, 1.0)
    big = ctypes.c_int64(1 << 31)
    assert L.pn_rhs(ctypes.byref(m), p, big, one, big, one, None) == pn.PN_EINVAL
    assert L.pn_step(ctypes.byref(m), p, ctypes.byref(pn.integrator_struct()), None, big, one, big, None,
                     ctypes.c_int64(1), None) == pn.PN_EINVAL
    so = pn.ScanOut(8, 8, 8, None, None, None, None, None, None, 0, 0)
    assert L.pn_fli_scan(ctypes.byref(m), p, ctypes.byref(pn.integrator_struct()),
                         ctypes.byref(pn.correction_struct()), ctypes.byref(pn.fli_struct()), big, one, big, None,
                         ctypes.c_double(1.0), ctypes.byref(so), None) == pn.PN_EINVAL


def test_missing_library_fails_loudly(monkeypatch):
    from paper_1802_00147_amd import pn as P
    monkeypatch.setattr(P, "_lib", None)
    monkeypatch.setattr(P, "LIB_PATH", "/nonexistent/libpn_hip.so")
    with pytest.raises(OSError):
        P.lib()


def test_balanced_scan_arguments(pn):
    """pn_fli_scan_balanced validates like pn_fli_scan (before any device
    call) and also rejects negative or oversized slot counts; its schedule
    query with explicit slots is host-only and agrees with pn_balanced_plan;
    the workspace is two tables of one pair record per slot."""
    L = pn.lib()
    m = pn.model_struct()
    p = pn.Params(None, None, None, 1.0, 1.0, 1.0)
    one = ctypes.c_void_p(8)
    so = pn.ScanOut(8, 8, 8, None, None, None, None, None, None, 0, 0)

    def scan(integ=None, corr=None, fli=None, t_all=1.0, out=so, n=4, ld=4, slots=16):
        return L.pn_fli_scan_balanced(ctypes.byref(m), p, ctypes.byref(pn.integrator_struct(integ)),
                                      ctypes.byref(pn.correction_struct(corr)), ctypes.byref(pn.fli_struct(fli)),
                                      ctypes.c_int64(n), one, ctypes.c_int64(ld), ctypes.c_double(t_all),
                                      ctypes.byref(out), ctypes.c_int64(slots), None, ctypes.c_size_t(0), None)

    assert scan(integ=dict(h=0.0)) == pn.PN_EINVAL
    assert scan(corr=dict(mode=7)) == pn.PN_EINVAL
    assert scan(fli=dict(d0=0.0)) == pn.PN_EINVAL
    assert scan(t_all=float("nan")) == pn.PN_EINVAL
    assert scan(t_all=1e30) == pn.PN_EINVAL                  # more than 4e18 steps
    assert scan(n=-1) == pn.PN_EINVAL
    assert scan(ld=3) == pn.PN_EINVAL
    assert scan(slots=-1) == pn.PN_EINVAL
    assert scan(slots=(1 << 24) + 1) == pn.PN_EINVAL
    assert scan(out=pn.ScanOut(8, None, 8, None, None, None, None, None, None, 0, 0)) == pn.PN_EINVAL
    m_rr = pn.model_struct(dict(rad_reaction=1))
    assert L.pn_fli_scan_balanced(ctypes.byref(m_rr), p, ctypes.byref(pn.integrator_struct()),
                                  ctypes.byref(pn.correction_struct()), ctypes.byref(pn.fli_struct()),
                                  ctypes.c_int64(4), one, ctypes.c_int64(4), ctypes.c_double(1.0),
                                  ctypes.byref(so), ctypes.c_int64(16), None, ctypes.c_size_t(0), None) == pn.PN_EINVAL
    # A valid call with explicit slots and no workspace: PN_ENOWS, nothing launched.
    assert scan(t_all=100.0, slots=2) == pn.PN_ENOWS
    # Explicit slots: the host plan, no device needed.
    sch = pn.balanced_schedule(1000, 300.0, slots=64)
    assert (sch["slot_len"], sch["launches"]) == pn.balanced_plan(1000, 300, 64) and sch["slots"] == 64
    assert pn.balanced_schedule(0, 300.0, slots=64)["launches"] == 0
    assert pn.balanced_schedule(1000, 0.0, slots=64)["launches"] == 0
    with pytest.raises(pn.PnError):
        pn.balanced_schedule(1000, 300.0, slots=-5)
    with pytest.raises(pn.PnError):
        pn.balanced_schedule(1000, 300.0, integrator=dict(h=0.0), slots=4)
    assert L.pn_fli_scan_balanced_workspace_size(0) == 0
    assert L.pn_fli_scan_balanced_workspace_size((1 << 24) + 1) == 0
    assert L.pn_fli_scan_balanced_workspace_size(1000) >= 2 * 1000 * 2 * (16 * 8 + 8 + 8 + 8 + 4 + 4)
    for args in ((9, 0), (0, 9)):
        v, w = ctypes.c_int32(0), ctypes.c_int32(0)
        sc = ctypes.c_int64(0)
        assert L.pn_balanced_kernel_resources(ctypes.c_int32(args[0]), ctypes.c_int32(args[1]), ctypes.byref(v),
                                              ctypes.byref(sc), ctypes.byref(w)) == pn.PN_EINVAL


def test_train_workspace_layout(pn):
    """The tensors a training step leaves in its workspace lie inside it, in
    order, 256-byte aligned, each large enough for its rows; after them the
    workspace still holds the step's own buffers: the FP32 weight and bias
    gradients, four 4 MB split-K partial buffers and the bfloat16 copies of
    W2^T and W3^T."""
    own = (2 * 256 * 256 + 256 * 7 + 2 * 256 + 4 * 256) * 4 + 4 * (1 << 22) + 2 * 256 * 256 * 2
    for batch in (1, 100, 2048, 4096):
        off = pn.mlp_train_workspace_layout(batch)
        size = pn.lib().pn_mlp_train_workspace_size(batch)
        need = [batch * 8 * 2, batch * 256 * 2, batch * 256 * 2, batch * 256 * 2, batch * 2 * 4,
                batch * 2 * 2, batch * 256 * 2, batch * 256 * 2, batch * 256 * 2]
        assert off[0] == 0 and all(o % 256 == 0 for o in off)
        for k in range(8):
            assert off[k + 1] >= off[k] + need[k]
        assert off[8] + need[8] + own <= size
    bad = (ctypes.c_size_t * 9)()
    assert pn.lib().pn_mlp_train_workspace_layout(ctypes.c_int32(0), bad) == pn.PN_EINVAL
    assert pn.lib().pn_mlp_train_workspace_layout(ctypes.c_int32(5), None) == pn.PN_EINVAL


def test_noalloc_batch_scan_rejects_more_orbits_than_its_static_workspace(pn):
    """pn_batch_scan_noalloc holds at most 2^20 orbits; more is refused with
    PN_EINVAL before anything touches a device (fake non-null pointers)."""
    m, integ, corr, fli = (pn.model_struct(), pn.integrator_struct(), pn.correction_struct(), pn.fli_struct())
    so = pn.ScanOut()
    for f in ("fli", "label", "status"):
        setattr(so, f, 8)
    p = pn.Params(None, None, None, 1.0, 1.0, 1.0)
    n = (1 << 20) + 1
    st = pn.lib().pn_batch_scan_noalloc(ctypes.byref(m), p, ctypes.byref(integ), ctypes.byref(corr),
                                       ctypes.byref(fli), ctypes.c_int64(n), ctypes.c_void_p(8),
                                       ctypes.c_int64(n), ctypes.c_void_p(8), ctypes.byref(so), None, None)
    assert st == pn.PN_EINVAL
    assert b"2^20" in pn.lib().pn_last_error()


def test_mlp_wrappers_reject_malformed_tensors(pn):
    """The binding checks the arrays the network's kernels address through
    bare pointers: host tensors, other dtypes and other shapes raise
    ValueError before any device call."""
    import torch
    host = torch.zeros(4, 8)
    with pytest.raises(ValueError):
        pn.mlp_infer_fused(None, host)
    with pytest.raises(ValueError):
        pn.mlp_infer(None, host)
    with pytest.raises(ValueError):
        pn.mlp_infer_fused(None, torch.zeros(4, 7))
    with pytest.raises(ValueError):
        pn.mlp_infer_fused(None, torch.zeros(32, dtype=torch.float32))
    with pytest.raises(ValueError):
        pn.mlp_train_step(None, host, torch.zeros(4), torch.zeros(4), torch.zeros(2, dtype=torch.int32), 1e-3,
                          torch.zeros(1))
    with pytest.raises(ValueError):
        pn.mlp_train(None, host, torch.zeros(4), torch.zeros(4), torch.zeros(2, dtype=torch.int32), 2, 1e-3,
                     torch.zeros(1))
