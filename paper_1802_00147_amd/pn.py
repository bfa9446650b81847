"""Thin ctypes binding of the C ABI in include/pn.h (libpn_hip.so).

Argument marshalling only: every computation runs in the HIP kernels of
csrc/pn_kernels.hip.  Arrays are torch tensors on a ROCm device (torch is used
for device memory and streams); states use the library's structure-of-arrays
layout, a (12, ld) float64 tensor whose row c holds component c of every orbit.

Settings are plain dicts whose keys are the fields of the C structs; missing
keys take the library's own defaults (pn_default_*).  The library is loaded on
first use; a missing library raises, there is no fallback path.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpn_hip.so")

PN_OK, PN_EINVAL, PN_ENOWS, PN_EDEVICE = 0, 1, 2, 3
ORBIT_OK, ORBIT_MERGED, ORBIT_ESCAPED, ORBIT_NONFINITE, ORBIT_UNBOUND_INIT, ORBIT_BADPARAM = range(6)
ORBIT_NEWTON_NOCONV = 0x100
METHODS = {"rk4": 0, "rk5": 1}
MODES = {"none": 0, "spin": 1, "six": 2, "dual": 3}
THR = {"literal": 0, "log_t": 1}


class PnError(RuntimeError):
    def __init__(self, fn, status, text):
        super().__init__(f"{fn} returned {status} ({text})")
        self.status = status


class Model(ctypes.Structure):
    _fields_ = [("pn_order", ctypes.c_int32), ("spin_orbit", ctypes.c_int32),
                ("spin_spin", ctypes.c_int32), ("quad_mono", ctypes.c_int32),
                ("spin_units", ctypes.c_int32), ("rad_reaction", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_void_p), ("chi1", ctypes.c_void_p), ("chi2", ctypes.c_void_p),
                ("beta0", ctypes.c_double), ("chi1_0", ctypes.c_double), ("chi2_0", ctypes.c_double)]


class Integrator(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("h", ctypes.c_double)]


class Correction(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("sweeps", ctypes.c_int32), ("w1", ctypes.c_double), ("w2", ctypes.c_double)]


class FliCfg(ctypes.Structure):
    _fields_ = [("d0", ctypes.c_double), ("d_renorm", ctypes.c_double), ("shadow_axis", ctypes.c_int32),
                ("thr_at_1e5", ctypes.c_double), ("thr_scaling", ctypes.c_int32),
                ("r_merge", ctypes.c_double), ("r_esc", ctypes.c_double)]


class ScanOut(ctypes.Structure):
    _fields_ = [("fli", ctypes.c_void_p), ("label", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("y_final", ctypes.c_void_p), ("dH", ctypes.c_void_p), ("dJ", ctypes.c_void_p),
                ("newton_max", ctypes.c_void_p), ("renorms", ctypes.c_void_p),
                ("trace", ctypes.c_void_p), ("trace_every", ctypes.c_int64), ("ntrace", ctypes.c_int64),
                ("steps", ctypes.c_void_p)]


class SurrogateCfg(ctypes.Structure):
    _fields_ = [("margin", ctypes.c_float), ("audit_frac", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("refine_epochs", ctypes.c_int32), ("refine_batch", ctypes.c_int32), ("refine_lr", ctypes.c_float),
                ("refine_seed", ctypes.c_uint64), ("refine_cosine", ctypes.c_int32), ("audit_split", ctypes.c_int64)]


class SurrogateStats(ctypes.Structure):
    _fields_ = [("phase_ms", ctypes.c_float * 4), ("scan_ms", ctypes.c_float * 2),
                ("scan_kernel", ctypes.c_int32 * 2), ("scan_launches", ctypes.c_int32 * 2),
                ("points", ctypes.c_int64 * 2), ("orbit_steps", ctypes.c_int64 * 2)]


SCAN_KERNELS = {0: None, 1: "k_fli_scan", 2: "k_wrap_scan", 3: "k_batch_scan"}


class Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32), ("chunk_steps", ctypes.c_int32)]


_lib = None

# Every symbol include/pn.h declares.
EXPORTS = ["pn_default_model", "pn_default_integrator", "pn_default_correction", "pn_default_fli_cfg",
           "pn_init_state", "pn_rhs", "pn_invariants", "pn_manifold_correct", "pn_step", "pn_fli_scan",
           "pn_default_tuning", "pn_batch_workspace_size", "pn_batch_scan", "pn_autotune_batch",
           "pn_batch_graph_create", "pn_graph_launch", "pn_graph_destroy",
           "pn_mlp_param_count", "pn_mlp_sync_bf16", "pn_mlp_features", "pn_mlp_train_workspace_size",
           "pn_mlp_train_workspace_layout",
           "pn_mlp_train_step", "pn_mlp_infer_workspace_size", "pn_mlp_infer", "pn_surrogate_gate",
           "pn_surrogate_merge", "pn_gemm_bf16", "pn_init_state_gather", "pn_mlp_targets",
           "pn_trajectory", "pn_gw_polarizations", "pn_mlp_infer_fused",
           "pn_default_surrogate_cfg", "pn_surrogate_scan_workspace_size", "pn_surrogate_scan",
           "pn_mlp_train", "pn_fli_scan_workspace_size", "pn_shutdown",
           "pn_batch_ckpt_workspace_size", "pn_batch_scan_resumable", "pn_batch_scan_pending",
           "pn_batch_scan_noalloc",
           "pn_batch_resident_pairs", "pn_scan_kernel_resources",
           "pn_balanced_plan", "pn_balanced_piece", "pn_fli_scan_balanced_schedule",
           "pn_fli_scan_balanced_workspace_size", "pn_fli_scan_balanced", "pn_balanced_kernel_resources",
           "pn_version", "pn_status_string", "pn_last_error"]


def lib():
    """Load libpn_hip.so (raises OSError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"{LIB_PATH} is missing: build it with paper_1802_00147_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        L.pn_status_string.restype = ctypes.c_char_p
        L.pn_last_error.restype = ctypes.c_char_p
        L.pn_version.restype = ctypes.c_int32
        for name in ("pn_init_state", "pn_rhs", "pn_invariants", "pn_manifold_correct", "pn_step",
                     "pn_fli_scan", "pn_batch_scan", "pn_autotune_batch", "pn_batch_graph_create",
                     "pn_graph_launch", "pn_mlp_sync_bf16", "pn_mlp_features", "pn_mlp_train_step",
                     "pn_mlp_infer", "pn_surrogate_gate", "pn_surrogate_merge", "pn_gemm_bf16",
                     "pn_init_state_gather", "pn_mlp_targets", "pn_trajectory", "pn_gw_polarizations",
                     "pn_mlp_infer_fused", "pn_surrogate_scan", "pn_mlp_train"):
            getattr(L, name).restype = ctypes.c_int
        L.pn_fli_scan_workspace_size.restype = ctypes.c_size_t
        L.pn_fli_scan_workspace_size.argtypes = [ctypes.c_int64]
        L.pn_shutdown.restype = None
        L.pn_surrogate_scan_workspace_size.restype = ctypes.c_size_t
        L.pn_surrogate_scan_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int32]
        for name in ("pn_mlp_param_count", "pn_mlp_train_workspace_size", "pn_mlp_infer_workspace_size"):
            getattr(L, name).restype = ctypes.c_size_t
        L.pn_mlp_param_count.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.pn_mlp_train_workspace_size.argtypes = [ctypes.c_int32]
        L.pn_mlp_infer_workspace_size.argtypes = [ctypes.c_int64]
        L.pn_batch_workspace_size.restype = ctypes.c_size_t
        L.pn_batch_workspace_size.argtypes = [ctypes.c_int64]
        L.pn_batch_resident_pairs.restype = ctypes.c_int64
        L.pn_fli_scan_balanced_workspace_size.restype = ctypes.c_size_t
        L.pn_fli_scan_balanced_workspace_size.argtypes = [ctypes.c_int64]
        L.pn_batch_ckpt_workspace_size.restype = ctypes.c_size_t
        L.pn_batch_ckpt_workspace_size.argtypes = [ctypes.c_int64]
        L.pn_graph_destroy.argtypes = [ctypes.c_void_p]
        _lib = L
    return _lib


def _defaults(struct, fill):
    s = struct()
    getattr(lib(), fill)(ctypes.byref(s))
    return s


def model_struct(over=None):
    s = _defaults(Model, "pn_default_model")
    for k, v in (over or {}).items():
        setattr(s, k, int(v))
    return s


def integrator_struct(over=None):
    s = _defaults(Integrator, "pn_default_integrator")
    for k, v in (over or {}).items():
        setattr(s, k, METHODS[v] if k == "method" and isinstance(v, str) else v)
    return s


def correction_struct(over=None):
    s = _defaults(Correction, "pn_default_correction")
    for k, v in (over or {}).items():
        setattr(s, k, MODES[v] if k == "mode" and isinstance(v, str) else v)
    return s


def fli_struct(over=None):
    s = _defaults(FliCfg, "pn_default_fli_cfg")
    for k, v in (over or {}).items():
        setattr(s, k, THR[v] if k == "thr_scaling" and isinstance(v, str) else v)
    return s


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check(fn, st):
    if st != PN_OK:
        L = lib()
        raise PnError(fn, st, (L.pn_status_string(st) or b"").decode() + " " + (L.pn_last_error() or b"").decode())


def _require(cond, msg):
    """Argument check that stays on under python -O."""
    if not cond:
        raise ValueError(msg)


def _dev(t, dtype, name, shape=None, min_numel=None):
    """A contiguous device tensor of the given dtype (and shape, or at least
    min_numel elements), else ValueError: the kernels read and write these
    arrays through bare pointers, so a wrong size would run past them."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {dtype} device tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name}: expected at least {min_numel} elements, got {t.numel()}")
    return t


def _feat_rows(feat):
    """Rows of a feature array [rows][8] (float32, contiguous, on the device)."""
    if not isinstance(feat, torch.Tensor) or feat.dim() != 2:
        raise ValueError("feat: expected a [rows][8] float32 device tensor")
    _dev(feat, torch.float32, "feat", shape=(feat.shape[0], 8))
    return feat.shape[0]


def _dev_f64(t, n=None):
    _require(t.dtype == torch.float64 and t.is_cuda, "expected a float64 device tensor")
    if n is not None:
        _require(t.numel() >= n, f"expected at least {n} elements, got {t.numel()}")
    return t.contiguous()


def params_struct(beta, chi1, chi2):
    """Scalars give one shared parameter set; tensors give per-orbit device arrays.
    Returns (struct, keepalive)."""
    if all(isinstance(v, torch.Tensor) for v in (beta, chi1, chi2)):
        keep = [_dev_f64(v) for v in (beta, chi1, chi2)]
        return Params(keep[0].data_ptr(), keep[1].data_ptr(), keep[2].data_ptr(), 0.0, 0.0, 0.0), keep
    return Params(None, None, None, float(beta), float(chi1), float(chi2)), []


def _state(y):
    _require(y.dim() == 2 and y.shape[0] == 12 and y.dtype == torch.float64 and y.is_cuda,
             "y: expected a float64 [12][ld] device tensor")
    _require(y.is_contiguous(), "y: expected a contiguous tensor")
    return y.shape[1]


def init_state(r0, p0, th1, ph1, th2, ph2, beta, chi1, chi2, model=None, ld=None):
    n = r0.numel()
    ld = ld or n
    cols = [_dev_f64(t, n) for t in (r0, p0, th1, ph1, th2, ph2)]
    y0 = torch.empty((12, ld), dtype=torch.float64, device=r0.device)
    m = model_struct(model)
    p, keep = params_struct(beta, chi1, chi2)
    st = lib().pn_init_state(ctypes.byref(m), p, ctypes.c_int64(n), *[_ptr(c) for c in cols], _ptr(y0),
                             ctypes.c_int64(ld), _stream(r0.device))
    _check("pn_init_state", st)
    return y0


def rhs(y, beta, chi1, chi2, model=None, n=None):
    ld = _state(y)
    n = ld if n is None else n
    f = torch.empty_like(y)
    p, keep = params_struct(beta, chi1, chi2)
    st = lib().pn_rhs(ctypes.byref(model_struct(model)), p, ctypes.c_int64(n), _ptr(y), ctypes.c_int64(ld),
                      _ptr(f), _stream(y.device))
    _check("pn_rhs", st)
    return f


def invariants(y, beta, chi1, chi2, model=None, n=None):
    ld = _state(y)
    n = ld if n is None else n
    H = torch.empty(ld, dtype=torch.float64, device=y.device)
    J = torch.empty((3, ld), dtype=torch.float64, device=y.device)
    p, keep = params_struct(beta, chi1, chi2)
    st = lib().pn_invariants(ctypes.byref(model_struct(model)), p, ctypes.c_int64(n), _ptr(y),
                             ctypes.c_int64(ld), _ptr(H), _ptr(J), _stream(y.device))
    _check("pn_invariants", st)
    return H, J


def manifold_correct(y, ref, beta, chi1, chi2, model=None, correction=None, n=None):
    """Correct y (12, ld) in place against ref (4, ld); returns iteration counts."""
    ld = _state(y)
    n = ld if n is None else n
    _require(ref.shape == (4, ld) and ref.dtype == torch.float64 and ref.is_contiguous(),
             "ref: expected a contiguous float64 [4][ld] tensor")
    it = torch.empty(ld, dtype=torch.int32, device=y.device)
    p, keep = params_struct(beta, chi1, chi2)
    st = lib().pn_manifold_correct(ctypes.byref(model_struct(model)), p,
                                   ctypes.byref(correction_struct(correction)), ctypes.c_int64(n), _ptr(y),
                                   ctypes.c_int64(ld), _ptr(ref), _ptr(it), _stream(y.device))
    _check("pn_manifold_correct", st)
    return it


def step(y, beta, chi1, chi2, nsteps, model=None, integrator=None, correction=None, ref=None, n=None):
    """nsteps steps of y (12, ld) in place; correction None means uncorrected.
    With model rad_reaction=1 a given ref (4, ld) advances in place too."""
    ld = _state(y)
    n = ld if n is None else n
    if ref is not None:
        _require(ref.shape == (4, ld) and ref.dtype == torch.float64 and ref.is_contiguous(),
                 "ref: expected a contiguous float64 [4][ld] tensor")
    p, keep = params_struct(beta, chi1, chi2)
    cc = ctypes.byref(correction_struct(correction)) if correction is not None else None
    st = lib().pn_step(ctypes.byref(model_struct(model)), p, ctypes.byref(integrator_struct(integrator)), cc,
                       ctypes.c_int64(n), _ptr(y), ctypes.c_int64(ld), _ptr(ref), ctypes.c_int64(nsteps),
                       _stream(y.device))
    _check("pn_step", st)
    return y


def scan_outputs(n, ld, device, full=True, trace_every=0, nsteps_max=0):
    o = dict(fli=torch.empty(ld, dtype=torch.float64, device=device),
             label=torch.empty(ld, dtype=torch.int8, device=device),
             status=torch.empty(ld, dtype=torch.int32, device=device),
             steps=torch.empty(ld, dtype=torch.int64, device=device))
    if full:
        o.update(y_final=torch.empty((12, ld), dtype=torch.float64, device=device),
                 dH=torch.empty(ld, dtype=torch.float64, device=device),
                 dJ=torch.empty(ld, dtype=torch.float64, device=device),
                 newton_max=torch.empty(ld, dtype=torch.int32, device=device),
                 renorms=torch.empty(ld, dtype=torch.int64, device=device))
    if trace_every > 0:
        ntrace = nsteps_max // trace_every
        o["trace"] = torch.full((ntrace, ld), float("nan"), dtype=torch.float64, device=device)
        o["trace_every"] = trace_every
    return o


def trajectory(y, beta, chi1, chi2, nsteps, every, model=None, integrator=None, correction=None, ref=None,
               n=None):
    """pn_step that also returns the states after every `every` steps as a
    (nsteps // every, 12, ld) tensor; y advances in place."""
    ld = _state(y)
    n = ld if n is None else n
    rows = nsteps // every
    traj = torch.empty((rows, 12, ld), dtype=torch.float64, device=y.device)
    if ref is not None:
        _require(ref.shape == (4, ld) and ref.dtype == torch.float64 and ref.is_contiguous(),
                 "ref: expected a contiguous float64 [4][ld] tensor")
    p, keep = params_struct(beta, chi1, chi2)
    cc = ctypes.byref(correction_struct(correction)) if correction is not None else None
    st = lib().pn_trajectory(ctypes.byref(model_struct(model)), p, ctypes.byref(integrator_struct(integrator)), cc,
                             ctypes.c_int64(n), _ptr(y), ctypes.c_int64(ld), _ptr(ref), ctypes.c_int64(nsteps),
                             ctypes.c_int64(every), _ptr(traj) if rows > 0 else None, _stream(y.device))
    _check("pn_trajectory", st)
    return traj


def gw_polarizations(traj, beta, chi1, chi2, nhat, phat, dist=1.0, model=None, n=None):
    """(h_plus, h_cross), each (ns, ld), of eq. (14) for states traj (ns, 12, ld)
    or (12, ld)."""
    if traj.dim() == 2:
        traj = traj.unsqueeze(0)
    _require(traj.dim() == 3 and traj.shape[1] == 12 and traj.dtype == torch.float64 and traj.is_contiguous(),
             "traj: expected a contiguous float64 [rows][12][ld] tensor")
    ns, _, ld = traj.shape
    n = ld if n is None else n
    hp = torch.empty((ns, ld), dtype=torch.float64, device=traj.device)
    hx = torch.empty_like(hp)
    p, keep = params_struct(beta, chi1, chi2)
    N3 = (ctypes.c_double * 3)(*[float(v) for v in nhat])
    P3 = (ctypes.c_double * 3)(*[float(v) for v in phat])
    st = lib().pn_gw_polarizations(ctypes.byref(model_struct(model)), p, ctypes.c_int64(n), ctypes.c_int64(ns),
                                   _ptr(traj), ctypes.c_int64(ld), N3, P3, ctypes.c_double(dist), _ptr(hp), _ptr(hx),
                                   _stream(traj.device))
    _check("pn_gw_polarizations", st)
    return hp, hx


def fli_scan(y0, t_end, beta, chi1, chi2, model=None, integrator=None, correction=None, fli=None,
             out=None, n=None, full=True, trace_every=0):
    """Fused FLI scan of the orbits in y0 (12, ld).  t_end: float or (ld,) tensor.
    Returns the dict of output tensors (allocated unless out is given)."""
    ld = _state(y0)
    n = ld if n is None else n
    integ = integrator_struct(integrator)
    if out is None:
        tmax = float(t_end.max()) if isinstance(t_end, torch.Tensor) else float(t_end)
        nmax = int(-(-tmax // integ.h)) if tmax > 0 else 0
        out = scan_outputs(n, ld, y0.device, full=full, trace_every=trace_every, nsteps_max=nmax)
    so = _scan_out_struct(out)
    p, keep = params_struct(beta, chi1, chi2)
    if isinstance(t_end, torch.Tensor):
        tptr, tall = _ptr(_dev_f64(t_end, n)), 0.0
    else:
        tptr, tall = None, float(t_end)
    st = lib().pn_fli_scan(ctypes.byref(model_struct(model)), p, ctypes.byref(integ),
                           ctypes.byref(correction_struct(correction)), ctypes.byref(fli_struct(fli)),
                           ctypes.c_int64(n), _ptr(y0), ctypes.c_int64(ld), tptr, ctypes.c_double(tall),
                           ctypes.byref(so), _stream(y0.device))
    _check("pn_fli_scan", st)
    return out


def tuning_struct(over=None):
    t = _defaults(Tuning, "pn_default_tuning")
    for k, v in (over or {}).items():
        setattr(t, k, int(v))
    return t


def batch_workspace(n, device):
    nbytes = int(lib().pn_batch_workspace_size(ctypes.c_int64(n)))
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def _scan_out_struct(out):
    return ScanOut(*[out[k].data_ptr() if k in out else None
                     for k in ("fli", "label", "status", "y_final", "dH", "dJ", "newton_max", "renorms", "trace")],
                   int(out.get("trace_every", 0)), int(out["trace"].shape[0]) if "trace" in out else 0,
                   out["steps"].data_ptr() if "steps" in out else None)


def _batch_common(y0, t_end, beta, chi1, chi2, model, integrator, correction, fli, out, n, full, trace_every, ws):
    ld = _state(y0)
    n = ld if n is None else n
    integ = integrator_struct(integrator)
    _require(isinstance(t_end, torch.Tensor), "batch scans take per-orbit end times")
    t_end = _dev_f64(t_end, n)
    if out is None:
        tmax = float(t_end[:n].max()) if n > 0 else 0.0
        nmax = int(-(-tmax // integ.h)) if tmax > 0 else 0
        out = scan_outputs(n, ld, y0.device, full=full, trace_every=trace_every, nsteps_max=nmax)
    if ws is None:
        ws = batch_workspace(n, y0.device)
    p, keep = params_struct(beta, chi1, chi2)
    return ld, n, integ, t_end, out, ws, p, keep


def batch_scan(y0, t_end, beta, chi1, chi2, model=None, integrator=None, correction=None, fli=None, out=None,
               n=None, full=True, trace_every=0, tuning=None, ws=None):
    """Persistent work-stealing scan of orbits with per-orbit t_end (tensor).
    tuning: dict or Tuning (None: the device's autotuned or default shape)."""
    ld, n, integ, t_end, out, ws, p, keep = _batch_common(y0, t_end, beta, chi1, chi2, model, integrator,
                                                          correction, fli, out, n, full, trace_every, ws)
    tu = None
    if tuning is not None:
        tu = ctypes.byref(tuning if isinstance(tuning, Tuning) else tuning_struct(tuning))
    so = _scan_out_struct(out)
    st = lib().pn_batch_scan(ctypes.byref(model_struct(model)), p, ctypes.byref(integ),
                             ctypes.byref(correction_struct(correction)), ctypes.byref(fli_struct(fli)),
                             ctypes.c_int64(n), _ptr(y0), ctypes.c_int64(ld), _ptr(t_end), ctypes.byref(so), tu,
                             _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(y0.device))
    _check("pn_batch_scan", st)
    return out


def batch_scan_noalloc(y0, t_end, beta, chi1, chi2, model=None, integrator=None, correction=None, fli=None,
                       out=None, n=None, full=True, tuning=None):
    """pn_batch_scan_noalloc: the persistent batch scan on the library's static
    device workspace (at most 2^20 orbits; calls on one device must not
    overlap).  Outputs as batch_scan."""
    ld = _state(y0)
    n = ld if n is None else n
    integ = integrator_struct(integrator)
    _require(isinstance(t_end, torch.Tensor), "batch scans take per-orbit end times")
    t_end = _dev_f64(t_end, n)
    if out is None:
        out = scan_outputs(n, ld, y0.device, full=full)
    p, keep = params_struct(beta, chi1, chi2)
    tu = None
    if tuning is not None:
        tu = ctypes.byref(tuning if isinstance(tuning, Tuning) else tuning_struct(tuning))
    so = _scan_out_struct(out)
    st = lib().pn_batch_scan_noalloc(ctypes.byref(model_struct(model)), p, ctypes.byref(integ),
                                     ctypes.byref(correction_struct(correction)), ctypes.byref(fli_struct(fli)),
                                     ctypes.c_int64(n), _ptr(y0), ctypes.c_int64(ld), _ptr(t_end), ctypes.byref(so),
                                     tu, _stream(y0.device))
    _check("pn_batch_scan_noalloc", st)
    return out


def batch_ckpt_workspace(n, device):
    nbytes = int(lib().pn_batch_ckpt_workspace_size(ctypes.c_int64(n)))
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def batch_scan_resumable(y0, t_end, beta, chi1, chi2, ws, resume, max_chunks, model=None, integrator=None,
                         correction=None, fli=None, out=None, n=None, full=True, tuning=None):
    """pn_batch_scan_resumable: one launch of a checkpointed batch scan.  ws
    (from batch_ckpt_workspace) holds the queue and the orbits in flight;
    resume=False starts the scan, resume=True continues it; max_chunks > 0
    interrupts every wavefront after that many chunks.  Returns the outputs;
    batch_scan_pending tells whether orbits remain."""
    ld = _state(y0)
    n = ld if n is None else n
    integ = integrator_struct(integrator)
    _require(isinstance(t_end, torch.Tensor), "batch scans take per-orbit end times")
    t_end = _dev_f64(t_end, n)
    if out is None:
        out = scan_outputs(n, ld, y0.device, full=full)
    p, keep = params_struct(beta, chi1, chi2)
    tu = None
    if tuning is not None:
        tu = ctypes.byref(tuning if isinstance(tuning, Tuning) else tuning_struct(tuning))
    so = _scan_out_struct(out)
    st = lib().pn_batch_scan_resumable(ctypes.byref(model_struct(model)), p, ctypes.byref(integ),
                                       ctypes.byref(correction_struct(correction)), ctypes.byref(fli_struct(fli)),
                                       ctypes.c_int64(n), _ptr(y0), ctypes.c_int64(ld), _ptr(t_end),
                                       ctypes.byref(so), tu, ctypes.c_int32(1 if resume else 0),
                                       ctypes.c_int32(max_chunks), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                       _stream(y0.device))
    _check("pn_batch_scan_resumable", st)
    return out


def scan_kernel_resources(integrator=None, correction=None):
    """pn_scan_kernel_resources: dict(vgprs, scratch_bytes, waves_per_simd)
    of the fused scan kernel for this integrator and correction mode."""
    integ = integrator_struct(integrator)
    mode = correction_struct(correction).mode
    v, w = ctypes.c_int32(0), ctypes.c_int32(0)
    sc = ctypes.c_int64(0)
    st = lib().pn_scan_kernel_resources(ctypes.c_int32(integ.method), ctypes.c_int32(mode), ctypes.byref(v),
                                        ctypes.byref(sc), ctypes.byref(w))
    _check("pn_scan_kernel_resources", st)
    return dict(vgprs=v.value, scratch_bytes=sc.value, waves_per_simd=w.value)


def balanced_kernel_resources(integrator=None, correction=None):
    """pn_balanced_kernel_resources: dict(vgprs, scratch_bytes, waves_per_simd)
    of the balanced scan's kernel for this integrator and correction mode."""
    integ = integrator_struct(integrator)
    mode = correction_struct(correction).mode
    v, w = ctypes.c_int32(0), ctypes.c_int32(0)
    sc = ctypes.c_int64(0)
    st = lib().pn_balanced_kernel_resources(ctypes.c_int32(integ.method), ctypes.c_int32(mode), ctypes.byref(v),
                                            ctypes.byref(sc), ctypes.byref(w))
    _check("pn_balanced_kernel_resources", st)
    return dict(vgprs=v.value, scratch_bytes=sc.value, waves_per_simd=w.value)


def balanced_plan(n, steps, slots):
    """pn_balanced_plan (host only): (slot length C, launches L)."""
    c, l = ctypes.c_int64(0), ctypes.c_int32(0)
    st = lib().pn_balanced_plan(ctypes.c_int64(n), ctypes.c_int64(steps), ctypes.c_int64(slots), ctypes.byref(c),
                                ctypes.byref(l))
    _check("pn_balanced_plan", st)
    return int(c.value), int(l.value)


def balanced_piece(n, steps, slot_len, slot, tau):
    """pn_balanced_piece (host only): (orbit, first_step, end_step, start)."""
    v = [ctypes.c_int64(0) for _ in range(4)]
    st = lib().pn_balanced_piece(ctypes.c_int64(n), ctypes.c_int64(steps), ctypes.c_int64(slot_len),
                                 ctypes.c_int64(slot), ctypes.c_int64(tau), *[ctypes.byref(x) for x in v])
    _check("pn_balanced_piece", st)
    return tuple(int(x.value) for x in v)


def balanced_schedule(n, t_end, integrator=None, correction=None, slots=0):
    """pn_fli_scan_balanced_schedule: dict(slots, slot_len, launches); launches
    0 means the plain fused scan runs."""
    p, c, l = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int32(0)
    st = lib().pn_fli_scan_balanced_schedule(ctypes.byref(integrator_struct(integrator)),
                                             ctypes.byref(correction_struct(correction)), ctypes.c_int64(n),
                                             ctypes.c_double(float(t_end)), ctypes.c_int64(slots),
                                             ctypes.byref(p), ctypes.byref(c), ctypes.byref(l))
    _check("pn_fli_scan_balanced_schedule", st)
    return dict(slots=int(p.value), slot_len=int(c.value), launches=int(l.value))


def balanced_workspace(slots, device):
    nbytes = int(lib().pn_fli_scan_balanced_workspace_size(ctypes.c_int64(slots)))
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def fli_scan_balanced(y0, t_end, beta, chi1, chi2, model=None, integrator=None, correction=None, fli=None,
                      out=None, n=None, full=True, trace_every=0, slots=0, ws=None):
    """pn_fli_scan_balanced: the fused scan of orbits that all end at t_end
    (a float), on the balanced schedule (slots = 0: the device's resident
    orbit pairs, balanced only where predicted faster).  Same outputs as
    fli_scan, bit for bit."""
    ld = _state(y0)
    n = ld if n is None else n
    integ = integrator_struct(integrator)
    corr = correction_struct(correction)
    if isinstance(t_end, torch.Tensor):
        if t_end.numel() != 1:
            raise ValueError("fli_scan_balanced takes one end time for all orbits; "
                             "orbits of uneven length go to batch_scan")
        t_end = t_end.item()
    t_end = float(t_end)
    if out is None:
        nmax = int(-(-t_end // integ.h)) if t_end > 0 else 0
        out = scan_outputs(n, ld, y0.device, full=full, trace_every=trace_every, nsteps_max=nmax)
    if ws is None:
        sch = balanced_schedule(n, t_end, integrator, correction, slots)
        ws = balanced_workspace(sch["slots"], y0.device) if sch["launches"] > 0 else None
    so = _scan_out_struct(out)
    p, keep = params_struct(beta, chi1, chi2)
    st = lib().pn_fli_scan_balanced(ctypes.byref(model_struct(model)), p, ctypes.byref(integ), ctypes.byref(corr),
                                    ctypes.byref(fli_struct(fli)), ctypes.c_int64(n), _ptr(y0), ctypes.c_int64(ld),
                                    ctypes.c_double(t_end), ctypes.byref(so), ctypes.c_int64(slots),
                                    _ptr(ws) if ws is not None else None,
                                    ctypes.c_size_t(ws.numel() if ws is not None else 0), _stream(y0.device))
    _check("pn_fli_scan_balanced", st)
    return out


def batch_scan_pending(ws, n):
    """Orbits of a resumable scan not finished yet (synchronises the stream)."""
    pending = ctypes.c_int64(0)
    st = lib().pn_batch_scan_pending(_ptr(ws), ctypes.c_int64(n), ctypes.byref(pending), _stream(ws.device))
    _check("pn_batch_scan_pending", st)
    return int(pending.value)


def autotune_batch(y0, t_end, beta, chi1, chi2, model=None, integrator=None, correction=None, fli=None,
                   step_scale=0.01, n=None, ws=None, out=None):
    """Run the library's autotuner; returns (tuning dict, best trial ms)."""
    ld, n, integ, t_end, out, ws, p, keep = _batch_common(y0, t_end, beta, chi1, chi2, model, integrator,
                                                          correction, fli, out, n, True, 0, ws)
    best = Tuning()
    ms = ctypes.c_float(0.0)
    so = _scan_out_struct(out)
    st = lib().pn_autotune_batch(ctypes.byref(model_struct(model)), p, ctypes.byref(integ),
                                 ctypes.byref(correction_struct(correction)), ctypes.byref(fli_struct(fli)),
                                 ctypes.c_int64(n), _ptr(y0), ctypes.c_int64(ld), _ptr(t_end), ctypes.byref(so),
                                 ctypes.c_double(step_scale), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                 ctypes.byref(best), ctypes.byref(ms), _stream(y0.device))
    _check("pn_autotune_batch", st)
    return dict(block=best.block, waves_per_simd=best.waves_per_simd, chunk_steps=best.chunk_steps), ms.value


class BatchGraph:
    """A batch scan captured once into a HIP graph; replay() relaunches it on
    the current stream with the buffers it was created with."""

    def __init__(self, y0, t_end, beta, chi1, chi2, model=None, integrator=None, correction=None, fli=None,
                 out=None, n=None, full=True, tuning=None, ws=None):
        ld, n, integ, t_end, out, ws, p, keep = _batch_common(y0, t_end, beta, chi1, chi2, model, integrator,
                                                              correction, fli, out, n, full, 0, ws)
        self._keep = (y0, t_end, ws, keep)
        self.out = out
        tu = None
        if tuning is not None:
            tu = ctypes.byref(tuning if isinstance(tuning, Tuning) else tuning_struct(tuning))
        so = _scan_out_struct(out)
        g = ctypes.c_void_p()
        st = lib().pn_batch_graph_create(ctypes.byref(model_struct(model)), p, ctypes.byref(integ),
                                         ctypes.byref(correction_struct(correction)), ctypes.byref(fli_struct(fli)),
                                         ctypes.c_int64(n), _ptr(y0), ctypes.c_int64(ld), _ptr(t_end),
                                         ctypes.byref(so), tu, _ptr(ws), ctypes.c_size_t(ws.numel()),
                                         ctypes.byref(g))
        _check("pn_batch_graph_create", st)
        self._g = g
        self._device = y0.device

    def replay(self):
        _check("pn_graph_launch", lib().pn_graph_launch(self._g, _stream(self._device)))
        return self.out

    def close(self):
        if self._g:
            lib().pn_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Learned surrogate.
# ---------------------------------------------------------------------------
P4 = ctypes.c_void_p * 4


class Mlp(ctypes.Structure):
    _fields_ = [("w", P4), ("b", P4), ("wb", P4), ("mw", P4), ("vw", P4), ("mb", P4), ("vb", P4)]


LAYER_IN = (7, 256, 256, 256)
LAYER_OUT = (256, 256, 256, 2)


class Network:
    """Device buffers of the 7-256-256-256-2 network (torch tensors) and the
    C struct pointing at them.  Weights come from the caller (FP32 arrays of
    shape [out, in]); the bfloat16 copies are made by the library."""

    def __init__(self, weights, biases, device, training=True):
        f32 = dict(dtype=torch.float32, device=device)
        self.w = [torch.as_tensor(W, **f32).contiguous() for W in weights]
        self.b = [torch.as_tensor(b, **f32).contiguous() for b in biases]
        for l in range(4):
            _require(tuple(self.w[l].shape) == (LAYER_OUT[l], LAYER_IN[l]), f"layer {l} weights: wrong shape")
        self.wb = [torch.empty(W.shape, dtype=torch.int16, device=device) for W in self.w]
        z = (lambda t: torch.zeros_like(t)) if training else (lambda t: None)
        self.mw, self.vw = [z(W) for W in self.w], [z(W) for W in self.w]
        self.mb, self.vb = [z(b) for b in self.b], [z(b) for b in self.b]
        self.step = 0
        self.struct = Mlp(*[P4(*[(t.data_ptr() if t is not None else None) for t in ts])
                            for ts in (self.w, self.b, self.wb, self.mw, self.vw, self.mb, self.vb)])
        _check("pn_mlp_sync_bf16", lib().pn_mlp_sync_bf16(ctypes.byref(self.struct), _stream(device)))

    def params(self):
        return [(W.detach().cpu().double().numpy(), b.detach().cpu().double().numpy())
                for W, b in zip(self.w, self.b)]


def mlp_features(n, r0, th1, th2, t_end, beta, chi1, chi2, mean, std, idx=None, out=None):
    """Standardised features [n, 8] (FP32) of scan points."""
    dev_ = r0.device
    if out is None:
        out = torch.empty((n, 8), dtype=torch.float32, device=dev_)
    p, keep = params_struct(beta, chi1, chi2)
    mean = (ctypes.c_float * 7)(*[float(x) for x in mean])
    std = (ctypes.c_float * 7)(*[float(x) for x in std])
    if isinstance(t_end, torch.Tensor):
        tptr, tall = _ptr(_dev_f64(t_end)), 0.0
    else:
        tptr, tall = None, float(t_end)
    st = lib().pn_mlp_features(p, ctypes.c_int64(n), _ptr(_dev_f64(r0)), _ptr(_dev_f64(th1)), _ptr(_dev_f64(th2)),
                               tptr, ctypes.c_double(tall), _ptr(idx), mean, std, _ptr(out), _stream(dev_))
    _check("pn_mlp_features", st)
    return out


def _train_args(feat, label, target, order, loss):
    rows = _feat_rows(feat)
    _dev(label, torch.float32, "label", shape=(rows,))
    _dev(target, torch.float32, "target", shape=(rows,))
    _dev(order, torch.int32, "idx/order")       # its values must lie in [0, rows)
    _dev(loss, torch.float32, "loss", min_numel=1)


def mlp_train_step(net, feat, label, target, idx, lr, loss, ws=None):
    _train_args(feat, label, target, idx, loss)
    batch = idx.numel()
    need = int(lib().pn_mlp_train_workspace_size(batch))
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=feat.device)
    _dev(ws, torch.uint8, "ws", min_numel=need)
    net.step += 1
    st = lib().pn_mlp_train_step(ctypes.byref(net.struct), _ptr(feat), _ptr(label), _ptr(target), _ptr(idx),
                                 ctypes.c_int32(batch), ctypes.c_int32(net.step), ctypes.c_float(lr), _ptr(loss),
                                 _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(feat.device))
    _check("pn_mlp_train_step", st)
    return ws


def mlp_train_workspace_layout(batch):
    """Byte offsets of (X, h1, h2, h3, out, g4, g3, g2, g1) in a training-step
    workspace (pn_mlp_train_workspace_layout)."""
    off = (ctypes.c_size_t * 9)()
    _check("pn_mlp_train_workspace_layout", lib().pn_mlp_train_workspace_layout(ctypes.c_int32(batch), off))
    return list(off)


def mlp_train_step_tensors(ws, batch):
    """Views of the tensors a completed training step left in its workspace:
    dict X, h1, h2, h3 (bfloat16 bit patterns, int16), out (float32), g4, g3,
    g2, g1 (int16)."""
    off = mlp_train_workspace_layout(batch)
    spec = [("X", 8, 2), ("h1", 256, 2), ("h2", 256, 2), ("h3", 256, 2), ("out", 2, 4), ("g4", 2, 2),
            ("g3", 256, 2), ("g2", 256, 2), ("g1", 256, 2)]
    res = {}
    for (name, cols, size), o in zip(spec, off):
        raw = ws[o:o + batch * cols * size]
        res[name] = (raw.view(torch.float32) if size == 4 else raw.view(torch.int16)).view(batch, cols)
    return res


def mlp_train(net, feat, label, target, order, batch, lr, loss, ws=None):
    """pn_mlp_train: len(order) // batch steps over the rows in `order` (device
    int32), advancing net.step; returns the workspace."""
    _train_args(feat, label, target, order, loss)
    nbatch = order.numel() // batch
    need = int(lib().pn_mlp_train_workspace_size(batch))
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=feat.device)
    _dev(ws, torch.uint8, "ws", min_numel=need)
    step = ctypes.c_int32(net.step)
    st = lib().pn_mlp_train(ctypes.byref(net.struct), ctypes.byref(step), _ptr(feat), _ptr(label), _ptr(target),
                            _ptr(order), ctypes.c_int64(nbatch), ctypes.c_int32(batch), ctypes.c_float(lr), _ptr(loss),
                            _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(feat.device))
    net.step = step.value
    _check("pn_mlp_train", st)
    return ws


def mlp_infer(net, feat, chunk=1 << 20, out=None, ws=None):
    n = _feat_rows(feat)
    if out is None:
        out = torch.empty((n, 2), dtype=torch.float32, device=feat.device)
    _dev(out, torch.float32, "out", shape=(n, 2))
    chunk = max(1, min(chunk, n))
    need = int(lib().pn_mlp_infer_workspace_size(chunk))
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=feat.device)
    _dev(ws, torch.uint8, "ws", min_numel=need)
    st = lib().pn_mlp_infer(ctypes.byref(net.struct), _ptr(feat), ctypes.c_int64(n), _ptr(out), ctypes.c_int64(chunk),
                            _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(feat.device))
    _check("pn_mlp_infer", st)
    return out


def mlp_infer_fused(net, feat, out=None):
    """pn_mlp_infer_fused: all four layers in one kernel; same bits as mlp_infer for finite features."""
    n = _feat_rows(feat)
    if out is None:
        out = torch.empty((n, 2), dtype=torch.float32, device=feat.device)
    _dev(out, torch.float32, "out", shape=(n, 2))
    st = lib().pn_mlp_infer_fused(ctypes.byref(net.struct), _ptr(feat), ctypes.c_int64(n), _ptr(out),
                                  _stream(feat.device))
    _check("pn_mlp_infer_fused", st)
    return out


def surrogate_cfg(over=None):
    s = SurrogateCfg()
    lib().pn_default_surrogate_cfg(ctypes.byref(s))
    for k, v in (over or {}).items():
        setattr(s, k, v)
    return s


def surrogate_scan(net, n, r0, p0, th1, ph1, th2, ph2, t_end, beta, chi1, chi2, mean, std, cfg=None, model=None,
                   integrator=None, correction=None, fli=None, ws=None):
    """pn_surrogate_scan: dict(label int8 [n], integrated, points int32 [integrated],
    phase_ms [audit, refine, infer+gate, fallback], scans (per integration, audit
    then fallback: kernel name, launches, points, orbit_steps, ms of the scan
    launches alone), ws).  The network is refined in place (net.step counts its
    Adam steps)."""
    dev_ = r0.device
    c = surrogate_cfg(cfg)
    need = int(lib().pn_surrogate_scan_workspace_size(n, c.refine_batch))
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev_)
    label = torch.empty(max(n, 1), dtype=torch.int8, device=dev_)
    points = torch.empty(max(n, 1), dtype=torch.int32, device=dev_)
    stats = SurrogateStats()
    p, keep = params_struct(beta, chi1, chi2)
    mean = (ctypes.c_float * 7)(*[float(x) for x in mean])
    std = (ctypes.c_float * 7)(*[float(x) for x in std])
    if isinstance(t_end, torch.Tensor):
        tptr, tall = _ptr(_dev_f64(t_end)), 0.0
    else:
        tptr, tall = None, float(t_end)
    cols = [_dev_f64(t) for t in (r0, p0, th1, ph1, th2, ph2)]
    step = ctypes.c_int32(net.step)
    integrated = ctypes.c_int64(0)
    st = lib().pn_surrogate_scan(ctypes.byref(net.struct), ctypes.byref(step), ctypes.byref(model_struct(model)), p,
                                 ctypes.byref(integrator_struct(integrator)),
                                 ctypes.byref(correction_struct(correction)), ctypes.byref(fli_struct(fli)),
                                 ctypes.c_int64(n), *[_ptr(t) for t in cols], tptr, ctypes.c_double(tall), mean, std,
                                 ctypes.byref(c), _ptr(label), _ptr(points), ctypes.byref(integrated), ctypes.byref(stats),
                                 _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(dev_))
    _check("pn_surrogate_scan", st)
    net.step = step.value
    m = integrated.value
    scans = [dict(kernel=SCAN_KERNELS[stats.scan_kernel[k]], launches=stats.scan_launches[k],
                  points=stats.points[k], orbit_steps=stats.orbit_steps[k], ms=stats.scan_ms[k]) for k in range(2)]
    return dict(label=label[:n], integrated=m, points=points[:m], phase_ms=list(stats.phase_ms), scans=scans, ws=ws)


def surrogate_gate(out, margin, audit_frac, seed):
    """Returns (labels int8 [n], predicted FLI - log10 t [n], list int32, count)."""
    n = out.shape[0]
    dev_ = out.device
    label = torch.empty(n, dtype=torch.int8, device=dev_)
    fli = torch.empty(n, dtype=torch.float32, device=dev_)
    lst = torch.empty(max(n, 1), dtype=torch.int32, device=dev_)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev_)
    st = lib().pn_surrogate_gate(_ptr(out), ctypes.c_int64(n), ctypes.c_float(margin), ctypes.c_double(audit_frac),
                                 ctypes.c_uint64(seed), _ptr(label), _ptr(fli), _ptr(lst), _ptr(cnt), _stream(dev_))
    _check("pn_surrogate_gate", st)
    m = int(cnt.item())
    return label, fli, lst[:m], m


def surrogate_merge(lst, integrated, label):
    st = lib().pn_surrogate_merge(_ptr(lst), ctypes.c_int64(lst.numel()), _ptr(integrated), _ptr(label),
                                  _stream(label.device))
    _check("pn_surrogate_merge", st)
    return label


def gemm_bf16(A, sam, sak, B, sbk, sbn, M, N, K, bias=None, relu=False, mask=None, ldm=0, out_f32=True,
              out_bf16=False):
    """Test access to the matrix-core product (A, B: int16 bit patterns of bfloat16)."""
    dev_ = A.device
    Cf = torch.empty((M, N), dtype=torch.float32, device=dev_) if out_f32 else None
    Cb = torch.empty((M, N), dtype=torch.int16, device=dev_) if out_bf16 else None
    st = lib().pn_gemm_bf16(ctypes.c_int32(M), ctypes.c_int32(N), ctypes.c_int32(K), _ptr(A), ctypes.c_int64(sam),
                            ctypes.c_int64(sak), _ptr(B), ctypes.c_int64(sbk), ctypes.c_int64(sbn), _ptr(bias),
                            ctypes.c_int32(int(relu)), _ptr(mask), ctypes.c_int64(ldm), _ptr(Cf),
                            ctypes.c_int64(N), _ptr(Cb), ctypes.c_int64(N), _stream(dev_))
    _check("pn_gemm_bf16", st)
    return Cf, Cb


def init_state_gather(idx, r0, p0, th1, ph1, th2, ph2, beta, chi1, chi2, model=None):
    m = idx.numel()
    y0 = torch.empty((12, max(m, 1)), dtype=torch.float64, device=idx.device)
    p, keep = params_struct(beta, chi1, chi2)
    cols = [_dev_f64(t) for t in (r0, p0, th1, ph1, th2, ph2)]
    st = lib().pn_init_state_gather(ctypes.byref(model_struct(model)), p, ctypes.c_int64(m), _ptr(idx),
                                    *[_ptr(c) for c in cols], _ptr(y0), ctypes.c_int64(max(m, 1)),
                                    _stream(idx.device))
    _check("pn_init_state_gather", st)
    return y0


def mlp_targets(fli, label, t_end):
    """(label 1/0, FLI - log10 t_end) as FP32 device arrays from scan outputs."""
    n = fli.numel()
    lab = torch.empty(n, dtype=torch.float32, device=fli.device)
    tgt = torch.empty(n, dtype=torch.float32, device=fli.device)
    if isinstance(t_end, torch.Tensor):
        tptr, tall = _ptr(_dev_f64(t_end)), 0.0
    else:
        tptr, tall = None, float(t_end)
    st = lib().pn_mlp_targets(_ptr(fli), _ptr(label), tptr, ctypes.c_double(tall), ctypes.c_int64(n), _ptr(lab),
                              _ptr(tgt), _stream(fli.device))
    _check("pn_mlp_targets", st)
    return lab, tgt
