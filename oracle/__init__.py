"""CPU FP64 oracle for the manifold-corrected PN spinning-binary FLI scan.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it to judge and time the GPU library.  Nothing in the
product path imports it, and it imports nothing from the product.

Arrays use the natural serial layout: one state is 12 consecutive doubles
(r, p, S1, S2), shape (n, 12).  Settings are plain dicts; missing keys take
the defaults below.  Every computation runs in pn_oracle.cpp (plain serial
C++ compiled without contraction); this module only marshals arguments.

Parity unpinned: none of the functions here -- each is pinned by a test in
tests/test_oracle_*.py against a closed form, the paper's printed equations,
an invariant, or brute force.
"""
import ctypes
import os

import numpy as np

from .build import LIB, ensure_built

MODEL = dict(pn_order=2, spin_orbit=1, spin_spin=1, quad_mono=1, spin_units=0, rad_reaction=0)
INTEGRATOR = dict(method=0, h=1.0)
CORRECTION = dict(mode=2, tol=1e-10, max_iter=20, sweeps=2, w1=1.0, w2=1.0)
FLI = dict(d0=1e-8, d_renorm=0.1, shadow_axis=0, thr_at_1e5=5.8, thr_scaling=1,
           r_merge=2.0, r_esc=1e3)

METHODS = {"rk4": 0, "rk5": 1}
MODES = {"none": 0, "spin": 1, "six": 2, "dual": 3}
STATUS_OK, STATUS_MERGED, STATUS_ESCAPED, STATUS_NONFINITE, STATUS_UNBOUND_INIT, STATUS_BADPARAM = range(6)
STATUS_NEWTON_NOCONV = 0x100


class _Model(ctypes.Structure):
    _fields_ = [("pn_order", ctypes.c_int32), ("spin_orbit", ctypes.c_int32),
                ("spin_spin", ctypes.c_int32), ("quad_mono", ctypes.c_int32),
                ("spin_units", ctypes.c_int32), ("rad_reaction", ctypes.c_int32)]


class _Integrator(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("h", ctypes.c_double)]


class _Correction(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("sweeps", ctypes.c_int32), ("w1", ctypes.c_double), ("w2", ctypes.c_double)]


class _Fli(ctypes.Structure):
    _fields_ = [("d0", ctypes.c_double), ("d_renorm", ctypes.c_double),
                ("shadow_axis", ctypes.c_int32), ("thr_at_1e5", ctypes.c_double),
                ("thr_scaling", ctypes.c_int32), ("r_merge", ctypes.c_double),
                ("r_esc", ctypes.c_double)]


_lib = None


def lib():
    """The oracle library; PN_ORACLE_LIB names another build of the same
    source (the sanitizer check loads an instrumented one)."""
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(os.environ.get("PN_ORACLE_LIB") or ensure_built())
    return _lib


def _fill(struct, defaults, over):
    d = dict(defaults)
    if over:
        unknown = set(over) - set(d)
        if unknown:
            raise KeyError(f"unknown settings {sorted(unknown)}")
        d.update(over)
    if struct is _Integrator and isinstance(d["method"], str):
        d["method"] = METHODS[d["method"]]
    if struct is _Correction and isinstance(d["mode"], str):
        d["mode"] = MODES[d["mode"]]
    return struct(**d)


def _p(a, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct)) if a is not None else None


def _states(y):
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64))
    if y.ndim == 1:
        y = y.reshape(1, 12)
    assert y.shape[1] == 12
    return y


def _params(n, beta, chi1, chi2):
    """Return contiguous parameter arrays and their stride (0 = broadcast)."""
    b, c1, c2 = (np.atleast_1d(np.asarray(v, dtype=np.float64)) for v in (beta, chi1, chi2))
    if b.size == 1 and c1.size == 1 and c2.size == 1:
        return b.copy(), c1.copy(), c2.copy(), 0
    b, c1, c2 = (np.ascontiguousarray(np.broadcast_to(v, (n,)), dtype=np.float64)
                 for v in (b, c1, c2))
    return b, c1, c2, 1


def coefficients(beta, chi1, chi2, model=None):
    """[eta, cso1, cso2, c12, c11, c22, s1, s2] for one parameter set."""
    out = np.zeros(8)
    lib().or_coefficients(ctypes.byref(_fill(_Model, MODEL, model)), ctypes.c_double(beta),
                          ctypes.c_double(chi1), ctypes.c_double(chi2), _p(out))
    return out


def hamiltonian(y, beta, chi1, chi2, model=None):
    y = _states(y)
    H = np.zeros(len(y))
    lib().or_hamiltonian(ctypes.byref(_fill(_Model, MODEL, model)), ctypes.c_double(beta),
                         ctypes.c_double(chi1), ctypes.c_double(chi2),
                         ctypes.c_int64(len(y)), _p(y), _p(H))
    return H


def gradient(y, beta, chi1, chi2, model=None):
    """Analytic (dH/dr, dH/dp, dH/dS1, dH/dS2), shape (n, 12)."""
    y = _states(y)
    g = np.zeros_like(y)
    lib().or_gradient(ctypes.byref(_fill(_Model, MODEL, model)), ctypes.c_double(beta),
                      ctypes.c_double(chi1), ctypes.c_double(chi2),
                      ctypes.c_int64(len(y)), _p(y), _p(g))
    return g


def gradient_complex_step(y, beta, chi1, chi2, model=None, delta=1e-30):
    y = _states(y)
    g = np.zeros_like(y)
    lib().or_gradient_complex_step(ctypes.byref(_fill(_Model, MODEL, model)), ctypes.c_double(beta),
                                   ctypes.c_double(chi1), ctypes.c_double(chi2),
                                   ctypes.c_int64(len(y)), _p(y), ctypes.c_double(delta), _p(g))
    return g


def rhs(y, beta, chi1, chi2, model=None):
    y = _states(y)
    b, c1, c2, s = _params(len(y), beta, chi1, chi2)
    d = np.zeros_like(y)
    lib().or_rhs(ctypes.byref(_fill(_Model, MODEL, model)), _p(b), _p(c1), _p(c2),
                 ctypes.c_int64(s), ctypes.c_int64(len(y)), _p(y), _p(d))
    return d


def invariants(y, beta, chi1, chi2, model=None):
    """Return (H[n], J[n,3])."""
    y = _states(y)
    b, c1, c2, s = _params(len(y), beta, chi1, chi2)
    out = np.zeros((len(y), 4))
    lib().or_invariants(ctypes.byref(_fill(_Model, MODEL, model)), _p(b), _p(c1), _p(c2),
                        ctypes.c_int64(s), ctypes.c_int64(len(y)), _p(y), _p(out))
    return out[:, 0].copy(), out[:, 1:].copy()


def gw_polarizations(y, beta, chi1, chi2, N, p, dist=1.0, model=None):
    """(h_plus[n], h_cross[n]) of eq. (14) for n states, observer direction N
    and line of nodes p (unit, orthogonal), distance dist in units of M."""
    y = _states(y)
    b, c1, c2, s = _params(len(y), beta, chi1, chi2)
    N = np.ascontiguousarray(N, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros((len(y), 2))
    lib().or_gw_polarizations(ctypes.byref(_fill(_Model, MODEL, model)), _p(b), _p(c1), _p(c2),
                              ctypes.c_int64(s), ctypes.c_int64(len(y)), _p(y), _p(N), _p(p),
                              ctypes.c_double(dist), _p(out))
    return out[:, 0].copy(), out[:, 1].copy()


def init_state(r0, p0, th1, ph1, th2, ph2, beta, chi1, chi2, model=None):
    r0 = np.ascontiguousarray(np.atleast_1d(r0), dtype=np.float64)
    n = len(r0)
    cols = [np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)))
            for v in (p0, th1, ph1, th2, ph2)]
    b, c1, c2, s = _params(n, beta, chi1, chi2)
    y = np.zeros((n, 12))
    lib().or_init_state(ctypes.byref(_fill(_Model, MODEL, model)), _p(b), _p(c1), _p(c2),
                        ctypes.c_int64(s), ctypes.c_int64(n), _p(r0), *[_p(c) for c in cols], _p(y))
    return y


def manifold_correct(y, ref, beta, chi1, chi2, model=None, correction=None):
    """Correct copies of the states against ref (n, 4) = (E0, J0); return (y, iters)."""
    y = _states(y).copy()
    ref = np.ascontiguousarray(np.asarray(ref, dtype=np.float64).reshape(len(y), 4))
    b, c1, c2, s = _params(len(y), beta, chi1, chi2)
    it = np.zeros(len(y), dtype=np.int32)
    lib().or_manifold_correct(ctypes.byref(_fill(_Model, MODEL, model)), _p(b), _p(c1), _p(c2),
                              ctypes.c_int64(s), ctypes.byref(_fill(_Correction, CORRECTION, correction)),
                              ctypes.c_int64(len(y)), _p(y), _p(ref), _p(it, ctypes.c_int32))
    return y, it


def step(y, beta, chi1, chi2, nsteps, model=None, integrator=None, correction=None, ref=None, return_ref=False):
    """nsteps RK (+ correction unless correction is None) steps of copies of the states.
    With radiation reaction the references (n, 4) advance with the states;
    return_ref=True also returns them (a copy of ref when it was given)."""
    y = _states(y).copy()
    b, c1, c2, s = _params(len(y), beta, chi1, chi2)
    cc = ctypes.byref(_fill(_Correction, CORRECTION, correction)) if correction is not None else None
    r = None
    if ref is not None:
        r = np.array(np.asarray(ref, dtype=np.float64).reshape(len(y), 4), copy=True)
    lib().or_step(ctypes.byref(_fill(_Model, MODEL, model)), _p(b), _p(c1), _p(c2), ctypes.c_int64(s),
                  ctypes.byref(_fill(_Integrator, INTEGRATOR, integrator)), cc,
                  ctypes.c_int64(len(y)), _p(y), _p(r), ctypes.c_int64(nsteps))
    return (y, r) if return_ref else y


def rk_linear_step(method, z):
    f = lib().or_rk_linear_step
    f.restype = ctypes.c_double
    m = METHODS[method] if isinstance(method, str) else method
    return f(ctypes.c_int32(m), ctypes.c_double(z))


def fli_scan(y0, t_end, beta, chi1, chi2, model=None, integrator=None, correction=None, fli=None,
             nthreads=1, trace_every=0):
    """Full FLI runs.  Returns a dict of per-orbit arrays."""
    y0 = _states(y0)
    n = len(y0)
    b, c1, c2, s = _params(n, beta, chi1, chi2)
    t = np.atleast_1d(np.asarray(t_end, dtype=np.float64))
    ts = 0 if t.size == 1 else 1
    t = np.ascontiguousarray(t)
    integ = _fill(_Integrator, INTEGRATOR, integrator)
    out = dict(fli=np.zeros(n), label=np.zeros(n, np.int8), status=np.zeros(n, np.int32),
               y_final=np.zeros((n, 12)), dH=np.zeros(n), dJ=np.zeros(n),
               newton_max=np.zeros(n, np.int32), renorms=np.zeros(n, np.int64),
               steps=np.zeros(n, np.int64))
    ntrace = 0
    trace = None
    if trace_every > 0:
        ntrace = int(np.ceil(t.max() / integ.h)) // trace_every
        trace = np.full((n, ntrace), np.nan)
    lib().or_fli_scan(ctypes.byref(_fill(_Model, MODEL, model)), _p(b), _p(c1), _p(c2),
                      ctypes.c_int64(s), ctypes.byref(integ),
                      ctypes.byref(_fill(_Correction, CORRECTION, correction)),
                      ctypes.byref(_fill(_Fli, FLI, fli)), ctypes.c_int64(n), _p(y0), _p(t),
                      ctypes.c_int64(ts), _p(out["fli"]), _p(out["label"], ctypes.c_int8),
                      _p(out["status"], ctypes.c_int32), _p(out["y_final"]), _p(out["dH"]),
                      _p(out["dJ"]), _p(out["newton_max"], ctypes.c_int32),
                      _p(out["renorms"], ctypes.c_int64), _p(out["steps"], ctypes.c_int64), _p(trace),
                      ctypes.c_int64(trace_every),
                      ctypes.c_int64(ntrace), ctypes.c_int32(nthreads))
    if trace is not None:
        out["trace"] = trace
    return out


def count_flops(y0, t_end, beta, chi1, chi2, model=None, integrator=None, correction=None, fli=None):
    """Algorithmic flop counts of one orbit's run (counting scalar).

    Returns dict(rhs, rk_step, correction, run_total, steps, newton_total, renorms).
    """
    y0 = _states(y0)[0].copy()
    out = np.zeros(7)
    lib().or_count_flops(ctypes.byref(_fill(_Model, MODEL, model)), ctypes.c_double(beta),
                         ctypes.c_double(chi1), ctypes.c_double(chi2),
                         ctypes.byref(_fill(_Integrator, INTEGRATOR, integrator)),
                         ctypes.byref(_fill(_Correction, CORRECTION, correction)),
                         ctypes.byref(_fill(_Fli, FLI, fli)), _p(y0), ctypes.c_double(t_end), _p(out))
    keys = ["rhs", "rk_step", "correction", "run_total", "steps", "newton_total", "renorms"]
    return dict(zip(keys, out.tolist()))
