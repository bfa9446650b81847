"""Runs every entry point of the CPU oracle on small inputs, including its
removal and error branches, so that an instrumented build (AddressSanitizer +
UndefinedBehaviorSanitizer, loaded through PN_ORACLE_LIB) can report any
invalid access or undefined operation.  Started by
test_oracle_sanitized.py in a process of its own; prints "driver ok" at the
end.  numpy only (no torch), so the preloaded runtime sees a small process.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402


def states(seed, n):
    rng = np.random.default_rng(seed)
    r0 = rng.uniform(8.0, 30.0, n)
    return O.init_state(r0, r0 ** -0.5, rng.uniform(0, np.pi, n), rng.uniform(0, 2 * np.pi, n),
                        rng.uniform(0, np.pi, n), rng.uniform(0, 2 * np.pi, n), 0.7, 0.8, 0.9)


def main():
    y = states(1, 6)
    beta = np.array([1.0, 0.5, 0.3, 1.0, 0.8, 0.6])
    chi = np.array([1.0, 0.0, 0.5, 0.9, 0.2, 1.0])
    for model in (None, dict(pn_order=0, spin_orbit=0, spin_spin=0, quad_mono=0), dict(spin_units=1),
                  dict(pn_order=1, quad_mono=0)):
        O.coefficients(0.5, 0.6, 0.7, model=model)
        O.hamiltonian(y, 0.5, 0.6, 0.7, model=model)
        O.gradient(y, 0.5, 0.6, 0.7, model=model)
        O.gradient_complex_step(y, 0.5, 0.6, 0.7, model=model)
        O.rhs(y, beta, chi, chi, model=model)
        O.invariants(y, beta, chi, chi, model=model)
    for mode in ("none", "spin", "six", "dual"):
        corr = dict(mode=O.MODES[mode])
        for method in (0, 1):
            yy = O.step(y, 1.0, 1.0, 1.0, 5, integrator=dict(method=method), correction=corr)
            assert np.all(np.isfinite(yy))
        O.step(y, 1.0, 1.0, 1.0, 3, correction=None)
    y2 = O.step(y, 1.0, 1.0, 1.0, 3, correction=None)
    H0, J0 = O.invariants(y, 1.0, 1.0, 1.0)
    refs = np.column_stack([H0, J0])
    for mode in ("none", "spin", "six", "dual"):
        yc, it = O.manifold_correct(y2, refs, 1.0, 1.0, 1.0, correction=dict(mode=O.MODES[mode]))
        assert np.all(np.isfinite(yc))
    O.step(y, 1.0, 1.0, 1.0, 4, ref=refs)
    # The dissipative system: references advanced and written back, both
    # integrators, and a scan refusing it.
    for method in (0, 1):
        yr, rr = O.step(y, 1.0, 1.0, 1.0, 20, model=dict(rad_reaction=1), integrator=dict(method=method),
                        correction=dict(mode=2), ref=refs, return_ref=True)
        assert np.all(np.isfinite(yr)) and np.all(np.isfinite(rr))
    O.step(y, 1.0, 1.0, 1.0, 5, model=dict(rad_reaction=1), correction=dict(mode=3))
    O.rhs(y, beta, chi, chi, model=dict(rad_reaction=1))
    assert O.fli_scan(y, 10.0, 1.0, 1.0, 1.0, model=dict(rad_reaction=1))["status"][0] == O.STATUS_BADPARAM
    for method in ("rk4", "rk5"):
        O.rk_linear_step(method, -0.5)
    O.gw_polarizations(y, 1.0, 1.0, 1.0, np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0]), dist=10.0)
    # Scans: every status (unbound, plunge, escape, non-finite, bad parameter,
    # zero time), a trace, per-orbit end times, both integrators, all modes,
    # a forced Newton non-convergence, several threads.
    rows = []
    z = np.zeros(12); z[0], z[4] = 10.0, 0.6; rows.append(z)
    z = np.zeros(12); z[0], z[4] = 6.0, 0.05; rows.append(z)
    z = np.zeros(12); z[0], z[4] = 10.0, 0.4; rows.append(z)
    z = np.zeros(12); z[0], z[4] = 10.0, np.nan; rows.append(z)
    z = np.zeros(12); z[0], z[4] = 8.0, 8 ** -0.5; rows.append(z)
    z = np.zeros(12); z[0], z[4] = 8.0, 8 ** -0.5; rows.append(z)
    y0 = np.vstack([np.array(rows), states(2, 4)])
    b = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.7, 1.0, 0.5, 0.9, 1.0])
    c = np.zeros(10)
    t = np.array([300.0, 300.0, 300.0, 300.0, 300.0, 300.0, 0.0, 120.5, 200.0, 300.0])
    out = O.fli_scan(y0, t, b, c, c, fli=dict(r_esc=11.0), nthreads=3, trace_every=50)
    assert out["status"][5] == O.STATUS_BADPARAM
    for mode in ("none", "spin", "dual"):
        for method in (0, 1):
            O.fli_scan(y0[6:], 100.0, 1.0, 1.0, 1.0, integrator=dict(method=method),
                       correction=dict(mode=O.MODES[mode]), nthreads=2)
    forced = O.fli_scan(y0[6:], 50.0, 1.0, 1.0, 1.0, correction=dict(max_iter=1, tol=1e-300))
    assert np.all(forced["status"] & O.STATUS_NEWTON_NOCONV)
    O.count_flops(y0[6], 200.0, 1.0, 1.0, 1.0)
    O.count_flops(y0[6], 100.0, 1.0, 1.0, 1.0, integrator=dict(method=1), correction=dict(mode=3))
    print("driver ok", flush=True)


if __name__ == "__main__":
    main()
