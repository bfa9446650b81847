"""The paper's own spin-angle scans (Sec. 3C, Figs. 6-7, Table 3) on the
oracle: the input states the paper prints, checked against closed forms.

* Fig. 6 prints (beta, r, p_y) = (1/3, 5.65, 0.765).  Its Newtonian energy
  p^2/2 - 1/r = +0.116 is positive and so is the orbital (2PN) part of H; the
  spin terms (|S_2| = 3 in units of mu M at beta = 1/3) lower H below zero
  only when the second spin tilts far from the orbital axis.  The bound part
  of the line is therefore a single interval of large theta2, where the
  paper places its chaotic orbits; the rest is removed as unbound.
* Fig. 7's state (r, p_y) = (10.14, 0.365) with beta = 1 (orbit 2, Sec. 3A)
  is bound for every (theta1, theta2) of the plane; its Newtonian eccentricity
  p^2 r - 1 = 0.351 is the 0.37 the paper quotes for orbit 2 up to PN terms.
"""
import numpy as np

from paper_1802_00147_amd import workloads as W


def _states(O, wl, model=None):
    return O.init_state(wl.r0, wl.p0, wl.th1, wl.ph1, wl.th2, wl.ph2, wl.beta, wl.chi1, wl.chi2, model=model)


def test_fig6_printed_state_bound_only_at_large_theta2(oracle):
    beta, r, p = W.FIG6_STATE
    assert p * p / 2 - 1 / r > 0.1                     # Newtonian energy, closed form
    for th1, first in ((np.pi / 2, 2.21), (0.0, 2.51)):   # panels (a) and (b)
        wl = W.fig6(th1)
        assert wl.n == 314 and np.isclose(wl.th2[-1], 3.13)
        y0 = _states(oracle, wl)
        H, _ = oracle.invariants(y0, wl.beta, wl.chi1, wl.chi2)
        bound = H < 0
        k = np.argmax(bound)
        assert np.all(bound[k:]) and not np.any(bound[:k])   # one interval at the end of the line
        assert np.isclose(wl.th2[k], first)
        # Without spins the same orbital state is unbound.
        y_ns = y0.copy()
        y_ns[:, 6:] = 0.0
        H_ns, _ = oracle.invariants(y_ns, wl.beta, wl.chi1, wl.chi2)
        assert np.all(H_ns > 0.01)
        # The scan removes exactly the unbound states (short run: statuses only).
        out = oracle.fli_scan(y0, 10.0, wl.beta, wl.chi1, wl.chi2, nthreads=8)
        assert np.array_equal(out["status"] == oracle.STATUS_UNBOUND_INIT, ~bound)
        assert np.all(out["label"][~bound] == -1) and np.all(np.isnan(out["fli"][~bound]))


def test_fig7_plane_is_bound(oracle):
    beta, r, p = W.FIG7_STATE
    assert abs(p * p * r - 1 - 0.351) < 1e-3         # Newtonian eccentricity of orbit 2
    wl = W.fig7()
    assert wl.n == 314 * 314 and wl.shape == (314, 314)
    idx = W.strided_sample(wl.n, 2000, seed=3)
    sub = wl.subset(idx)
    y0 = _states(oracle, sub)
    H, J = oracle.invariants(y0, sub.beta, sub.chi1, sub.chi2)
    assert np.all(H < -0.01)
    # Spin lengths chi m_i^2 / (mu M) with beta = 1: |S_i| = 1.
    assert np.allclose(np.linalg.norm(y0[:, 6:9], axis=1), 1.0, rtol=0, atol=1e-15)
    assert np.allclose(np.linalg.norm(y0[:, 9:12], axis=1), 1.0, rtol=0, atol=1e-15)
    # theta1 = theta2 = 0 puts both spins along z: J_z = L + 2, J_x = J_y = 0.
    y00 = _states(oracle, wl.subset([0]))
    _, J0 = oracle.invariants(y00, 1.0, 1.0, 1.0)
    assert np.allclose(J0[0], [0.0, 0.0, r * p + 2.0], rtol=0, atol=1e-14)
