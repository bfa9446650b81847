"""Pins of the oracle's gravitational-wave polarisations (Sec. 4, eq. 14),
each against mathematics the oracle's code does not contain.

* Newtonian circular orbit seen face-on (N = z, p = x, q = y): the quadrupole
  field is h_plus = -(4 eta M / (D r)) cos 2phi, h_cross = -(4 eta M / (D r))
  sin 2phi at orbital phase phi (v = r omega (-sin phi, cos phi, 0),
  omega^2 = M / r^3): amplitude, twice the orbital frequency and phase.
* The same orbit seen edge-on (N = x, p = y, q = z): h_cross = 0 and
  h_plus = (2 eta M / (D r)) cos 2phi, half the face-on amplitude.
* Spin-2 behaviour: turning p and q by psi about N turns (h_plus, h_cross)
  by 2 psi, for any state (PN terms and spins included).
* 1/D scaling, and eta = beta / (1 + beta)^2 in the amplitude.
"""
import numpy as np
import pytest

NEWTON = dict(pn_order=0, spin_orbit=0, spin_spin=0, quad_mono=0)


def circular_states(r, phis):
    v = r ** -0.5
    y = np.zeros((len(phis), 12))
    y[:, 0], y[:, 1] = r * np.cos(phis), r * np.sin(phis)
    y[:, 3], y[:, 4] = -v * np.sin(phis), v * np.cos(phis)
    return y


@pytest.mark.parametrize("beta", [1.0, 0.25])
def test_face_on_circular_closed_form(oracle, beta):
    r, D = 17.0, 250.0
    eta = beta / (1 + beta) ** 2
    phis = np.linspace(0, 2 * np.pi, 37)
    hp, hx = oracle.gw_polarizations(circular_states(r, phis), beta, 0.0, 0.0, [0, 0, 1], [1, 0, 0], D, NEWTON)
    amp = 4 * eta / (D * r)
    assert np.allclose(hp, -amp * np.cos(2 * phis), rtol=0, atol=1e-14 * amp)
    assert np.allclose(hx, -amp * np.sin(2 * phis), rtol=0, atol=1e-14 * amp)


def test_edge_on_circular_closed_form(oracle):
    # N = x, p = y, q = N x p = z.  h_cross = h_yz = 0; h_plus = (h_yy - h_zz) / 2
    # = (2 eta / D) (v_y^2 - n_y^2 / r) = (2 eta / (D r)) (cos^2 phi - sin^2 phi)
    # = (2 eta / (D r)) cos 2phi.
    r, D, beta = 12.0, 1.0, 1.0
    eta = 0.25
    phis = np.linspace(0, 2 * np.pi, 29)
    hp, hx = oracle.gw_polarizations(circular_states(r, phis), beta, 0.0, 0.0, [1, 0, 0], [0, 1, 0], D, NEWTON)
    assert np.allclose(hx, 0.0, atol=1e-16)
    assert np.allclose(hp, 2 * eta / (D * r) * np.cos(2 * phis), rtol=0, atol=1e-14)


def test_spin2_rotation_and_distance(oracle):
    rng = np.random.default_rng(3)
    y = np.zeros((16, 12))
    y[:, 0:3] = rng.normal(size=(16, 3)) * 15
    y[:, 3:6] = rng.normal(size=(16, 3)) * 0.2
    y[:, 6:12] = rng.normal(size=(16, 6)) * 0.4
    N = np.array([0.3, -0.5, 0.8])
    N /= np.linalg.norm(N)
    p = np.cross(N, [1.0, 0.0, 0.0])
    p /= np.linalg.norm(p)
    q = np.cross(N, p)
    hp, hx = oracle.gw_polarizations(y, 0.6, 0.9, 0.7, N, p, 100.0)
    for psi in (0.3, 1.1, -2.0):
        p2 = np.cos(psi) * p + np.sin(psi) * q
        hp2, hx2 = oracle.gw_polarizations(y, 0.6, 0.9, 0.7, N, p2, 100.0)
        c, s = np.cos(2 * psi), np.sin(2 * psi)
        scale = np.abs(hp).max() + np.abs(hx).max()
        assert np.allclose(hp2, c * hp + s * hx, rtol=0, atol=1e-13 * scale)
        assert np.allclose(hx2, -s * hp + c * hx, rtol=0, atol=1e-13 * scale)
    hp3, hx3 = oracle.gw_polarizations(y, 0.6, 0.9, 0.7, N, p, 25.0)
    assert np.allclose(hp3, 4 * hp, rtol=1e-14) and np.allclose(hx3, 4 * hx, rtol=1e-14)


def test_velocity_is_the_hamiltonian_flow(oracle):
    # With the PN terms on, v = dH/dp differs from p; the polarisations must
    # follow dr/dt of the oracle's own equations of motion: compare with the
    # Newtonian-formula contraction built here from the oracle's rhs.
    rng = np.random.default_rng(5)
    y = np.zeros((8, 12))
    y[:, 0:3] = rng.normal(size=(8, 3)) * 10
    y[:, 3:6] = rng.normal(size=(8, 3)) * 0.25
    y[:, 6:12] = rng.normal(size=(8, 6)) * 0.5
    beta, D = 0.5, 3.0
    eta = beta / (1 + beta) ** 2
    v = oracle.rhs(y, beta, 1.0, 1.0)[:, 0:3]
    r = np.linalg.norm(y[:, 0:3], axis=1)
    n = y[:, 0:3] / r[:, None]
    hp, hx = oracle.gw_polarizations(y, beta, 1.0, 1.0, [0, 0, 1], [1, 0, 0], D)
    hxx = 4 * eta / D * (v[:, 0] ** 2 - n[:, 0] ** 2 / r)
    hyy = 4 * eta / D * (v[:, 1] ** 2 - n[:, 1] ** 2 / r)
    hxy = 4 * eta / D * (v[:, 0] * v[:, 1] - n[:, 0] * n[:, 1] / r)
    assert np.allclose(hp, 0.5 * (hxx - hyy), rtol=1e-12, atol=1e-16)
    assert np.allclose(hx, hxy, rtol=1e-12, atol=1e-16)
