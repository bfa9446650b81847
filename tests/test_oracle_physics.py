"""Pins of the oracle's Hamiltonian and equations of motion against physics
that does not come from the oracle itself.

* 2PN circular-orbit energy E(x) (gauge invariant closed form) for several
  mass ratios -- pins every orbital coefficient that survives n.p = 0.
* 2PN periastron advance k(E, j) (Damour-Schaefer), by quadrature of the
  oracle's Hamiltonian -- pins the n.p terms that the circular test misses.
* eta -> 0: the isotropic Schwarzschild test-particle Hamiltonian.
* 1.5PN spin-orbit circular-orbit coefficient (aligned spins).
* The paper's printed spin precession vectors, eqs. (8)-(9) (Sec. 2).
* Complex-step derivatives of H against the analytic gradient.
* dH/dt = 0 and dJ/dt = 0 along the flow, pointwise (eqs. 6-7).
"""
import numpy as np
import pytest

from orbit_tools import (circular_energy_2pn, circular_orbit, apsidal_k, periastron_k_2pn,
                         schwarzschild_isotropic_energy, so_circular_coefficient)

ORBITAL = dict(spin_orbit=0, spin_spin=0, quad_mono=0)
ALL_MODELS = [
    dict(pn_order=2, spin_orbit=1, spin_spin=1, quad_mono=1, spin_units=0),
    dict(pn_order=2, spin_orbit=1, spin_spin=1, quad_mono=1, spin_units=1),
    dict(pn_order=1, spin_orbit=1, spin_spin=0, quad_mono=1, spin_units=0),
    dict(pn_order=0, spin_orbit=0, spin_spin=1, quad_mono=0, spin_units=0),
    dict(pn_order=2, spin_orbit=0, spin_spin=0, quad_mono=0, spin_units=0),
]


def random_states(rng, n, rscale=15.0):
    y = np.zeros((n, 12))
    y[:, 0:3] = rng.normal(size=(n, 3))
    y[:, 0:3] *= (rscale * rng.uniform(0.5, 1.5, size=(n, 1))) / np.linalg.norm(y[:, 0:3], axis=1, keepdims=True)
    y[:, 3:6] = 0.3 * rng.normal(size=(n, 3))
    y[:, 6:12] = 0.5 * rng.normal(size=(n, 6))
    return y


def _poly_extrapolate(xs, vals):
    """Value at x = 0 of the polynomial through (xs, vals)."""
    coef = np.polyfit(np.asarray(xs), np.asarray(vals), len(xs) - 1)
    return coef[-1]


@pytest.mark.parametrize("beta", [1.0, 0.5, 0.25, 0.1])
def test_circular_energy_2pn(oracle, beta):
    """E(x) = -(x/2)[1 - (3/4 + eta/12) x - (27/8 - 19 eta/8 + eta^2/24) x^2] + O(x^4):
    the 1PN and 2PN coefficients extracted from circular orbits of the oracle's
    Hamiltonian, extrapolated to x -> 0, match the closed form."""
    eta = beta / (1 + beta) ** 2
    xs, c1s, c2s = [], [], []
    for r in (100.0, 200.0, 400.0, 800.0):
        _, x, E = circular_orbit(oracle, r, beta, 0.0, 0.0, ORBITAL)
        c1 = (E / (-x / 2) - 1) / x
        xs.append(x)
        c1s.append(c1)
        c2s.append((E / (-x / 2) - 1 + (0.75 + eta / 12) * x) / x ** 2)
    c1 = _poly_extrapolate(xs, c1s)
    c2 = _poly_extrapolate(xs, c2s)
    assert abs(c1 - (-(0.75 + eta / 12))) < 1e-6
    assert abs(c2 - (-(27 / 8 - 19 / 8 * eta + eta ** 2 / 24))) < 2e-4
    # And the residual after the 2PN closed form is third-post-Newtonian small.
    _, x, E = circular_orbit(oracle, 400.0, beta, 0.0, 0.0, ORBITAL)
    assert abs(E - circular_energy_2pn(x, eta)) < 20 * x ** 4


@pytest.mark.parametrize("beta", [1.0, 0.3])
def test_periastron_advance_2pn(oracle, beta):
    """k(E, j) = 3/j^2 [1 + (5/4)(7 - 2 eta)/j^2 + (1/2)(5 - 2 eta) E] + O(j^-6).
    The residual of the oracle's apsidal angle scales as j^-6: a wrong 2PN
    coefficient would leave a j^-4 remainder that grows in res * j^6."""
    eta = beta / (1 + beta) ** 2
    scaled = []
    for a in (100.0, 200.0, 400.0):
        e = 0.3
        E, j = -1.0 / (2 * a), np.sqrt(a * (1 - e * e))
        k = apsidal_k(oracle, E, j, beta, ORBITAL)
        scaled.append((k - periastron_k_2pn(E, j, eta)) * j ** 6)
    scaled = np.array(scaled)
    assert np.all(np.abs(scaled) < 300)
    assert np.ptp(scaled) < 0.08 * np.abs(scaled).max()


def test_periastron_advance_newtonian_and_1pn(oracle):
    """Newtonian orbits close (k = 0); at 1PN k = 3/j^2 + O(j^-4)."""
    a, e = 60.0, 0.4
    E, j = -1 / (2 * a), np.sqrt(a * (1 - e * e))
    k0 = apsidal_k(oracle, E, j, 1.0, dict(ORBITAL, pn_order=0))
    assert abs(k0) < 1e-10
    for a in (200.0, 800.0):
        E, j = -1 / (2 * a), np.sqrt(a * (1 - e * e))
        k1 = apsidal_k(oracle, E, j, 0.5, dict(ORBITAL, pn_order=1))
        assert abs(k1 - 3 / j ** 2) < 100 / j ** 4


def test_schwarzschild_test_mass_limit(oracle):
    """eta -> 0: the ADM Hamiltonian equals the 2PN expansion of the isotropic
    Schwarzschild test-particle Hamiltonian; the remainder is 3PN, O(eps^4),
    so halving eps (r -> 2r, p -> p/sqrt 2) divides it by ~16."""
    rng = np.random.default_rng(11)
    for _ in range(4):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        m = rng.normal(size=3)
        m /= np.linalg.norm(m)
        res = []
        for lam in (1.0, 2.0, 4.0, 8.0):
            r, p = 25.0 * lam, 0.22 / np.sqrt(lam)
            y = np.zeros(12)
            y[:3], y[3:6] = r * n, p * m
            H = oracle.hamiltonian(y, 1e-14, 0, 0, model=ORBITAL)[0]
            res.append(H - schwarzschild_isotropic_energy(r, p * p))
        ratios = np.array(res[:-1]) / np.array(res[1:])
        assert np.all((ratios > 14.5) & (ratios < 17.0)), ratios


@pytest.mark.parametrize("beta,chi1,chi2", [(1.0, 0.7, 0.3), (0.5, 0.9, 0.2), (0.2, 0.4, 1.0)])
def test_spin_orbit_circular_coefficient(oracle, beta, chi1, chi2):
    """Aligned spins: E = E_2PN(x) - (x/2) K x^(3/2) + O(x^(7/2)) with
    K = 14/3 (S1 + S2) + 2 delta (S2/X2 - S1/X1) (spins in M^2)."""
    model = dict(spin_spin=0, quad_mono=0)
    cf = oracle.coefficients(beta, chi1, chi2)
    eta, s1, s2 = cf[0], cf[6], cf[7]
    spins = np.array([0, 0, s1, 0, 0, s2])
    K = so_circular_coefficient(beta, eta * s1, eta * s2)   # physical spins = eta * (mu M units)
    xs, ks = [], []
    for r in (200.0, 400.0, 800.0):
        _, x, E = circular_orbit(oracle, r, beta, chi1, chi2, model, spins=spins)
        xs.append(x)
        ks.append((E - circular_energy_2pn(x, eta)) / (-x / 2 * x ** 1.5))
    assert abs(_poly_extrapolate(xs, ks) - K) < 2e-4 * max(1.0, abs(K))


def test_paper_eqs_8_9_spin_precession(oracle):
    """With spins in M^2 the oracle's dH/dS_i, crossed with S_i, equals the
    paper's printed Omega_i x S_i, eqs. (8)-(9) (Sec. 2)."""
    rng = np.random.default_rng(5)
    model = dict(spin_units=1)
    for beta in (1.0, 0.6, 0.2):
        eta = beta / (1 + beta) ** 2
        y = random_states(rng, 20)
        g = oracle.gradient(y, beta, 0.8, 0.6, model=model)
        d = oracle.rhs(y, beta, 0.8, 0.6, model=model)
        for k in range(len(y)):
            r, p, S1, S2 = y[k, 0:3], y[k, 3:6], y[k, 6:9], y[k, 9:12]
            rl = np.linalg.norm(r)
            n = r / rl
            L = np.cross(r, p)
            om1 = ((2 + 3 / (2 * beta)) * L / rl ** 3
                   + (3 * n * S2.dot(n) - S2) / (eta * rl ** 3)
                   + 3 / rl ** 3 * (1 + 1 / beta) ** 2 * n * S1.dot(n))
            om2 = ((2 + 3 * beta / 2) * L / rl ** 3
                   + (3 * n * S1.dot(n) - S1) / (eta * rl ** 3)
                   + 3 / rl ** 3 * (1 + beta) ** 2 * n * S2.dot(n))
            scale1 = np.linalg.norm(om1) * np.linalg.norm(S1)
            scale2 = np.linalg.norm(om2) * np.linalg.norm(S2)
            assert np.allclose(np.cross(g[k, 6:9], S1), np.cross(om1, S1), rtol=0, atol=1e-14 * scale1)
            assert np.allclose(np.cross(g[k, 9:12], S2), np.cross(om2, S2), rtol=0, atol=1e-14 * scale2)
            assert np.allclose(d[k, 6:9], np.cross(om1, S1), rtol=0, atol=1e-14 * scale1)
            assert np.allclose(d[k, 9:12], np.cross(om2, S2), rtol=0, atol=1e-14 * scale2)


def test_spin_unit_tables_describe_one_hamiltonian(oracle):
    """Spins in M^2 are eta times spins in mu*M: both coefficient tables give
    the same H for the same physical state."""
    rng = np.random.default_rng(9)
    for beta in (1.0, 0.35):
        eta = beta / (1 + beta) ** 2
        y = random_states(rng, 10)
        y_m2 = y.copy()
        y_m2[:, 6:] *= eta
        H_phys = oracle.hamiltonian(y, beta, 0.5, 0.5, model=dict(spin_units=0))
        H_m2 = oracle.hamiltonian(y_m2, beta, 0.5, 0.5, model=dict(spin_units=1))
        assert np.allclose(H_phys, H_m2, rtol=1e-14, atol=0)
        c0 = oracle.coefficients(beta, 0.5, 0.5, model=dict(spin_units=0))
        c1 = oracle.coefficients(beta, 0.5, 0.5, model=dict(spin_units=1))
        assert np.allclose(c0[6:8] * eta, c1[6:8], rtol=1e-15)
        # Kerr spin lengths: chi m_i^2 in M^2.
        m1, m2 = beta / (1 + beta), 1 / (1 + beta)
        assert np.allclose(c1[6:8], [0.5 * m1 ** 2, 0.5 * m2 ** 2], rtol=1e-15)


@pytest.mark.parametrize("model", ALL_MODELS)
def test_gradient_matches_complex_step(oracle, model):
    rng = np.random.default_rng(3)
    y = random_states(rng, 50)
    for beta in (1.0, 0.4):
        g = oracle.gradient(y, beta, 0.9, 0.7, model=model)
        gc = oracle.gradient_complex_step(y, beta, 0.9, 0.7, model=model)
        scale = np.abs(g).max(axis=1, keepdims=True)
        assert np.all(np.abs(g - gc) <= 2e-14 * scale)


@pytest.mark.parametrize("model", ALL_MODELS)
def test_flow_conserves_H_and_J_pointwise(oracle, model):
    """dH/dt = grad H . ydot = 0 and dJ/dt = rdot x p + r x pdot + S1dot + S2dot = 0."""
    rng = np.random.default_rng(4)
    y = random_states(rng, 50)
    for beta in (1.0, 0.3):
        g = oracle.gradient_complex_step(y, beta, 0.6, 1.0, model=model)
        d = oracle.rhs(y, beta, 0.6, 1.0, model=model)
        Hdot = np.sum(g * d, axis=1)
        assert np.all(np.abs(Hdot) <= 1e-14 * np.linalg.norm(g, axis=1) * np.linalg.norm(d, axis=1))
        r, p = y[:, 0:3], y[:, 3:6]
        Jdot = np.cross(d[:, 0:3], p) + np.cross(r, d[:, 3:6]) + d[:, 6:9] + d[:, 9:12]
        scale = (np.linalg.norm(d[:, 0:3], axis=1) * np.linalg.norm(p, axis=1)
                 + np.linalg.norm(r, axis=1) * np.linalg.norm(d[:, 3:6], axis=1)
                 + np.linalg.norm(d[:, 6:], axis=1))
        assert np.all(np.linalg.norm(Jdot, axis=1) <= 1e-14 * scale)


def test_spin_lengths_constant_along_flow(oracle):
    rng = np.random.default_rng(6)
    y = random_states(rng, 30)
    d = oracle.rhs(y, 0.7, 0.5, 0.5)
    for a, b in ((6, 9), (9, 12)):
        S, Sd = y[:, a:b], d[:, a:b]
        assert np.all(np.abs(np.sum(S * Sd, axis=1))
                      <= 1e-15 * np.linalg.norm(S, axis=1) * np.linalg.norm(Sd, axis=1) + 1e-300)


def test_newtonian_limit_is_kepler(oracle):
    rng = np.random.default_rng(7)
    y = random_states(rng, 20)
    y[:, 6:] = 0
    model = dict(pn_order=0, spin_orbit=0, spin_spin=0, quad_mono=0)
    H = oracle.hamiltonian(y, 0.5, 0, 0, model=model)
    r = np.linalg.norm(y[:, :3], axis=1)
    assert np.allclose(H, 0.5 * np.sum(y[:, 3:6] ** 2, axis=1) - 1 / r, rtol=1e-15, atol=0)
    d = oracle.rhs(y, 0.5, 0, 0, model=model)
    assert np.allclose(d[:, 0:3], y[:, 3:6], rtol=1e-15, atol=0)
    assert np.allclose(d[:, 3:6], -y[:, 0:3] / r[:, None] ** 3, rtol=1e-14, atol=0)
