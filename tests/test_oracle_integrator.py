"""Pins of the oracle's fixed-step Runge-Kutta integrators.

* Stability polynomials on y' = z y: RK4 gives the degree-4 Taylor polynomial
  of exp(z); the Dormand-Prince fifth-order weights give the degree-5 Taylor
  polynomial plus z^6/600 (b^T A^5 1 of that tableau).
* Global error against the exact Kepler solution (Kepler's equation): slopes
  4 (RK4) and 5 (RK5) in h.
* Uncorrected RK drifts in energy (the paper's Sec. 1 motivation).
"""
import math

import numpy as np
import pytest

from orbit_tools import kepler_position

KEPLER = dict(pn_order=0, spin_orbit=0, spin_spin=0, quad_mono=0)


@pytest.mark.parametrize("z", [-2.5, -1.0, -0.3, 0.1, 0.7, 1.9])
def test_stability_polynomials(oracle, z):
    taylor = [z ** k / math.factorial(k) for k in range(7)]
    r4 = sum(taylor[:5])
    r5 = sum(taylor[:6]) + z ** 6 / 600.0
    assert oracle.rk_linear_step("rk4", z) == pytest.approx(r4, rel=1e-15, abs=1e-15)
    assert oracle.rk_linear_step("rk5", z) == pytest.approx(r5, rel=1e-15, abs=1e-15)


def _kepler_error(oracle, method, h, t_end, r0=10.0, p0=0.36):
    y = np.zeros(12)
    y[0], y[4] = r0, p0
    n = int(round(t_end / h))
    yt = oracle.step(y, 1.0, 0.0, 0.0, n, model=KEPLER, integrator=dict(method=method, h=h))
    return np.linalg.norm(yt[0, :3] - kepler_position(r0, p0, t_end))


def test_kepler_exact_solution_tool():
    """The Kepler's-equation tool returns the start point after one period."""
    r0, p0 = 10.0, 0.36
    E = 0.5 * p0 ** 2 - 1 / r0
    a = -1 / (2 * E)
    T = 2 * np.pi * a ** 1.5
    assert np.allclose(kepler_position(r0, p0, T), [r0, 0, 0], atol=1e-9)
    assert np.allclose(kepler_position(r0, p0, 0.0), [r0, 0, 0], atol=1e-12)


@pytest.mark.parametrize("method,order", [("rk4", 4), ("rk5", 5)])
def test_order_against_exact_kepler(oracle, method, order):
    hs = [1.0, 0.5, 0.25]
    errs = [_kepler_error(oracle, method, h, 200.0) for h in hs]
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(len(hs) - 1)]
    for s in slopes:
        assert order - 0.25 < s < order + 0.35, (errs, slopes)


def test_kepler_period_and_energy(oracle):
    """After one period 2 pi a^(3/2) the RK4 orbit returns to its start, and its
    energy matches p^2/2 - 1/r up to the RK4 truncation error."""
    r0, p0 = 10.0, 0.36
    E0 = 0.5 * p0 ** 2 - 1 / r0
    a = -1 / (2 * E0)
    T = 2 * np.pi * a ** 1.5
    h = T / 2000
    y = np.zeros(12)
    y[0], y[4] = r0, p0
    yt = oracle.step(y, 1.0, 0, 0, 2000, model=KEPLER, integrator=dict(method="rk4", h=h))[0]
    assert np.linalg.norm(yt[:3] - y[:3]) < 1e-7 * r0
    H = oracle.hamiltonian(yt, 1.0, 0, 0, model=KEPLER)[0]
    assert abs(H - E0) < 1e-12


def test_uncorrected_rk_energy_drift_grows(oracle):
    """Without correction the RK4 energy error grows secularly in time."""
    y = np.zeros(12)
    y[0], y[4] = 10.14, 0.365
    H0 = oracle.hamiltonian(y, 1.0, 0, 0)[0]
    errs = []
    yy = y.copy()
    for _ in range(4):
        yy = oracle.step(yy, 1.0, 0, 0, 2500)
        errs.append(abs(oracle.hamiltonian(yy, 1.0, 0, 0)[0] - H0))
    assert errs[-1] > 2.5 * errs[0] and errs[0] > 1e-12
