"""Trajectory recording and gravitational-wave polarisations (Sec. 4, eq. 14,
Fig. 10) on the GPU, through the C ABI, against the oracle.

Tolerances: recorded states are those of pn_step itself (bitwise) and of the
oracle to the trajectory bound of 1e-10 relative up to t = 1e3; h_plus and
h_cross from identical states agree to 1e-13 of the largest |h| (one RHS
evaluation, a reciprocal square root and a few products: a few ulps on terms
that partly cancel); from the two sides' own trajectories they agree to
1e-9 of the largest |h| (the trajectory bound times the field's
sensitivity, ~2/|v| per unit relative change of v).
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import DEV, dev, from_soa, random_states, to_soa
from test_oracle_gw import NEWTON, circular_states

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pn():
    assert torch.cuda.is_available(), "GPU parity tests need a ROCm device"
    from paper_1802_00147_amd import pn as P
    P.lib()
    return P


def test_trajectory_rows_equal_stepwise_runs(pn):
    rng = np.random.default_rng(41)
    n = 70                                           # two wavefronts, ragged
    ys = np.zeros((n, 12))
    beta = rng.uniform(0.2, 1.0, n)
    for i in range(n):
        r0 = rng.uniform(9, 30)
        ys[i] = O.init_state(r0, r0 ** -0.5 * rng.uniform(0.9, 1.1), *rng.uniform(0, 3, 4), beta[i], 0.9, 0.7)[0]
    H0, J0 = O.invariants(ys, beta, 0.9, 0.7)
    ref = dev(np.vstack([H0, J0.T]))
    b, c1, c2 = dev(beta), dev(np.full(n, 0.9)), dev(np.full(n, 0.7))
    corr = dict(mode="six")
    y = to_soa(ys)
    traj = pn.trajectory(y, b, c1, c2, 50, 7, correction=corr, ref=ref)
    assert traj.shape == (7, 12, n)
    y2 = to_soa(ys)
    for k in range(7):
        pn.step(y2, b, c1, c2, 7, correction=corr, ref=ref)
        torch.cuda.synchronize()
        assert torch.equal(traj[k], y2), k
    pn.step(y2, b, c1, c2, 1, correction=corr, ref=ref)
    torch.cuda.synchronize()
    assert torch.equal(y, y2)                        # y advanced by all 50 steps
    # Against the oracle at row 6 (t = 49).
    refn = np.vstack([H0, J0.T]).T.copy()
    yo = O.step(ys, beta, 0.9, 0.7, 49, correction=corr, ref=refn)
    got = from_soa(traj[6])
    assert np.all(np.abs(got - yo).max(axis=1) <= 1e-10 * np.abs(yo).max(axis=1))


def test_gw_parity_on_identical_states(pn):
    rng = np.random.default_rng(42)
    n = 300
    ys = random_states(rng, n)
    beta = rng.uniform(0.1, 1.0, n)
    N = np.array([0.2, 0.7, -0.5])
    N /= np.linalg.norm(N)
    p = np.cross(N, [0.0, 0.0, 1.0])
    p /= np.linalg.norm(p)
    for model in (dict(), dict(spin_units=1), NEWTON):
        hp, hx = pn.gw_polarizations(to_soa(ys), dev(beta), dev(np.full(n, 0.8)), dev(np.full(n, 0.6)), N, p,
                                     dist=40.0, model=model)
        ep, ex = O.gw_polarizations(ys, beta, 0.8, 0.6, N, p, 40.0, model=model)
        scale = max(np.abs(ep).max(), np.abs(ex).max())
        assert np.abs(hp.cpu().numpy()[0] - ep).max() <= 1e-13 * scale
        assert np.abs(hx.cpu().numpy()[0] - ex).max() <= 1e-13 * scale


def test_gw_circular_closed_form_and_bad_parameters(pn):
    r, D = 17.0, 250.0
    phis = np.linspace(0, 2 * np.pi, 97)
    ys = circular_states(r, phis)
    hp, hx = pn.gw_polarizations(to_soa(ys), 1.0, 0.0, 0.0, [0, 0, 1], [1, 0, 0], dist=D, model=NEWTON)
    amp = 4 * 0.25 / (D * r)
    assert np.allclose(hp.cpu().numpy()[0], -amp * np.cos(2 * phis), rtol=0, atol=1e-14 * amp)
    assert np.allclose(hx.cpu().numpy()[0], -amp * np.sin(2 * phis), rtol=0, atol=1e-14 * amp)
    # A column with an out-of-range mass ratio gets NaN, the others are unaffected.
    beta = np.full(97, 1.0)
    beta[5] = 1.5
    hp2, _ = pn.gw_polarizations(to_soa(ys), dev(beta), dev(np.zeros(97)), dev(np.zeros(97)), [0, 0, 1],
                                 [1, 0, 0], dist=D, model=NEWTON)
    h = hp2.cpu().numpy()[0]
    assert np.isnan(h[5]) and np.array_equal(np.delete(h, 5), np.delete(hp.cpu().numpy()[0], 5))


@pytest.mark.parametrize("orbit", ["orbit4", "case2_orbit2"])
def test_fig10_waveforms(pn, orbit):
    """Fig. 10's setting: N = z, p = x, q = y; RK5 with the six-integral
    correction; h_plus and h_cross sampled every 5 steps up to t = 1000."""
    rows = {}
    for line in open(__file__.replace("test_gpu_gw.py", "golden/paper_orbits.txt")):
        if line.strip() and not line.startswith("#"):
            f = line.split()
            rows[f[0]] = f
    f = rows[orbit]
    beta, r0, py, chi1, chi2 = map(float, f[1:6])
    s1, s2 = np.array(f[6:9], float), np.array(f[9:12], float)
    c = O.coefficients(beta, chi1, chi2)
    y0 = np.zeros((1, 12))
    y0[0, 0], y0[0, 4] = r0, py
    y0[0, 6:9] = c[6] * s1 / np.linalg.norm(s1)
    y0[0, 9:12] = c[7] * s2 / np.linalg.norm(s2)
    H0, J0 = O.invariants(y0, beta, chi1, chi2)
    refn = np.concatenate([H0, J0[0]])[None, :]
    integ, corr = dict(method="rk5"), dict(mode="six")
    traj = pn.trajectory(to_soa(y0), beta, chi1, chi2, 1000, 5, integrator=integ, correction=corr,
                         ref=dev(refn.T.copy()))
    hp, hx = pn.gw_polarizations(traj, beta, chi1, chi2, [0, 0, 1], [1, 0, 0], dist=1.0)
    states, yo = [], y0.copy()
    for _ in range(200):
        yo = O.step(yo, beta, chi1, chi2, 5, integrator=integ, correction=corr, ref=refn)
        states.append(yo[0].copy())
    states = np.array(states)
    ep, ex = O.gw_polarizations(states, beta, chi1, chi2, [0, 0, 1], [1, 0, 0], 1.0)
    got = traj.cpu().numpy()[:, :, 0]
    assert np.all(np.abs(got - states).max(axis=1) <= 1e-10 * np.abs(states).max(axis=1))
    scale = max(np.abs(ep).max(), np.abs(ex).max())
    assert np.abs(hp.cpu().numpy()[:, 0] - ep).max() <= 1e-9 * scale
    assert np.abs(hx.cpu().numpy()[:, 0] - ex).max() <= 1e-9 * scale
    # The waveform oscillates at twice the orbital frequency: h_plus changes
    # sign several times over 1000 M for these orbits (periods ~ 200-300 M).
    assert np.sum(np.diff(np.sign(ep)) != 0) >= 4


def _gw_raw(pn, traj, n, ns, ld, hp, hx, dist=3.0):
    """pn_gw_polarizations called directly (explicit n, ns, ld)."""
    N3 = (ctypes.c_double * 3)(0.0, 0.0, 1.0)
    P3 = (ctypes.c_double * 3)(1.0, 0.0, 0.0)
    p, keep = pn.params_struct(1.0, 0.8, 0.6)
    return pn.lib().pn_gw_polarizations(ctypes.byref(pn.model_struct()), p, ctypes.c_int64(n), ctypes.c_int64(ns),
                                        pn._ptr(traj), ctypes.c_int64(ld), N3, P3, ctypes.c_double(dist), pn._ptr(hp),
                                        pn._ptr(hx), pn._stream(traj.device))


def test_trajectory_and_gw_padded_layout_and_edges(pn):
    """Columns beyond n (ld > n) are never written; every > nsteps records no
    row and still advances the state; n = 0 and ns = 0 are no-ops."""
    rng = np.random.default_rng(44)
    n, ld = 37, 48
    ys = random_states(rng, n, rscale=20.0)
    sentinel = -12345.0
    y = to_soa(ys, ld=ld)
    y[:, n:] = sentinel
    traj = pn.trajectory(y, 1.0, 0.8, 0.6, 9, 4, correction=dict(mode="spin"), n=n)
    torch.cuda.synchronize()
    assert traj.shape == (2, 12, ld)
    assert torch.all(y[:, n:] == sentinel)
    y2 = to_soa(ys, ld=ld)
    pn.step(y2, 1.0, 0.8, 0.6, 8, correction=dict(mode="spin"), n=n)
    torch.cuda.synchronize()
    assert torch.equal(traj[1][:, :n], y2[:, :n])
    # every > nsteps: no rows, the state still advances.
    y3 = to_soa(ys, ld=ld)
    t0 = pn.trajectory(y3, 1.0, 0.8, 0.6, 3, 5, n=n)
    torch.cuda.synchronize()
    assert t0.shape[0] == 0 and not torch.equal(y3[:, :n], to_soa(ys, ld=ld)[:, :n])
    # Polarisations of the padded layout: only the first n columns are written.
    hp = torch.full((2, ld), sentinel, dtype=torch.float64, device=DEV)
    hx = torch.full((2, ld), sentinel, dtype=torch.float64, device=DEV)
    assert _gw_raw(pn, traj, n, 2, ld, hp, hx) == pn.PN_OK
    torch.cuda.synchronize()
    assert torch.all(hp[:, n:] == sentinel) and torch.all(hx[:, n:] == sentinel)
    ep, ex = O.gw_polarizations(from_soa(traj[1], n), 1.0, 0.8, 0.6, [0, 0, 1], [1, 0, 0], 3.0)
    scale = max(np.abs(ep).max(), np.abs(ex).max())
    assert np.abs(hp[1, :n].cpu().numpy() - ep).max() <= 1e-13 * scale
    assert np.abs(hx[1, :n].cpu().numpy() - ex).max() <= 1e-13 * scale
    assert _gw_raw(pn, traj, 0, 2, ld, hp, hx) == pn.PN_OK
    assert _gw_raw(pn, traj, n, 0, ld, hp, hx) == pn.PN_OK


@pytest.mark.parametrize("reaction", [0, 1])
def test_waveform_with_and_without_dissipation(pn, reaction):
    """Fig. 10's comparison: h_plus of a near-circular binary (r0 = 12,
    beta = 1, no spins) seen face-on, recorded every step for 1,000 steps
    (RK4, six-integral correction; with the 2.5PN reaction the references
    advance).  Without dissipation the wave keeps its period and amplitude
    (zero crossings in the second half within 20% of the first half's
    count, peak within 10%); with it the orbit shrinks and the wave chirps:
    at least 40% more zero crossings and a 20% larger peak in the second
    half.  The GPU's waveform equals the oracle's (each side on its own
    trajectory) to 1e-8 of its peak."""
    model = dict(rad_reaction=reaction)
    y0 = O.init_state(np.array([12.0]), 12 ** -0.5, 0.3, 0.0, 0.5, 0.0, 1.0, 0.0, 0.0)
    H0, J0 = O.invariants(y0, 1.0, 0.0, 0.0, model=model)
    ref0 = np.column_stack([H0, J0])
    steps = 1000
    yd, rd = to_soa(y0), dev(ref0.T)
    traj = pn.trajectory(yd, 1.0, 0.0, 0.0, steps, 1, model=model, correction=dict(mode=2), ref=rd)
    hp, hx = pn.gw_polarizations(traj, 1.0, 0.0, 0.0, [0, 0, 1], [1, 0, 0], dist=1.0, model=model)
    torch.cuda.synchronize()
    hp = hp.cpu().numpy()[:, 0]
    # The oracle's own trajectory and waveform.
    rows, ye, re = [], y0, ref0
    for _ in range(steps):
        ye, re = O.step(ye, 1.0, 0.0, 0.0, 1, model=model, correction=dict(mode=2), ref=re, return_ref=True)
        rows.append(ye[0].copy())
    ep, _ = O.gw_polarizations(np.array(rows), 1.0, 0.0, 0.0, np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0]),
                               dist=1.0, model=model)
    ep = np.asarray(ep).ravel()
    assert np.max(np.abs(hp - ep)) <= 1e-8 * np.max(np.abs(ep))
    h = steps // 2
    zc = np.where(np.diff(np.sign(hp)) != 0)[0]
    n0, n1 = np.sum(zc < h), np.sum(zc >= h)
    a0, a1 = np.max(np.abs(hp[:h])), np.max(np.abs(hp[h:]))
    if reaction:
        assert n1 >= 1.4 * n0 and a1 > 1.2 * a0, (n0, n1, a0, a1)
    else:
        assert abs(n1 / n0 - 1.0) <= 0.2 and abs(a1 / a0 - 1.0) < 0.1, (n0, n1, a0, a1)
