"""Oracle pins of the 2.5PN radiation reaction (eq. 6, a_2.5PN) and of the
correction against the integral-invariant references of a dissipative orbit
(Sec. 3B, orbit 3).

The acceleration is the leading-order reaction of a point-mass binary; its
pins are the quadrupole-formula fluxes: on a circular orbit the energy and
angular-momentum losses are -(32/5) eta^2 / r^5 and -(32/5) eta^2 / r^(7/2)
(per unit reduced mass: one factor eta less), averaged over an eccentric
Kepler orbit they are the Peters-Mathews fluxes, and a quasi-circular
inspiral follows r^4 = r0^4 - (256/5) eta t.
"""
import numpy as np
import pytest

NEWT = dict(pn_order=0, spin_orbit=0, spin_spin=0, quad_mono=0)
NEWT_RR = dict(NEWT, rad_reaction=1)


def reaction(O, y, beta, model_rr, model):
    """(v, a): the flow's velocity dH/dp and the reaction acceleration, as the
    difference of the two right-hand sides."""
    f1 = O.rhs(y, beta, 0.0, 0.0, model=model_rr)
    f0 = O.rhs(y, beta, 0.0, 0.0, model=model)
    return f1[:, 0:3], f1[:, 3:6] - f0[:, 3:6]


def kepler_samples(a, e, m):
    """Position and velocity on the Newtonian ellipse (G = M = 1) at m
    equally spaced eccentric anomalies, and the time weights dt/dE / T."""
    E = 2.0 * np.pi * np.arange(m) / m
    b = a * np.sqrt(1.0 - e * e)
    nmean = a ** -1.5
    den = 1.0 - e * np.cos(E)
    y = np.zeros((m, 12))
    y[:, 0] = a * (np.cos(E) - e)
    y[:, 1] = b * np.sin(E)
    y[:, 3] = -a * nmean * np.sin(E) / den
    y[:, 4] = b * nmean * np.cos(E) / den
    return y, den / m


@pytest.mark.parametrize("beta", [1.0, 0.5, 0.1])
def test_circular_fluxes(oracle, beta):
    eta = beta / (1.0 + beta) ** 2
    for R in (10.0, 37.5):
        y = np.zeros((1, 12))
        y[0, 0], y[0, 4] = R, R ** -0.5
        v, a = reaction(oracle, y, beta, NEWT_RR, NEWT)
        dE = float(np.dot(v[0], a[0]))
        dL = float(np.cross(y[0, 0:3], a[0])[2])
        assert abs(dE / (-(32.0 / 5.0) * eta * R ** -5) - 1.0) < 1e-14
        assert abs(dL / (-(32.0 / 5.0) * eta * R ** -3.5) - 1.0) < 1e-14


@pytest.mark.parametrize("a_,e", [(20.0, 0.1), (15.0, 0.4), (30.0, 0.7)])
def test_orbit_averaged_fluxes_are_peters_mathews(oracle, a_, e):
    """The instantaneous losses differ from the quadrupole flux by total time
    derivatives, so their averages over a Kepler orbit are the
    Peters-Mathews fluxes; a dropped term or a wrong coefficient in the
    acceleration changes them."""
    beta = 0.6
    eta = beta / (1.0 + beta) ** 2
    y, w = kepler_samples(a_, e, 4096)
    v, acc = reaction(oracle, y, beta, NEWT_RR, NEWT)
    dE = np.sum(w * np.einsum("ij,ij->i", v, acc))
    dL = np.sum(w * np.cross(y[:, 0:3], acc)[:, 2])
    fE = (1.0 + 73.0 / 24.0 * e ** 2 + 37.0 / 96.0 * e ** 4) / (1.0 - e * e) ** 3.5
    fL = (1.0 + 7.0 / 8.0 * e ** 2) / (1.0 - e * e) ** 2
    assert abs(dE / (-(32.0 / 5.0) * eta * a_ ** -5 * fE) - 1.0) < 1e-9
    assert abs(dL / (-(32.0 / 5.0) * eta * a_ ** -3.5 * fL) - 1.0) < 1e-9


def test_quasi_circular_inspiral_follows_peters(oracle):
    """Newtonian binary with the reaction only, from a circular orbit at
    r0 = 20 (beta = 1): r^4 falls linearly, r^4 = r0^4 - (256/5) eta t, to
    the adiabatic accuracy of the quadrupole approximation."""
    eta = 0.25
    r0 = 20.0
    y = np.zeros((1, 12))
    y[0, 0], y[0, 4] = r0, r0 ** -0.5
    t = 0.0
    for chunk in (2000, 2000, 2000):
        y = oracle.step(y, 1.0, 0.0, 0.0, chunk, model=NEWT_RR, integrator=dict(method=1, h=0.5))
        t += 0.5 * chunk
        r = float(np.linalg.norm(y[0, 0:3]))
        expect = (r0 ** 4 - (256.0 / 5.0) * eta * t) ** 0.25
        assert abs(r / expect - 1.0) < 2e-3, (t, r, expect)


ORBIT3 = dict(beta=1.0, r0=50.0, p0=0.140, th1=np.pi / 4, th2=np.pi / 6, chi1=1.0, chi2=0.85)


def orbit3_state(oracle):
    o = ORBIT3
    return oracle.init_state(np.array([o["r0"]]), o["p0"], o["th1"], 0.0, o["th2"], 0.0, o["beta"],
                             o["chi1"], o["chi2"])


def test_references_follow_the_radiated_energy_and_angular_momentum(oracle):
    """Orbit 3 of the paper (Sec. 3B) with the full Hamiltonian and the
    reaction: the advanced references equal the initial integrals plus the
    time integrals of v.a and r x a along the (uncorrected) trajectory, and
    the uncorrected state's own H and J stay close to them."""
    o = ORBIT3
    full = dict(rad_reaction=1)
    y0 = orbit3_state(oracle)
    H0, J0 = oracle.invariants(y0, o["beta"], o["chi1"], o["chi2"], model=full)
    ref0 = np.column_stack([H0, J0])
    y, ref = oracle.step(y0, o["beta"], o["chi1"], o["chi2"], 2000, model=full, ref=ref0, return_ref=True,
                         integrator=dict(method=1, h=0.25))
    H, J = oracle.invariants(y, o["beta"], o["chi1"], o["chi2"], model=full)
    assert ref[0, 0] < H0[0]                                       # energy radiated
    assert abs(H[0] - ref[0, 0]) < 1e-9 * abs(H0[0])
    assert np.max(np.abs(J[0] - ref[0, 1:])) < 1e-9 * np.linalg.norm(J0[0])
    assert abs(ref[0, 0] - H0[0]) > 1e3 * abs(H[0] - ref[0, 0])    # the change is resolved


def test_correction_holds_the_dissipative_orbit_on_its_references(oracle):
    """With the six-integral correction against the advancing references the
    energy error stays at rounding level while the energy itself falls (no
    secular growth, the paper's Fig. 5(a)); the corrected h = 1 trajectory
    stays closer to a fine-step reference than the uncorrected one."""
    o = ORBIT3
    full = dict(rad_reaction=1)
    args = (o["beta"], o["chi1"], o["chi2"])
    y0 = orbit3_state(oracle)
    H0, J0 = oracle.invariants(y0, *args, model=full)
    ref0 = np.column_stack([H0, J0])
    yc, refc = y0, ref0
    errs = []
    for _ in range(10):
        yc, refc = oracle.step(yc, *args, 500, model=full, ref=refc, return_ref=True, correction=dict(mode=2))
        H, J = oracle.invariants(yc, *args, model=full)
        errs.append(abs(H[0] - refc[0, 0]) / abs(refc[0, 0]))
    assert max(errs) < 1e-14
    assert refc[0, 0] < H0[0]
    yu = oracle.step(y0, *args, 5000, model=full)
    yf = oracle.step(y0, *args, 40000, model=full, integrator=dict(method=1, h=0.125))
    ec = np.linalg.norm(yc[0, 0:3] - yf[0, 0:3])
    eu = np.linalg.norm(yu[0, 0:3] - yf[0, 0:3])
    assert ec < eu and ec < 1e-3 * o["r0"]
    # Spin lengths are untouched by the reaction.
    s1 = np.linalg.norm(yc[0, 6:9])
    s1_0 = np.linalg.norm(y0[0, 6:9])
    assert abs(s1 - s1_0) < 1e-14 * s1_0


def test_scans_refuse_radiation_reaction(oracle):
    y0 = orbit3_state(oracle)
    r = oracle.fli_scan(y0, 100.0, 1.0, 1.0, 0.85, model=dict(rad_reaction=1))
    assert r["status"][0] == oracle.STATUS_BADPARAM
