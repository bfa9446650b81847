"""Closed-form and numerical tools the oracle pins use (test helpers only).

Nothing here implements the method: these are textbook results (Kepler's
equation, circular-orbit energies, periastron advance) and root finders /
quadratures that evaluate the oracle's Hamiltonian and gradient.
"""
import numpy as np


# --------------------------------------------------------------------------
# Kepler problem (Newtonian, G = M = 1).
# --------------------------------------------------------------------------
def kepler_position(r0, p0, t):
    """Exact position at time t of the orbit starting at periapsis or apoapsis
    r = (r0, 0, 0), p = (0, p0, 0) (Kepler's equation solved by Newton)."""
    E = 0.5 * p0 * p0 - 1.0 / r0
    a = -1.0 / (2.0 * E)
    L = r0 * p0
    e = np.sqrt(max(0.0, 1.0 - L * L / a))
    n = a ** -1.5
    # Start at periapsis when r0 < a, at apoapsis otherwise.
    at_peri = r0 < a
    M0 = 0.0 if at_peri else np.pi
    M = M0 + n * t
    Ean = M if e < 0.8 else np.pi
    for _ in range(60):
        f = Ean - e * np.sin(Ean) - M
        Ean -= f / (1.0 - e * np.cos(Ean))
    # Perifocal coordinates (x towards periapsis, y along the motion).
    xp = a * (np.cos(Ean) - e)
    yp = a * np.sqrt(1.0 - e * e) * np.sin(Ean)
    if at_peri:
        return np.array([xp, yp, 0.0])
    # Apoapsis at +x: periapsis direction is -x, the motion still along +y.
    return np.array([-xp, -yp, 0.0])


# --------------------------------------------------------------------------
# Closed forms from the PN literature (gauge invariant).
# --------------------------------------------------------------------------
def circular_energy_2pn(x, eta):
    """E(x) per unit reduced mass through 2PN, x = (M omega)^(2/3)."""
    return -0.5 * x * (1.0 - (0.75 + eta / 12.0) * x
                       - (27.0 / 8.0 - 19.0 / 8.0 * eta + eta * eta / 24.0) * x * x)


def so_circular_coefficient(beta, S1_m2, S2_m2):
    """Coefficient K of the 1.5PN spin-orbit circular-orbit energy,
    E_SO = -(x/2) K x^(3/2), spins along L in units of M^2:
    K = 14/3 (S1 + S2) + 2 delta (S2/X2 - S1/X1), delta = X1 - X2."""
    X1 = beta / (1.0 + beta)
    X2 = 1.0 / (1.0 + beta)
    return 14.0 / 3.0 * (S1_m2 + S2_m2) + 2.0 * (X1 - X2) * (S2_m2 / X2 - S1_m2 / X1)


def periastron_k_2pn(E, j, eta):
    """Fractional periastron advance k = Delta_phi/(2 pi) - 1 through 2PN
    (Damour-Schaefer), E the reduced energy, j the reduced angular momentum."""
    return 3.0 / j ** 2 * (1.0 + (1.25 * (7.0 - 2.0 * eta) / j ** 2 + 0.5 * (5.0 - 2.0 * eta) * E))


def schwarzschild_isotropic_energy(r, p2):
    """Test-particle Hamiltonian per unit mass minus rest mass, isotropic
    Schwarzschild coordinates: alpha sqrt(1 + p^2/psi^4) - 1."""
    u = 1.0 / r
    alpha = (1.0 - u / 2.0) / (1.0 + u / 2.0)
    psi = 1.0 + u / 2.0
    return alpha * np.sqrt(1.0 + p2 / psi ** 4) - 1.0


# --------------------------------------------------------------------------
# Numerical circular orbits and apsidal angles of the oracle's Hamiltonian.
# --------------------------------------------------------------------------
def _planar_state(r, pr, j, spins=None):
    y = np.zeros(12)
    y[0] = r
    y[3] = pr
    y[4] = j / r
    if spins is not None:
        y[6:] = spins
    return y


def circular_orbit(O, r, beta, chi1, chi2, model, spins=None):
    """Tangential momentum p of the circular orbit through r = (r, 0, 0) in the
    xy plane, and its (x, E).  Condition: dH/dr at fixed j vanishes, i.e.
    dH/dx - (j/r^2) dH/dpy = 0 with p = (0, j/r, 0)."""
    def f(j):
        y = _planar_state(r, 0.0, j, spins)
        g = O.gradient(y, beta, chi1, chi2, model=model)[0]
        return g[0] - (j / r ** 2) * g[4]
    j0 = np.sqrt(r)
    lo, hi = 0.8 * j0, 1.25 * j0
    flo, fhi = f(lo), f(hi)
    assert flo * fhi < 0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        fm = f(mid)
        if fm == 0.0 or hi - lo <= 4e-16 * mid:
            break
        if (fm < 0) == (flo < 0):
            lo, flo = mid, fm
        else:
            hi, fhi = mid, fm
    j = 0.5 * (lo + hi)
    y = _planar_state(r, 0.0, j, spins)
    g = O.gradient(y, beta, chi1, chi2, model=model)[0]
    omega = g[4] / r
    E = O.hamiltonian(y, beta, chi1, chi2, model=model)[0]
    return j, omega ** (2.0 / 3.0), E


def apsidal_k(O, E, j, beta, model, nodes=96):
    """Fractional periastron advance of the oracle's planar, spinless
    Hamiltonian at energy E and angular momentum j, by quadrature:
    Delta_phi = 2 int (dH/dp_phi)/(dH/dp_r) dr between the turning points."""
    chi = 0.0

    def H(r, pr):
        return O.hamiltonian(_planar_state(r, pr, j), beta, chi, chi, model=model)[0]

    def turning(rguess):
        r = rguess
        for _ in range(100):
            y = _planar_state(r, 0.0, j)
            g = O.gradient(y, beta, chi, chi, model=model)[0]
            dHdr = g[0] - (j / r ** 2) * g[4]
            dr = -(H(r, 0.0) - E) / dHdr
            r += dr
            if abs(dr) < 1e-15 * r:
                break
        return r

    a = -1.0 / (2.0 * E)
    e = np.sqrt(max(0.0, 1.0 - j * j / a))
    rmin = turning(a * (1 - e))
    rmax = turning(a * (1 + e))
    rm, ra = 0.5 * (rmax + rmin), 0.5 * (rmax - rmin)
    xg, wg = np.polynomial.legendre.leggauss(nodes)
    chis = 0.5 * np.pi * (xg + 1.0)
    w = 0.5 * np.pi * wg
    total = 0.0
    for c, wi in zip(chis, w):
        r = rm - ra * np.cos(c)
        # H is even in p_r: Newton on q = p_r^2, dH/dq = (dH/dp_r) / (2 p_r).
        q = max(2.0 * (E + 1.0 / r) - j * j / (r * r), 1e-12)
        for _ in range(100):
            pr = np.sqrt(q)
            y = _planar_state(r, pr, j)
            g = O.gradient(y, beta, chi, chi, model=model)[0]
            dq = -(H(r, pr) - E) / (g[3] / (2.0 * pr))
            q = max(q + dq, 0.25 * q)
            if abs(dq) < 1e-15 * q:
                break
        pr = np.sqrt(q)
        y = _planar_state(r, pr, j)
        g = O.gradient(y, beta, chi, chi, model=model)[0]
        dphi_dr = (g[4] / r) / g[3]
        total += wi * dphi_dr * ra * np.sin(c)
    return 2.0 * total / (2.0 * np.pi) - 1.0
