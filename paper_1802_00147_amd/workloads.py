"""Seeded synthetic scan inputs, shared by the GPU path, the tests and the
benchmark.  This module only draws and lays out raw per-orbit parameters
(initial radius and momentum, spin angles, mass ratio, spins, end times); it
contains none of the method's arithmetic.

The paper's own scans (Sec. 3C, Table 3) vary spin angles of one orbit; there
is no public dataset, so these grids stand in for them with the same shapes
and kinds of axes:

* single   : one orbit at r0 = 20, beta = 1, chi = 1, isotropic spin
             directions (seed 1), p0 = 20^-1/2 (1 + 0.05 xi), t = 1e4.
* grid64   : 64 x 64 grid, r0 in [10, 40] x spin polar angle theta in [0, pi]
             (theta1 = pi/2, theta2 = theta, azimuths 0, as in Fig. 6),
             p0 = r0^-1/2, beta = 1, chi = 1, t = 1e5.
* grid314  : 314 x 314 grid (Table 3 size), r0 in [10, 40] x p-scaling
             s in [0.8, 1.2], p0 = s r0^-1/2, theta1 = 1.0, theta2 = 1.325
             (orbit 4 of Sec. 4), chi = 1, t = 1e6; variants beta in {1, 0.5}
             x quadrupole-monopole on/off.
* batch1M  : 10^6 orbits (seed 4): beta ~ U[0.1, 1], chi_i ~ U[0, 1],
             isotropic spin directions, r0 ~ U[8, 60], p0 = r0^-1/2,
             t_end = 10^U[3, 6].
* grid4096 : 4096 x 4096 grid over (r0, theta) as grid64.
* fig6     : the paper's spin-angle line (Sec. 3C, Fig. 6): theta2 = 0.01 k,
             k = 0..313, theta1 = pi/2 (panel a) or 0 (panel b), phi = 0,
             (beta, r, p_y) = (1/3, 5.65, 0.765), chi = 1, t = 1e5.  The
             orbital energy of that state is positive; the spin terms make it
             bound only at large theta2 (>= 2.21 in panel a, >= 2.51 in b),
             and the scan removes the rest as UNBOUND_INIT.
* paper orbits: the single test orbits of Sec. 3B (Table 2 Cases I-II,
             orbit 3 with the 2.5PN reaction), PAPER_ORBITS.
* fig7     : the paper's (theta1, theta2) plane (Sec. 3C, Fig. 7, Table 3):
             314 x 314 points theta_i = 0.01 k, r = 10.14, p_y = 0.365,
             beta = 1 (orbit 2 of Sec. 3A), chi = 1, t = 1e5.

All orbits start at r = (r0, 0, 0), p = (0, p0, 0).
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Workload:
    name: str
    r0: np.ndarray
    p0: np.ndarray
    th1: np.ndarray
    ph1: np.ndarray
    th2: np.ndarray
    ph2: np.ndarray
    beta: object            # float, or np.ndarray per orbit
    chi1: object
    chi2: object
    t_end: object           # float, or np.ndarray per orbit
    model: dict = field(default_factory=dict)
    shape: Optional[tuple] = None

    @property
    def n(self):
        return len(self.r0)

    def subset(self, idx):
        idx = np.asarray(idx)
        pick = (lambda v: v[idx] if isinstance(v, np.ndarray) else v)
        return Workload(self.name + "[subset]", *(pick(getattr(self, k)) for k in
                        ("r0", "p0", "th1", "ph1", "th2", "ph2", "beta", "chi1", "chi2", "t_end")),
                        model=dict(self.model), shape=None)

    def steps(self, h=1.0):
        """Orbit-steps of the whole workload (each orbit takes ceil(t_end/h) steps)."""
        t = np.broadcast_to(np.asarray(self.t_end, dtype=np.float64), (self.n,))
        return int(np.ceil(t / h).sum())


def _isotropic(rng, n):
    return np.arccos(rng.uniform(-1.0, 1.0, n)), rng.uniform(0.0, 2.0 * np.pi, n)


def single(seed=1, t_end=1e4):
    rng = np.random.default_rng(seed)
    th1, ph1 = _isotropic(rng, 1)
    th2, ph2 = _isotropic(rng, 1)
    xi = rng.uniform(-1.0, 1.0, 1)
    r0 = np.array([20.0])
    p0 = r0 ** -0.5 * (1.0 + 0.05 * xi)
    return Workload("single", r0, p0, th1, ph1, th2, ph2, 1.0, 1.0, 1.0, float(t_end))


def grid_r_theta(nr, nth, t_end, name):
    r = np.linspace(10.0, 40.0, nr)
    th = np.linspace(0.0, np.pi, nth)
    R, TH = np.meshgrid(r, th, indexing="ij")
    r0 = R.ravel().copy()
    n = r0.size
    return Workload(name, r0, r0 ** -0.5, np.full(n, np.pi / 2), np.zeros(n), TH.ravel().copy(), np.zeros(n),
                    1.0, 1.0, 1.0, float(t_end), shape=(nr, nth))


def grid64(t_end=1e5):
    return grid_r_theta(64, 64, t_end, "grid64")


def grid4096(t_end=1e5):
    return grid_r_theta(4096, 4096, t_end, "grid4096")


def grid314(beta=1.0, quad_mono=1, t_end=1e6):
    r = np.linspace(10.0, 40.0, 314)
    s = np.linspace(0.8, 1.2, 314)
    R, S = np.meshgrid(r, s, indexing="ij")
    r0 = R.ravel().copy()
    n = r0.size
    return Workload(f"grid314_beta{beta:g}_qm{int(quad_mono)}", r0, S.ravel() * r0 ** -0.5,
                    np.full(n, 1.0), np.zeros(n), np.full(n, 1.325), np.zeros(n), float(beta), 1.0, 1.0,
                    float(t_end), model=dict(quad_mono=int(quad_mono)), shape=(314, 314))


# Initial (beta, r0, p_y) of the paper's spin-angle scans (Sec. 3C).
FIG6_STATE = (1.0 / 3.0, 5.65, 0.765)
FIG7_STATE = (1.0, 10.14, 0.365)
FIG_ANGLES = 0.01 * np.arange(314)      # 0 .. 3.13 rad in steps of 0.01


def fig6(theta1=np.pi / 2, t_end=1e5):
    beta, r, p = FIG6_STATE
    n = FIG_ANGLES.size
    return Workload(f"fig6_th1_{theta1:.4g}", np.full(n, r), np.full(n, p), np.full(n, float(theta1)),
                    np.zeros(n), FIG_ANGLES.copy(), np.zeros(n), beta, 1.0, 1.0, float(t_end), shape=(1, n))


def fig7(t_end=1e5):
    beta, r, p = FIG7_STATE
    T1, T2 = np.meshgrid(FIG_ANGLES, FIG_ANGLES, indexing="ij")
    n = T1.size
    return Workload("fig7", np.full(n, r), np.full(n, p), T1.ravel().copy(), np.zeros(n), T2.ravel().copy(),
                    np.zeros(n), beta, 1.0, 1.0, float(t_end), shape=T1.shape)


# Single test orbits printed in the paper: (beta, r0, p_y, chi1, chi2, spin
# unit vectors).  Case I orbits 1-2 and Case II orbits 1-2 of Sec. 3B (Table
# 2; Case II inherits the (beta, r, p) of Case I), orbit 3 of Sec. 3B (the
# dissipative run with the 2.5PN reaction, Fig. 5).
PAPER_ORBITS = {
    "I-1": (1.0 / 3.0, 20.0, 0.2461, 0.0, 0.0, (0.0, 0.0, 1.0), (0.0, 0.0, 1.0)),
    "I-2": (1.0, 10.14, 0.365, 0.0, 0.0, (0.0, 0.0, 1.0), (0.0, 0.0, 1.0)),
    "II-1": (1.0 / 3.0, 20.0, 0.2461, 0.75, 0.75, (np.sin(np.pi / 3), 0.0, np.cos(np.pi / 3)),
             (np.sin(np.pi / 4), 0.0, np.cos(np.pi / 4))),
    "II-2": (1.0, 10.14, 0.365, 1.0, 1.0, (0.13036, 0.262852, -0.955989), (0.118966, -0.13459, -0.983734)),
    "orbit3": (1.0, 50.0, 0.140, 1.0, 0.85, (np.sin(np.pi / 4), 0.0, np.cos(np.pi / 4)),
               (np.sin(np.pi / 6), 0.0, np.cos(np.pi / 6))),
}


def paper_orbit(name, t_end=1e5):
    """One of the paper's test orbits as a one-orbit workload (spin
    directions as polar and azimuthal angles)."""
    beta, r0, py, chi1, chi2, s1, s2 = PAPER_ORBITS[name]
    ang = []
    for s in (s1, s2):
        v = np.asarray(s, dtype=np.float64)
        v = v / np.linalg.norm(v)
        ang += [np.array([np.arccos(np.clip(v[2], -1.0, 1.0))]), np.array([np.arctan2(v[1], v[0])])]
    return Workload(name, np.array([r0]), np.array([py]), ang[0], ang[1], ang[2], ang[3], float(beta),
                    float(chi1), float(chi2), float(t_end))


def batch(n=1_000_000, seed=4, tmin=1e3, tmax=1e6):
    rng = np.random.default_rng(seed)
    beta = rng.uniform(0.1, 1.0, n)
    chi1 = rng.uniform(0.0, 1.0, n)
    chi2 = rng.uniform(0.0, 1.0, n)
    th1, ph1 = _isotropic(rng, n)
    th2, ph2 = _isotropic(rng, n)
    r0 = rng.uniform(8.0, 60.0, n)
    t_end = 10.0 ** rng.uniform(np.log10(tmin), np.log10(tmax), n)
    return Workload("batch1M" if n == 1_000_000 else f"batch{n}", r0, r0 ** -0.5, th1, ph1, th2, ph2,
                    beta, chi1, chi2, t_end)


def strided_sample(n, k, seed=0):
    """k distinct indices in [0, n), seeded, spread over the whole range."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False))


MLP_LAYERS = (7, 256, 256, 256, 2)


def mlp_init_weights(seed=50):
    """Seeded initial weights of the surrogate network: He-uniform W_l of shape
    [n_out, n_in] (bound sqrt(6 / n_in)) and zero biases, float64."""
    rng = np.random.default_rng(seed)
    params = []
    for n_in, n_out in zip(MLP_LAYERS[:-1], MLP_LAYERS[1:]):
        bound = np.sqrt(6.0 / n_in)
        params.append((rng.uniform(-bound, bound, (n_out, n_in)), np.zeros(n_out)))
    return params

