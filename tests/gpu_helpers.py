"""Shared helpers for the GPU parity tests: layout conversion between the
oracle's (n, 12) rows and the library's (12, ld) structure of arrays, and
seeded random states."""
import numpy as np
import torch

DEV = "cuda:0"


def to_soa(y_aos, ld=None):
    y_aos = np.asarray(y_aos, dtype=np.float64)
    n = y_aos.shape[0]
    ld = ld or n
    out = np.zeros((12, ld))
    out[:, :n] = y_aos.T
    return torch.from_numpy(out).to(DEV).contiguous()


def from_soa(t, n=None):
    a = t.detach().cpu().numpy()
    n = a.shape[1] if n is None else n
    return np.ascontiguousarray(a[:, :n].T)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def random_states(rng, n, rscale=15.0):
    """Generic states (not on orbits): r ~ rscale, p ~ 0.3, spins ~ 0.5."""
    y = np.zeros((n, 12))
    d = rng.normal(size=(n, 3))
    y[:, 0:3] = d / np.linalg.norm(d, axis=1, keepdims=True) * rscale * rng.uniform(0.5, 1.5, (n, 1))
    y[:, 3:6] = 0.3 * rng.normal(size=(n, 3))
    y[:, 6:12] = 0.5 * rng.normal(size=(n, 6))
    return y


def orbit_states(O, rng, n, beta=None, chi=(0.8, 0.6), steps=(5, 200)):
    """States on bound orbits, moved a random number of RK steps along them."""
    ys, betas = [], []
    for _ in range(n):
        b = rng.uniform(0.2, 1.0) if beta is None else beta
        r0 = rng.uniform(8, 40)
        p0 = rng.uniform(0.85, 1.15) / np.sqrt(r0)
        th = rng.uniform(0, np.pi, 2)
        ph = rng.uniform(0, 2 * np.pi, 2)
        y = O.init_state(r0, p0, th[0], ph[0], th[1], ph[1], b, chi[0], chi[1])[0]
        y = O.step(y, b, chi[0], chi[1], int(rng.integers(*steps)))[0]
        ys.append(y)
        betas.append(b)
    return np.array(ys), np.array(betas)


def rel_err_rows(a, b, floor=1e-300):
    """Row-wise max |a - b| / max|b| over the 12 components."""
    num = np.abs(a - b).max(axis=1)
    den = np.maximum(np.abs(b).max(axis=1), floor)
    return num / den
