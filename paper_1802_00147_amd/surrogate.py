"""Surrogate-assisted FLI scans: a small network trained on FLIs that the
FP64 scan itself produced predicts the chaos label of scan points; points it
is unsure of, and a random audit sample, are integrated, and the integrated
labels win.

The assisted scan itself is one library call (pn_surrogate_scan); training
on a finished scan is a loop of pn_mlp_train_step calls.  This module holds
the host-side bookkeeping of a data loader: feature statistics and the seeded
order of training samples.
"""
import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import pn
from . import workloads as W


@dataclass
class FeatureStats:
    mean: np.ndarray
    std: np.ndarray


def feature_stats(wl):
    """Mean and standard deviation of the seven raw inputs over a workload
    (host preprocessing of the training set)."""
    n = wl.n
    col = (lambda v: np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)))
    raw = np.column_stack([col(wl.beta), col(wl.chi1), col(wl.chi2), wl.r0, np.cos(wl.th1), np.cos(wl.th2),
                           np.log10(col(wl.t_end))])
    std = raw.std(axis=0)
    std[std == 0] = 1.0
    return FeatureStats(raw.mean(axis=0), std)


def _dev(a, device):
    return torch.as_tensor(a, device=device) if isinstance(a, np.ndarray) else a


def workload_features(wl, stats, device, idx=None):
    cols = {k: torch.as_tensor(getattr(wl, k), device=device) for k in ("r0", "th1", "th2")}
    n = wl.n if idx is None else idx.numel()
    return pn.mlp_features(n, cols["r0"], cols["th1"], cols["th2"], _dev(wl.t_end, device),
                           _dev(wl.beta, device), _dev(wl.chi1, device), _dev(wl.chi2, device),
                           stats.mean, stats.std, idx=idx)


@dataclass
class TrainingSet:
    feat: torch.Tensor         # [n, 8] standardised features (device)
    label: torch.Tensor        # [n] 1.0 chaotic / 0.0 regular
    target: torch.Tensor       # [n] FLI - log10 t_end
    valid: np.ndarray          # indices of orbits with a valid status
    stats: FeatureStats


def training_set(wl, scan_out, device):
    """Pairs (features, integrated label and FLI) from a scan of `wl`."""
    stats = feature_stats(wl)
    feat = workload_features(wl, stats, device)
    status = scan_out["status"].cpu().numpy()
    lab = scan_out["label"].cpu().numpy()
    valid = np.nonzero(((status & 0xFF) == 0) & (lab >= 0))[0]
    label, target = pn.mlp_targets(scan_out["fli"], scan_out["label"], _dev(wl.t_end, device))
    return TrainingSet(feat, label, target, valid, stats)


def train(ts, epochs=20, batch=4096, lr=1e-3, cosine=True, seed=50, init_seed=50, device="cuda:0", log=None):
    """Train the network on the valid samples of `ts`; returns (network, mean
    loss per epoch).  cosine: the learning rate of epoch e is
    lr (1 + cos(pi e / epochs)) / 2, else constant."""
    params = W.mlp_init_weights(init_seed)
    net = pn.Network([W_ for W_, _ in params], [b for _, b in params], device)
    rng = np.random.default_rng(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=device)
    ws = None
    history = []
    nb = len(ts.valid) // batch
    for ep in range(epochs):
        lr_ep = lr * 0.5 * (1.0 + math.cos(math.pi * ep / epochs)) if cosine else lr
        order = torch.as_tensor(rng.permutation(ts.valid).astype(np.int32), device=device)
        loss.zero_()
        ws = pn.mlp_train(net, ts.feat, ts.label, ts.target, order[:nb * batch], batch, lr_ep, loss, ws)
        history.append(float(loss.item()) / max(nb, 1))
        if log:
            log(f"epoch {ep}: mean loss {history[-1]:.5f}")
    return net, history


@dataclass
class SurrogateResult:
    label: torch.Tensor          # final labels of the grid (int8)
    integrated: int              # number of points integrated
    points: torch.Tensor         # their indices (int32)
    timings: dict = field(default_factory=dict)
    ws: object = None            # the device workspace, reusable by the next call
    scans: list = field(default_factory=list)   # the audit's and the fallback's FP64 scan launches


def surrogate_scan(net, wl, stats, margin=0.5, audit=0.01, seed=5, model=None,
                   refine_epochs=0, refine_batch=2048, refine_lr=5e-4, refine_seed=51, refine_cosine=0, audit_split=0,
                   ws=None):
    """Labels of every point of the workload `wl` through pn_surrogate_scan:

    1. the audit sample (SplitMix64(seed + i) / 2^64 < audit) is integrated
       (with audit_split, its first whole number of batch-kernel rounds);
    2. with refine_epochs > 0 the network is first trained further on those
       integrated points (FLIs the method produced on this very scan);
    3. fused inference on every point; points with |logit| < margin are
       integrated, with the rest of the audit;
    4. integrated labels replace the network's wherever they exist.
    """
    device = net.w[0].device
    cols = {k: torch.as_tensor(getattr(wl, k), device=device) for k in ("r0", "p0", "th1", "ph1", "th2", "ph2")}
    cfg = dict(margin=margin, audit_frac=audit, seed=seed, refine_epochs=refine_epochs, refine_batch=refine_batch,
               refine_lr=refine_lr, refine_seed=refine_seed, refine_cosine=refine_cosine, audit_split=audit_split)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = pn.surrogate_scan(net, wl.n, cols["r0"], cols["p0"], cols["th1"], cols["ph1"], cols["th2"], cols["ph2"],
                          _dev(wl.t_end, device), _dev(wl.beta, device), _dev(wl.chi1, device),
                          _dev(wl.chi2, device), stats.mean, stats.std, cfg=cfg, model=model, ws=ws)
    torch.cuda.synchronize()
    ph = r["phase_ms"]
    t = dict(audit_s=ph[0] * 1e-3, refine_s=ph[1] * 1e-3, infer_gate_s=ph[2] * 1e-3, fallback_s=ph[3] * 1e-3,
             total_s=time.perf_counter() - t0)
    return SurrogateResult(r["label"], r["integrated"], r["points"], t, r["ws"], r["scans"])
