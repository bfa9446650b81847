"""CPU FP64 oracle of the learned surrogate (test infrastructure only).

A plain numpy implementation of the multilayer perceptron that predicts, from
seven orbit features, the chaos label (as a logit) and the FLI relative to
log10(t_end): 7 -> 256 -> 256 -> 256 -> 2 with ReLU, bias in every layer.
Loss per sample: binary cross-entropy of the logit against the integrated
label (1 chaotic, 0 regular) plus a Huber loss (delta = 1) of the second
output against the integrated FLI - log10(t_end); averaged over the batch.
Optimiser: Adam with bias correction on FP32 master weights.

The GPU keeps weights and activations in bfloat16 and accumulates products in
FP32.  To compare like with like, every function here can round its operands
to bfloat16 (round to nearest, ties to even, the IEEE-style rounding of a
float32 to its upper 16 bits) at the same points the GPU stores them: the
inputs, the weights and each hidden activation.  All arithmetic is FP64.

Pins (tests/test_oracle_mlp.py): the gradient against central finite
differences, the losses against closed forms, the first Adam step against its
closed form, the bfloat16 rounding against torch's conversion and hand cases.
"""
import numpy as np

LAYERS = (7, 256, 256, 256, 2)


def round_bf16(x):
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64.  Values are first rounded to float32, as the GPU holds them."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def features(beta, chi1, chi2, r0, th1, th2, t_end, mean, std):
    """Standardised inputs [n, 7]: (beta, chi1, chi2, r0, cos th1, cos th2,
    log10 t_end), each (x - mean) / std."""
    n = len(r0)
    col = (lambda v: np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)))
    raw = np.column_stack([col(beta), col(chi1), col(chi2), col(r0), np.cos(col(th1)), np.cos(col(th2)),
                           np.log10(col(t_end))])
    return (raw - np.asarray(mean, dtype=np.float64)) / np.asarray(std, dtype=np.float64)


def splitmix64(x):
    """SplitMix64 (Steele, Lea & Flood 2014) of uint64 values, elementwise."""
    with np.errstate(over="ignore"):
        x = np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return x ^ (x >> np.uint64(31))


def gate(out, margin, audit, seed):
    """Surrogate labels (logit > 0) and the set of points to integrate:
    |logit| < margin, or drawn for the audit: SplitMix64(seed + i) / 2^64 < audit
    (the top 53 bits as a double in [0, 1))."""
    n = out.shape[0]
    z = out[:, 0]
    with np.errstate(over="ignore"):
        u = (splitmix64(np.uint64(seed) + np.arange(n, dtype=np.uint64)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    label = (z > 0).astype(np.int8)
    chosen = np.nonzero((np.abs(z) < margin) | (u < audit))[0]
    return label, chosen


def forward(params, X, bf16=False):
    """Returns (outputs [B, 2], activations [X, h1, h2, h3]).  With bf16, the
    input, the weights and the hidden activations are rounded to bfloat16."""
    rnd = round_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    h = rnd(X)
    acts = [h]
    for li, (W, b) in enumerate(params):
        z = h @ rnd(W).T + b
        if li < len(params) - 1:
            h = rnd(np.maximum(z, 0.0))
            acts.append(h)
        else:
            h = z
    return h, acts


def bce_with_logits(z, y):
    """log(1 + exp(z)) - y z, evaluated stably."""
    return np.maximum(z, 0.0) - y * z + np.log1p(np.exp(-np.abs(z)))


def huber(x, delta=1.0):
    a = np.abs(x)
    return np.where(a <= delta, 0.5 * x * x, delta * (a - 0.5 * delta))


def loss_and_grad_out(out, label, target, w_reg=1.0):
    """Mean loss over the batch and its gradient with respect to the outputs."""
    B = out.shape[0]
    z, f = out[:, 0], out[:, 1]
    loss = np.mean(bce_with_logits(z, label) + w_reg * huber(f - target))
    sig = 1.0 / (1.0 + np.exp(-z))
    g = np.zeros_like(out)
    g[:, 0] = (sig - label) / B
    g[:, 1] = w_reg * np.clip(f - target, -1.0, 1.0) / B
    return loss, g


def backward(params, acts, g_out, bf16=False):
    """Gradients [(dW_l, db_l)] of the loss given dL/d(outputs), by the chain
    rule through the affine layers and ReLUs (mask: activation > 0)."""
    rnd = round_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    grads = [None] * len(params)
    g = g_out
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        g = rnd(g)                      # the GPU feeds bfloat16 gradients to its GEMMs
        h_in = acts[li]
        grads[li] = (g.T @ h_in, g.sum(axis=0))
        if li > 0:
            g = (g @ rnd(W)) * (acts[li] > 0.0)
    return grads


def adam_step(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), returning new params, m, v."""
    new_p, new_m, new_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        out = []
        for p, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm = b1 * mm + (1.0 - b1) * g
            vv = b2 * vv + (1.0 - b2) * g * g
            mhat = mm / (1.0 - b1 ** step)
            vhat = vv / (1.0 - b2 ** step)
            out.append((p - lr * mhat / (np.sqrt(vhat) + eps), mm, vv))
        new_p.append((out[0][0], out[1][0]))
        new_m.append((out[0][1], out[1][1]))
        new_v.append((out[0][2], out[1][2]))
    return new_p, new_m, new_v


def zeros_like_params(params):
    return [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]


def train_step(params, m, v, step, X, label, target, lr=1e-3, bf16=False):
    """Forward, loss, backward and Adam update on one batch."""
    out, acts = forward(params, X, bf16=bf16)
    loss, g = loss_and_grad_out(out, label, target)
    grads = backward(params, acts, g, bf16=bf16)
    p2, m2, v2 = adam_step(params, grads, m, v, step, lr=lr)
    return p2, m2, v2, loss, grads, out
