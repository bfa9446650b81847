"""Pins of the surrogate's CPU oracle (oracle/mlp.py): gradients against
central finite differences, losses and the first Adam step against closed
forms, and bfloat16 rounding against torch's conversion and hand cases."""
import numpy as np
import torch

from oracle import mlp as M
from paper_1802_00147_amd.workloads import mlp_init_weights


def small_params(seed=3):
    p = mlp_init_weights(seed)
    # shrink to keep finite differences well conditioned
    return [(W * 0.5, b + 0.01 * np.arange(b.size)) for W, b in p]


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    params = small_params()
    X = rng.normal(size=(16, 7))
    label = (rng.uniform(size=16) < 0.3).astype(float)
    target = rng.normal(size=16)

    def loss_of(ps):
        out, _ = M.forward(ps, X)
        return M.loss_and_grad_out(out, label, target)[0]

    out, acts = M.forward(params, X)
    _, g = M.loss_and_grad_out(out, label, target)
    grads = M.backward(params, acts, g)
    h = 1e-6
    for li in range(4):
        W, b = params[li]
        for (i, j) in [(0, 0), (W.shape[0] - 1, W.shape[1] - 1), (W.shape[0] // 2, W.shape[1] // 3)]:
            Wp, Wm = W.copy(), W.copy()
            Wp[i, j] += h
            Wm[i, j] -= h
            pp = list(params); pp[li] = (Wp, b)
            pm = list(params); pm[li] = (Wm, b)
            fd = (loss_of(pp) - loss_of(pm)) / (2 * h)
            assert abs(fd - grads[li][0][i, j]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9
        k = b.size // 2
        bp, bm = b.copy(), b.copy()
        bp[k] += h
        bm[k] -= h
        pp = list(params); pp[li] = (W, bp)
        pm = list(params); pm[li] = (W, bm)
        fd = (loss_of(pp) - loss_of(pm)) / (2 * h)
        assert abs(fd - grads[li][1][k]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9


def test_loss_closed_forms():
    assert np.isclose(M.bce_with_logits(np.array([0.0]), np.array([1.0]))[0], np.log(2.0))
    assert M.bce_with_logits(np.array([40.0]), np.array([1.0]))[0] < 1e-15
    assert np.isclose(M.bce_with_logits(np.array([-3.0]), np.array([1.0]))[0], np.log1p(np.exp(3.0)))
    assert np.allclose(M.huber(np.array([0.5, -2.0, 1.0])), [0.125, 1.5, 0.5])


def test_first_adam_step_closed_form():
    """From zero moments the first bias-corrected step is -lr g/(|g| + eps)."""
    params = [(np.ones((2, 3)), np.zeros(2))]
    g = [(np.array([[0.5, -2.0, 1e-3], [3.0, -1.0, 0.0]]), np.array([0.25, -0.5]))]
    new, m, v = M.adam_step(params, g, M.zeros_like_params(params), M.zeros_like_params(params), 1, lr=0.01)
    exp = 1.0 - 0.01 * g[0][0] / (np.abs(g[0][0]) + 1e-8)
    assert np.allclose(new[0][0], exp, rtol=1e-12, atol=1e-15)
    assert np.allclose(m[0][0], 0.1 * g[0][0]) and np.allclose(v[0][0], 0.001 * g[0][0] ** 2)


def test_bf16_rounding():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=1000) * 10 ** rng.uniform(-5, 5, 1000), [0.0, -0.0, 1.0, 1e-40]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.round_bf16(x), ref)
    # ties to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> 1; 1 + 3*2^-8 -> 1 + 2^-6
    assert M.round_bf16(np.array([1 + 2 ** -8]))[0] == 1.0
    assert M.round_bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6


def test_training_reduces_loss_on_a_separable_toy():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(256, 7))
    label = (X[:, 0] + 0.5 * X[:, 3] > 0).astype(float)
    target = 0.3 * X[:, 1]
    params = mlp_init_weights(7)
    m, v = M.zeros_like_params(params), M.zeros_like_params(params)
    losses = []
    for step in range(1, 61):
        params, m, v, loss, _, _ = M.train_step(params, m, v, step, X, label, target, lr=3e-3)
        losses.append(loss)
    assert losses[-1] < 0.3 * losses[0]


def test_splitmix64_reference_values():
    """SplitMix64 from state 0: the published first outputs of the generator
    (successive calls add the golden gamma 0x9E3779B97F4A7C15 to the state)."""
    outs = M.splitmix64(np.array([0, 0x9E3779B97F4A7C15, (2 * 0x9E3779B97F4A7C15) % 2 ** 64], dtype=np.uint64))
    assert [int(v) for v in outs] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_gate_selects_margin_and_audit():
    rng = np.random.default_rng(3)
    out = np.column_stack([rng.normal(size=20000), rng.normal(size=20000)])
    label, chosen = M.gate(out, 0.5, 0.01, 5)
    inside = np.abs(out[:, 0]) < 0.5
    assert set(np.nonzero(inside)[0]) <= set(chosen)
    extra = len(set(chosen) - set(np.nonzero(inside)[0]))
    assert 0.6 * 0.01 * (~inside).sum() < extra < 1.4 * 0.01 * (~inside).sum()
    assert np.array_equal(label, (out[:, 0] > 0).astype(np.int8))
