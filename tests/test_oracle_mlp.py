"""Pins of the closure-network oracle: bfloat16 rounding against its definition
and a library conversion, the zero-weight and linear special cases against
independent matrix chains, back-propagation against central finite
differences, Adam's first step against its closed form, and overfitting."""
import numpy as np
import pytest
import torch

import dig_workloads as wl
from oracle import mlp


def test_bf16_rounding_definition():
    assert mlp.bf16(1.0) == 1.0
    # halfway between 1 and 1 + 2^-7: ties to the even mantissa (1)
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    # halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert mlp.bf16(-(1.0 + 3 * 2.0 ** -8)) == -(1.0 + 2.0 ** -6)
    assert mlp.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert mlp.bf16(0.0) == 0.0
    rng = np.random.default_rng(0)
    x = rng.standard_normal(100000) * 10.0 ** rng.uniform(-6, 6, 100000)
    r = mlp.bf16(x)
    _, e = np.frexp(x)  # half a unit in the 8th significant bit
    assert np.all(np.abs(r - x) <= np.ldexp(1.0, e - 9))
    # agrees with torch's float32 -> bfloat16 conversion on float32 inputs
    x32 = x.astype(np.float32)
    tb = torch.tensor(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x32.astype(np.float64)), tb)


def _rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    p = {}
    for l, (fin, fout) in enumerate(mlp.DIMS):
        p[f"W{l}"] = scale * rng.standard_normal((fout, fin))
        p[f"b{l}"] = 0.1 * rng.standard_normal(fout)
    return p


def test_zero_weights_give_the_bias():
    p = _rand_params(1)
    for l in range(4):
        p[f"W{l}"][:] = 0.0
    x = np.random.default_rng(2).standard_normal((10, 9))
    y, _ = mlp.forward(p, x, bf16_on=True)
    np.testing.assert_array_equal(y, np.broadcast_to(p["b3"][:7], (10, 7)))


def test_linear_network_equals_collapsed_matrix_chain():
    p = _rand_params(3)
    x = np.random.default_rng(4).standard_normal((17, 9))
    y, _ = mlp.forward(p, x, bf16_on=False, act="linear")
    M = p["W3"] @ p["W2"] @ p["W1"] @ p["W0"]
    c = p["W3"] @ (p["W2"] @ (p["W1"] @ p["b0"] + p["b1"]) + p["b2"]) + p["b3"]
    xp = np.zeros((17, 32))
    xp[:, :9] = x
    np.testing.assert_allclose(y, (xp @ M.T + c)[:, :7], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("act", ["tanh", "linear"])
def test_gradients_match_central_differences(act):
    p = _rand_params(5, scale=0.2)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((12, 9))
    t = rng.standard_normal((12, 7))
    _, g = mlp.loss_and_grads(p, x, t, bf16_on=False, act=act)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        gk = g[k].reshape(-1)
        cols = np.arange(flat.size)
        if k.startswith("W0"):
            cols = cols[(cols % 32) < 9]  # padded inputs are always zero
        if k in ("W3", "b3"):
            cols = cols[(cols // (128 if k == "W3" else 1)) < 7]
        for idx in rng.choice(cols, size=min(12, len(cols)), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grads(p, x, t, bf16_on=False, act=act)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grads(p, x, t, bf16_on=False, act=act)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gk[idx]) <= 1e-6 * max(abs(gk[idx]), 1e-3), (k, idx, fd, gk[idx])


def test_padding_gets_no_gradient():
    p = wl.mlp_init(3)
    rng = np.random.default_rng(8)
    x = rng.standard_normal((40, 9))
    t = rng.standard_normal((40, 7))
    _, g = mlp.loss_and_grads(p, x, t)
    assert np.all(g["W0"][:, 9:] == 0)
    assert np.all(g["W3"][7:] == 0) and np.all(g["b3"][7:] == 0)


def test_adam_first_step_closed_form():
    p = _rand_params(9)
    rng = np.random.default_rng(10)
    g = {k: rng.standard_normal(v.shape) for k, v in p.items()}
    m = mlp.zeros_like_params(p)
    v = mlp.zeros_like_params(p)
    p0 = {k: a.copy() for k, a in p.items()}
    mlp.adam(p, g, m, v, 1, lr=1e-2, eps=1e-8)
    for k in p:
        np.testing.assert_allclose(p[k] - p0[k], -1e-2 * g[k] / (np.abs(g[k]) + 1e-8),
                                   rtol=1e-12, atol=1e-15)


def test_overfits_64_samples():
    p = wl.mlp_init(11)
    rng = np.random.default_rng(12)
    x = rng.standard_normal((64, 9))
    t = 0.5 * np.tanh(x[:, :7] + 0.3 * x[:, 1:8] ** 2)
    m = mlp.zeros_like_params(p)
    v = mlp.zeros_like_params(p)
    loss = None
    for it in range(1, 1001):
        loss, g = mlp.loss_and_grads(p, x, t, bf16_on=False)
        mlp.adam(p, g, m, v, it, lr=2e-3)
    assert loss < 1e-6, loss


def test_bf16_path_is_close_to_exact():
    p = wl.mlp_init(13)
    rng = np.random.default_rng(14)
    x = rng.standard_normal((256, 9))
    t = rng.standard_normal((256, 7))
    la, ga = mlp.loss_and_grads(p, x, t, bf16_on=True)
    lb, gb = mlp.loss_and_grads(p, x, t, bf16_on=False)
    assert abs(la - lb) < 1e-2 * lb
    for k in ga:
        nb = np.linalg.norm(gb[k])
        if nb > 0:
            assert np.linalg.norm(ga[k] - gb[k]) < 0.05 * nb, k
