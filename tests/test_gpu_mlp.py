"""Closure network on the matrix cores vs its FP64 oracle (same BF16 rounding
points): forward outputs, loss and gradients norm-wise, Adam on identical
gradients, ragged batch tails, padding invariants and a training run.

Tolerances: the oracle rounds the same quantities to bfloat16 but from exact
sums, the GPU from FP32 accumulations; a value within an FP32 rounding of a
bfloat16 tie can round the other way (one bf16 unit, 2^-8 relative), so the
comparisons are norm-wise: outputs 5e-4, gradients 1e-3 of each block's norm
(a block is one weight matrix or bias vector), loss 1e-3.  Loss and gradients
are sums in a fixed order: repeated calls give identical bits.  Adam from
identical gradients is FP32 vs FP64 arithmetic: 1e-5."""
import numpy as np
import pytest
import torch

import dig_workloads as wl
from gpu_common import np_, say
from oracle import mlp as omlp
from paper_2501_10965_amd import _lib as L
from paper_2501_10965_amd.mlp import MLP, pack, unpack

pytestmark = pytest.mark.gpu


def rand_params(seed, scale=0.25):
    rng = np.random.default_rng(seed)
    p = wl.mlp_init(seed)
    for l in range(4):
        W = p[f"W{l}"]
        W[W != 0] += scale * rng.standard_normal(int((W != 0).sum()))
        p[f"W{l}"] = W.astype(np.float32).astype(np.float64)
        b = 0.1 * rng.standard_normal(p[f"b{l}"].shape)
        if l == 3:
            b[7:] = 0.0
        p[f"b{l}"] = b.astype(np.float32).astype(np.float64)
    return p


def batch(seed, n):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 9)).astype(np.float32)
    t = (0.5 * np.tanh(x[:, :7]) + 0.1 * rng.standard_normal((n, 7))).astype(np.float32)
    return x, t


def nrel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("n", [1, 64, 1000, 4096, 100_003])
def test_forward_matches_oracle(n):
    """Tiles of 64 samples; 100,003 samples make the persistent inference grid
    (two workgroups per compute unit) take several tiles each, with a ragged
    last tile."""
    say(f"case mlp forward n={n}")
    p = rand_params(1)
    net = MLP(p, max_batch=64)
    x, _ = batch(2, n)
    y = np_(net.forward(torch.from_numpy(x)))
    ref, _ = omlp.forward(p, x.astype(np.float64))
    assert y.shape == (n, 7)
    say(f"  forward norm-wise error {nrel(y, ref):.2e}")
    assert nrel(y, ref) < 5e-4, nrel(y, ref)
    assert np.abs(y - ref).max() < 0.05 * (np.abs(ref).max() + 0.1)


def test_zero_weights_give_bias_exactly():
    p = rand_params(3)
    for l in range(4):
        p[f"W{l}"][:] = 0.0
    net = MLP(p, max_batch=64)
    x, _ = batch(4, 100)
    y = np_(net.forward(torch.from_numpy(x)))
    np.testing.assert_array_equal(y, np.broadcast_to(p["b3"][:7].astype(np.float32), (100, 7)))


@pytest.mark.parametrize("n,max_batch", [(64, 4096), (333, 4096), (4096, 4096),
                                         (65536, 65536), (40001, 65536)])
def test_gradients_match_oracle(n, max_batch):
    """Batches from one tile to the 65,536 of the training benchmark (the
    weight gradients then split the samples into 64 chunks), with ragged
    tails and a batch below the workspace's capacity."""
    say(f"case mlp grad n={n} max_batch={max_batch}")
    p = rand_params(5)
    net = MLP(p, max_batch=max_batch)
    x, t = batch(6, n)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    loss = float(net.grad(xd, td).item())
    g = net.get_grads()
    lref, gref = omlp.loss_and_grads(p, x.astype(np.float64), t.astype(np.float64))
    assert abs(loss - lref) <= 1e-3 * lref, (loss, lref)
    say("  gradient errors " + " ".join(f"{k}:{nrel(g[k], gref[k]):.1e}" for k in gref))
    for k in gref:
        assert nrel(g[k], gref[k]) < 1e-3, (k, nrel(g[k], gref[k]))
    # fixed summation order: the same call again gives the same bits
    loss2 = float(net.grad(xd, td).item())
    g2 = net.get_grads()
    assert loss2 == loss
    for k in g:
        assert np.array_equal(g[k], g2[k]), k
    # padding receives exactly zero gradient
    assert np.all(g["W0"][:, 9:] == 0) and np.all(g["W3"][7:] == 0) and np.all(g["b3"][7:] == 0)


def test_adam_matches_oracle_on_identical_gradients():
    p = rand_params(7)
    net = MLP(p, max_batch=64)
    po = {k: v.copy() for k, v in p.items()}
    m = omlp.zeros_like_params(po)
    v = omlp.zeros_like_params(po)
    rng = np.random.default_rng(8)
    for step in range(1, 4):
        g = {k: (1e-2 * rng.standard_normal(a.shape)).astype(np.float32).astype(np.float64)
             for k, a in p.items()}
        g["W0"][:, 9:] = 0.0
        g["W3"][7:] = 0.0
        g["b3"][7:] = 0.0
        net.grads.copy_(torch.from_numpy(pack(g)))
        net.adam(1e-3, step)
        omlp.adam(po, g, m, v, step, lr=1e-3)
    got = net.get_params()
    for k in po:
        np.testing.assert_allclose(got[k], po[k], rtol=1e-5, atol=1e-8)
    # the BF16 copies follow the masters: zero weights reproduce the bias
    y = np_(net.forward(torch.zeros((3, 9))))
    assert np.all(np.isfinite(y))


def test_argument_errors():
    net = MLP(rand_params(9), max_batch=64)
    x = torch.zeros((65, 9), device="cuda")
    t = torch.zeros((65, 7), device="cuda")
    with pytest.raises(L.DigError):
        net.grad(x, t)  # above max_batch
    y = torch.empty((0, 7), device="cuda")
    L.check(net.lib.mlp_forward(net.handle, None, None, 0, None))
    assert y.numel() == 0


def test_training_follows_oracle_and_reduces_loss():
    """Twenty Adam steps on GPU and oracle from the same start and batches:
    the loss curves agree to 2 %, and the GPU run reduces the loss."""
    say("case mlp training")
    p = wl.mlp_init(10)
    net = MLP(p, max_batch=512)
    po = {k: v.copy() for k, v in p.items()}
    m = omlp.zeros_like_params(po)
    v = omlp.zeros_like_params(po)
    x, t = batch(11, 512)
    xg, tg = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    lg, lo = [], []
    for step in range(1, 21):
        lg.append(float(net.train_step(xg, tg, 3e-3).item()))
        l, g = omlp.loss_and_grads(po, x.astype(np.float64), t.astype(np.float64))
        omlp.adam(po, g, m, v, step, lr=3e-3)
        lo.append(l)
    lg, lo = np.array(lg), np.array(lo)
    assert np.all(np.abs(lg - lo) <= 0.02 * lo), (lg, lo)
    assert lg[-1] < 0.5 * lg[0]


def test_train_step_equals_grad_then_adam():
    """The fused training step (loss, reduction and Adam in one launch) gives
    bit for bit what mlp_grad followed by mlp_adam gives, over several steps
    and a ragged batch."""
    say("case mlp fused train step")
    p = wl.mlp_init(12)
    a = MLP(p, max_batch=1024)
    b = MLP(p, max_batch=1024)
    for step in range(1, 5):
        n = 1000 - 37 * step
        x, t = batch(20 + step, n)
        xg, tg = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
        la = float(a.train_step(xg, tg, 2e-3).item())
        lb = float(b.grad(xg, tg).item())
        b.adam(2e-3, step)
        assert la == lb, (step, la, lb)
        assert torch.equal(a.grads, b.grads), step
        pa, pb = a.get_params(), b.get_params()
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), (step, k)
    ya = a.forward(torch.from_numpy(batch(30, 300)[0]).cuda())
    yb = b.forward(torch.from_numpy(batch(30, 300)[0]).cuda())
    assert torch.equal(ya, yb)
