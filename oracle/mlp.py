"""FP64 oracle of the learned closure network (a multilayer perceptron that
predicts the higher-order constitutive terms from local gradients and the
local Knudsen number).

TEST INFRASTRUCTURE ONLY: only the test suite may import this module; the
product path never calls it.  It shares no code with the HIP kernels.

The network: 4 linear layers, inputs padded from 9 to 32, hidden width 128,
outputs padded from 7 to 16; tanh on the hidden layers, linear output.
Weights W_l are [out][in], biases b_l [out].  Loss = mean over samples and
the 7 real outputs of (y - t)^2.  Training is Adam with bias correction
(Kingma and Ba, 2015).

Precision points of the reduced-precision path (bf16=True), mirroring what
matrix cores with BF16 operands and FP32 accumulation compute: the inputs,
every weight matrix used in a product, every hidden activation and every
back-propagated pre-activation gradient are rounded to bfloat16 (8 significant
bits, round to nearest even); products and sums are exact FP64 here.
With bf16=False every rounding is the identity (the plain FP64 network).
"""
from __future__ import annotations

import numpy as np

N_IN, N_OUT = 9, 7
DIMS = [(32, 128), (128, 128), (128, 128), (128, 16)]  # (in, out), padded


def bf16(x):
    """Round to the nearest bfloat16 value (8 significant bits, ties to even),
    returned as float64.  Zeros, infinities and NaN pass through."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)  # x = m 2^e, 0.5 <= |m| < 1
    r = np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)
    return np.where(np.isfinite(x), r, x)


def _rnd(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def zeros_like_params(p):
    return {k: np.zeros_like(v) for k, v in p.items()}


def forward(p, x, bf16_on=True, act="tanh"):
    """p: {'W0'..'W3', 'b0'..'b3'} float64; x [n, 9].  Returns (y [n, 7], cache)."""
    n = x.shape[0]
    a = np.zeros((n, DIMS[0][0]))
    a[:, :N_IN] = x
    a = _rnd(a, bf16_on)
    acts = [a]
    for l in range(4):
        z = a @ _rnd(p[f"W{l}"], bf16_on).T + p[f"b{l}"]
        if l < 3:
            a = _rnd(np.tanh(z) if act == "tanh" else z, bf16_on)
            acts.append(a)
        else:
            y = z
    return y[:, :N_OUT], {"acts": acts, "y": y}


def loss_and_grads(p, x, t, bf16_on=True, act="tanh"):
    """Mean-squared loss over the real outputs and its gradient for every
    parameter (back-propagation through the network above)."""
    n = x.shape[0]
    y7, cache = forward(p, x, bf16_on, act)
    d = y7 - t
    loss = float(np.mean(d * d))
    dy = np.zeros((n, DIMS[3][1]))
    dy[:, :N_OUT] = 2.0 * d / (n * N_OUT)
    g = _rnd(dy, bf16_on)
    acts = cache["acts"]
    grads = {}
    for l in (3, 2, 1, 0):
        grads[f"W{l}"] = g.T @ acts[l]
        grads[f"b{l}"] = g.sum(axis=0)
        if l > 0:
            da = g @ _rnd(p[f"W{l}"], bf16_on)
            deriv = (1.0 - acts[l] ** 2) if act == "tanh" else 1.0
            g = _rnd(da * deriv, bf16_on)
    return loss, grads


def adam(p, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step at step number t >= 1, in place on p, m, v."""
    c1 = 1.0 - beta1 ** t
    c2 = 1.0 - beta2 ** t
    for k in p:
        g = grads[k]
        m[k] = beta1 * m[k] + (1.0 - beta1) * g
        v[k] = beta2 * v[k] + (1.0 - beta2) * g * g
        p[k] = p[k] - lr * (m[k] / c1) / (np.sqrt(v[k] / c2) + eps)
