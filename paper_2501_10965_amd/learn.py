"""Learned closure: training data from DSMC runs, training on the GPU with the
library's network kernels, and the closure hook that the DIG loop calls.

The network replaces the noisy DSMC-extracted higher-order terms (Section 3.1)
by a function of local gradients and the local Knudsen number where
Kn_lo <= Kn_GLL < Kn_hi; the DSMC terms remain the fallback outside that band
and the judge inside it (closure_blend)."""
from __future__ import annotations

import math

import numpy as np
import torch

from .dsmc import DSMC
from .mlp import MLP

UNIT_SCALING = {"x_mean": [0.0] * 9, "x_std": [1.0] * 9, "y_mean": [0.0] * 7,
                "y_std": [1.0] * 7}


def default_A(omega):
    return (2.0 / 3.0, 0.0, 0.0, 5.0 / (7.0 - 2.0 * omega))


def collect(sim: DSMC, windows: int, window_steps: int, kn_min: float = 0.01, A=None,
            graph: bool = True):
    """Training pairs from `windows` consecutive windows of `window_steps` DSMC
    steps.  The targets of window k are its DSMC-extracted higher-order terms;
    its inputs come from the mean field of the other windows, so that the
    sampling noise of inputs and targets is independent and the network learns
    the conditional mean of the terms given smooth gradients (the field it
    sees in use is a smooth macroscopic one).  Cells with finite Kn_GLL >=
    kn_min.  Returns device tensors x [m, 9], t [m, 7] (unscaled) and the
    instance index of every sample."""
    assert windows >= 2
    A = A if A is not None else default_A(sim.workloads[0]["omega"])
    inst = torch.repeat_interleave(torch.arange(sim.n_inst, device=sim.device),
                                   torch.tensor(sim.ncells, device=sim.device))
    fields, hots = [], []
    for _ in range(windows):
        sim.reset_average()
        sim.step(window_steps, graph=graph)
        f = sim.sample("average")
        # Kn_ref = 0: the DSMC-extracted terms of every cell (no equilibrium mask)
        hot, _, _, _ = sim.closure(f, A, 0.0)
        fields.append(f)
        hots.append(hot)
    total = torch.stack(fields).sum(0)
    xs, ts, ins = [], [], []
    for k in range(windows):
        smooth = (total - fields[k]) / (windows - 1)
        _, _, kn, _ = sim.closure(smooth, A, 0.0)
        x, t = sim.features(smooth, kn, UNIT_SCALING, hot=hots[k])
        sel = torch.isfinite(kn) & (kn >= kn_min)
        xs.append(x[sel])
        ts.append(t[sel])
        ins.append(inst[sel])
    return torch.cat(xs), torch.cat(ts), torch.cat(ins)


def smooth_fields(m: torch.Tensor) -> torch.Tensor:
    """A [20, C] field array whose first six rows are a macroscopic state
    (rho, u, Tt, Tr), e.g. the synthetic-equation solution; the remaining rows
    are zero.  The network's inputs need only those six."""
    out = torch.zeros((20, m.shape[1]), dtype=torch.float64, device=m.device)
    out[0:6] = m[0:6]
    return out


def fit_scaling(x: torch.Tensor, t: torch.Tensor) -> dict:
    """Means and standard deviations of the training inputs and targets."""
    xd, td = x.double().cpu().numpy(), t.double().cpu().numpy()
    sx, sy = xd.std(axis=0), td.std(axis=0)
    return {"x_mean": xd.mean(axis=0).tolist(), "x_std": np.where(sx > 0, sx, 1.0).tolist(),
            "y_mean": td.mean(axis=0).tolist(), "y_std": np.where(sy > 0, sy, 1.0).tolist()}


def standardise(x, t, sc):
    dev = x.device
    xm = torch.tensor(sc["x_mean"], dtype=torch.float32, device=dev)
    xs = torch.tensor(sc["x_std"], dtype=torch.float32, device=dev)
    ym = torch.tensor(sc["y_mean"], dtype=torch.float32, device=dev)
    ys = torch.tensor(sc["y_std"], dtype=torch.float32, device=dev)
    return ((x - xm) / xs).contiguous(), ((t - ym) / ys).contiguous()


def train(net: MLP, x: torch.Tensor, t: torch.Tensor, steps: int, batch: int = 4096,
          lr: float = 1e-3, seed: int = 0, lr_final: float | None = None, log_every: int = 0):
    """Adam on shuffled mini-batches (standardised data); cosine decay to
    lr_final when given.  Returns the loss of every logged step."""
    g = torch.Generator(device=x.device)
    g.manual_seed(seed)
    n = x.shape[0]
    batch = min(batch, n, net.max_batch)
    perm = torch.randperm(n, device=x.device, generator=g)
    pos = 0
    losses = []
    for k in range(steps):
        if pos + batch > n:
            perm = torch.randperm(n, device=x.device, generator=g)
            pos = 0
        idx = perm[pos:pos + batch]
        pos += batch
        xb, tb = x[idx].contiguous(), t[idx].contiguous()
        if lr_final is not None:
            lr_k = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * k / steps))
        else:
            lr_k = lr
        loss = net.train_step(xb, tb, lr_k)
        if log_every and (k % log_every == 0 or k == steps - 1):
            losses.append(float(loss.item()))
    return losses


def evaluate(net: MLP, x: torch.Tensor, t: torch.Tensor) -> float:
    """Mean-squared error of the network on standardised data."""
    y = net.forward(x)
    return float(((y - t) ** 2).mean().item())


class LearnedClosure:
    """Closure hook for DIG: network prediction in the band, DSMC terms as
    fallback and judge."""

    def __init__(self, net: MLP, scaling: dict, kn_lo: float = 0.05, kn_hi: float = math.inf,
                 judge_abs: float = 1.0, judge_rel: float = 0.5):
        self.net = net
        self.scaling = scaling
        self.kn_lo, self.kn_hi = kn_lo, kn_hi
        self.judge_abs, self.judge_rel = judge_abs, judge_rel
        self.last_src = None

    def __call__(self, sim: DSMC, fields, hot, mask, kn, smooth=None):
        """fields, hot, mask, kn: the DSMC-averaged fields and their closure.
        smooth: a smooth macroscopic field [20, C] (the previous synthetic
        solution) from which the network's inputs are taken; without it the
        DSMC-averaged fields are used."""
        src_f, src_kn = fields, kn
        if smooth is not None:
            _, _, src_kn, _ = sim.closure(smooth, default_A(sim.workloads[0]["omega"]), 0.0)
            src_f = smooth
        x, _ = sim.features(src_f, src_kn, self.scaling)
        y = self.net.forward(x)
        self.last_src = sim.blend(fields, src_kn, mask, y, self.scaling, hot, self.kn_lo,
                                  self.kn_hi, self.judge_abs, self.judge_rel)
        return hot
