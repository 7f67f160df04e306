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
    kn_min.  The library's kernels sample, close and build the features; the
    window means and the selection are host (numpy) work.  Returns host
    arrays x [m, 9], t [m, 7] (float32, unscaled) and the instance of every
    sample."""
    assert windows >= 2
    A = A if A is not None else default_A(sim.workloads[0]["omega"])
    inst = np.repeat(np.arange(sim.n_inst), np.asarray(sim.ncells))
    fields, hots = [], []
    for _ in range(windows):
        sim.reset_average()
        sim.step(window_steps, graph=graph)
        f = sim.sample("average")
        # Kn_ref = 0: the DSMC-extracted terms of every cell (no equilibrium mask)
        hot, _, _, _ = sim.closure(f, A, 0.0)
        fields.append(f.cpu().numpy())
        hots.append(hot)
    total = np.sum(fields, axis=0)
    xs, ts, ins = [], [], []
    for k in range(windows):
        smooth = torch.from_numpy((total - fields[k]) / (windows - 1)).to(sim.device)
        _, _, kn, _ = sim.closure(smooth, A, 0.0)
        x, t = sim.features(smooth, kn, UNIT_SCALING, hot=hots[k])
        knh = kn.cpu().numpy()
        sel = np.isfinite(knh) & (knh >= kn_min)
        xs.append(x.cpu().numpy()[sel])
        ts.append(t.cpu().numpy()[sel])
        ins.append(inst[sel])
    return np.concatenate(xs), np.concatenate(ts), np.concatenate(ins)


def smooth_fields(m: torch.Tensor) -> torch.Tensor:
    """A [20, C] field array whose first six rows are a macroscopic state
    (rho, u, Tt, Tr), e.g. the synthetic-equation solution; the remaining rows
    are zero.  The network's inputs need only those six."""
    out = torch.zeros((20, m.shape[1]), dtype=torch.float64, device=m.device)
    out[0:6].copy_(m[0:6])
    return out


def fit_scaling(x: np.ndarray, t: np.ndarray) -> dict:
    """Means and standard deviations of the training inputs and targets."""
    xd, td = np.asarray(x, np.float64), np.asarray(t, np.float64)
    sx, sy = xd.std(axis=0), td.std(axis=0)
    return {"x_mean": xd.mean(axis=0).tolist(), "x_std": np.where(sx > 0, sx, 1.0).tolist(),
            "y_mean": td.mean(axis=0).tolist(), "y_std": np.where(sy > 0, sy, 1.0).tolist()}


def standardise(x: np.ndarray, t: np.ndarray, sc: dict):
    """(x - mean) / std and (t - mean) / std on the host, float32."""
    xs = (np.asarray(x, np.float64) - sc["x_mean"]) / sc["x_std"]
    ts = (np.asarray(t, np.float64) - sc["y_mean"]) / sc["y_std"]
    return np.ascontiguousarray(xs, np.float32), np.ascontiguousarray(ts, np.float32)


def train(net: MLP, x: np.ndarray, t: np.ndarray, steps: int, batch: int = 4096,
          lr: float = 1e-3, seed: int = 0, lr_final: float | None = None, log_every: int = 0):
    """Adam on shuffled mini-batches of standardised host data (x [n, 9],
    t [n, 7] float32): each batch is gathered on the host and copied to the
    GPU, where the library's kernels take the training step.  Cosine decay to
    lr_final when given.  Returns the loss of every logged step."""
    rng = np.random.default_rng(seed)
    n = x.shape[0]
    batch = min(batch, n, net.max_batch)
    dev = net.ws.device
    xb = torch.empty((batch, 9), dtype=torch.float32, device=dev)
    tb = torch.empty((batch, 7), dtype=torch.float32, device=dev)
    perm = rng.permutation(n)
    pos = 0
    losses = []
    for k in range(steps):
        if pos + batch > n:
            perm = rng.permutation(n)
            pos = 0
        idx = perm[pos:pos + batch]
        pos += batch
        xb.copy_(torch.from_numpy(x[idx]))
        tb.copy_(torch.from_numpy(t[idx]))
        if lr_final is not None:
            lr_k = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * k / steps))
        else:
            lr_k = lr
        loss = net.train_step(xb, tb, lr_k)
        if log_every and (k % log_every == 0 or k == steps - 1):
            losses.append(float(loss.item()))
    return losses


def evaluate(net: MLP, x: np.ndarray, t: np.ndarray) -> float:
    """Mean-squared error of the network on standardised host data."""
    y = net.forward(torch.from_numpy(np.ascontiguousarray(x)).to(net.ws.device))
    return float(np.mean((y.cpu().numpy().astype(np.float64) - t) ** 2))


def judge_steps(w: dict, nsteps: int) -> float:
    """Independent samples per particle in an average over nsteps DSMC steps:
    velocities decorrelate over about two mean collision times (at unit
    density and temperature), so nsteps dt / (2 tau_c), at least 1."""
    tau_c = (5.0 - 2.0 * w["omega"]) * (7.0 - 2.0 * w["omega"]) * w["kn"] * \
        math.sqrt(2.0 / math.pi) / 30.0
    return max(1.0, nsteps * w["dt"] / (2.0 * tau_c))


class LearnedClosure:
    """Closure hook for DIG: network prediction in the band, DSMC terms as
    fallback and judge.  The judge rejects a prediction that differs from the
    DSMC-extracted term by more than judge_sigma standard errors of that term
    (its sampling noise over the averaged steps, closure_blend) plus
    judge_rel of its size; defaults 3 and 0.1."""

    def __init__(self, net: MLP, scaling: dict, kn_lo: float = 0.05, kn_hi: float = math.inf,
                 judge_sigma: float = 3.0, judge_rel: float = 0.1, avg_steps: int = 50):
        self.net = net
        self.scaling = scaling
        self.kn_lo, self.kn_hi = kn_lo, kn_hi
        self.judge_sigma, self.judge_rel = judge_sigma, judge_rel
        self.avg_steps = avg_steps
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
                                  self.kn_hi, self.judge_sigma, self.judge_rel,
                                  judge_steps(sim.workloads[0], self.avg_steps))
        return hot
