"""Time to steady state at a fixed field error, on one GPU: plain DSMC, DIG
with DSMC-extracted higher-order terms, and DIG with the learned closure.

The convergence observable is the paper's for the cavity (Section 4.1): the
velocity u_x along the vertical centreline x = 0.5.  It is taken from the
DSMC samples of every cycle (N_s steps), averaged over a sliding window of the
last `window` cycles, reduced to `points` block averages along y (of the
`columns` centre columns), and compared with a reference profile from a long plain-DSMC
run: err = RMS over the points of |profile - reference| / (max - min of the
reference).  Steady state is the first wall time after which err stays at or
below the threshold.  Wall time counts every GPU operation of the method (DSMC
steps, sampling, closure, synthetic solve, particle modification, network
inference); the error evaluation is excluded.
"""
from __future__ import annotations

import collections
import time

import torch

from .dig import DIG
from .dsmc import DSMC


def centreline(f: torch.Tensor, nx: int, ny: int, points: int, columns: int = 2,
               w: dict | None = None) -> torch.Tensor:
    """u_x of the `columns` centre columns, averaged across them and over
    `points` equal blocks along y.  On a graded grid (w given, geometry
    "graded") the columns are averaged with their widths and each block
    averages the cells it overlaps, weighted by the overlap, so that profiles
    of different grids compare at the same y blocks."""
    h = columns // 2
    if w is None or w.get("geometry") != "graded":
        ux = f[1].view(ny, nx)[:, nx // 2 - h: nx // 2 + h].mean(1)
        return ux.view(points, ny // points).mean(1)
    fx = torch.tensor(w["xfaces"], dtype=torch.float64, device=f.device)
    fy = torch.tensor(w["yfaces"], dtype=torch.float64, device=f.device)
    cw = (fx[1:] - fx[:-1])[nx // 2 - h: nx // 2 + h]
    ux = (f[1].view(ny, nx)[:, nx // 2 - h: nx // 2 + h] * cw).sum(1) / cw.sum()
    L = float(fy[-1])
    b = torch.linspace(0.0, L, points + 1, dtype=torch.float64, device=f.device)
    lo = torch.maximum(b[:-1, None], fy[None, :-1])
    hi = torch.minimum(b[1:, None], fy[None, 1:])
    wgt = (hi - lo).clamp(min=0.0)           # [points, ny] overlap lengths
    return (wgt * ux[None, :]).sum(1) / wgt.sum(1)


def _tune(sim: DSMC, tuning: dict | None):
    """Applies a launch configuration (results do not depend on it)."""
    if tuning:
        sim.tuning(**{k: tuning[k] for k in ("group_particles", "group_cells", "seq_max",
                                             "big_stage_kib")})


def reference_profile(w: dict, transient: int, average: int, points: int,
                      columns: int = 2, tuning: dict | None = None,
                      progress=None, chunk: int = 5000) -> torch.Tensor:
    """Plain DSMC from rest: `transient` steps, then the average of `average`
    (run in chunks of `chunk` steps, `progress(message)` after each; the state
    does not depend on the chunking)."""
    sim = DSMC(w)
    _tune(sim, tuning)
    sim.init()

    def run(n, what):
        done = 0
        while done < n:
            k = min(chunk, n - done)
            sim.step(k, graph=True)
            done += k
            if progress is not None:
                torch.cuda.synchronize()
                progress(f"reference {what}: {done} of {n} steps")

    run(transient, "transient")
    sim.reset_average()
    run(average, "average")
    f = sim.sample("average")
    return centreline(f, w["nx"], w["ny"], points, columns)


class Tracker:
    def __init__(self, ref: torch.Tensor, window: int, threshold: float):
        self.ref = ref
        self.range = float(ref.max() - ref.min())
        self.buf = collections.deque(maxlen=window)
        self.threshold = threshold
        # (wall seconds, steps, RMS error, largest pointwise error), both
        # relative to the reference profile's range
        self.history = []

    def add(self, prof: torch.Tensor, wall: float, steps: int):
        self.buf.append(prof)
        if len(self.buf) < self.buf.maxlen:
            return None
        avg = torch.stack(list(self.buf)).mean(0)
        err = float(((avg - self.ref) ** 2).mean().sqrt()) / self.range
        err_max = float((avg - self.ref).abs().max()) / self.range
        self.history.append((wall, steps, err, err_max))
        return err

    def time_to_steady(self, threshold: float | None = None, metric: str = "rms"):
        """(wall, steps) of the first point after which the error ("rms" or
        "max") stays <= threshold (the tracker's own by default)."""
        thr = self.threshold if threshold is None else threshold
        k = 2 if metric == "rms" else 3
        t = None
        for h in self.history:
            wall, steps, err = h[0], h[1], h[k]
            if err <= thr:
                if t is None:
                    t = (wall, steps)
            else:
                t = None
        return t


def run_plain(w, ref, ns, max_cycles, window, threshold, points, columns=2, tuning=None):
    # construction and particle initialisation count, as they do for DIG
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim = DSMC(w)
    _tune(sim, tuning)
    sim.init()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tr = Tracker(ref, window, threshold)
    for k in range(max_cycles):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.reset_average()
        sim.step(ns, graph=True)
        f = sim.sample("average")
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        tr.add(centreline(f, w["nx"], w["ny"], points, columns, w), wall, (k + 1) * ns)
        if _settled(tr, window):
            break
    return tr


def run_dig(w, ref, max_cycles, window, threshold, points, closure=None, columns=2,
            tuning=None, **kw):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d = DIG(w, closure=closure, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0  # NSF initialisation counts
    _tune(d.sim, tuning)
    tr = Tracker(ref, window, threshold)
    for k in range(max_cycles):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = d.cycle()
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        tr.add(centreline(f, w["nx"], w["ny"], points, columns, w), wall, (k + 1) * d.ns)
        if _settled(tr, window):
            break
    return tr, d


def _settled(tr: Tracker, window: int) -> bool:
    """Stop once the error has stayed below the threshold for 4 windows."""
    h = tr.history
    need = 4 * window
    return len(h) >= need and all(e[2] <= tr.threshold for e in h[-need:])
