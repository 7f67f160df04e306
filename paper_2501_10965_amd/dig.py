"""The DIG iteration (Section 3) on one GPU, driving the library's C ABI.

  1. initialise: solve the synthetic equations with the NSF closure from the
     workload's uniform field, then draw the particles from the local
     equilibrium of that solution;
  2. N_s DSMC steps with time averaging -> M^{n+1/2}; closure assembly gives
     the higher-order terms HoT^{n+1/2}, masked where Kn_GLL < Kn_ref;
  3. synthetic solve with the full closure (at most N_m pseudo-time steps or
     relative change below tol) -> M^{n+1};
  4. particle modification toward M^{n+1}.
Steps 2-4 repeat.  With mode="dsmc" the same driver runs plain DSMC (steps 2
only, same sampling), which is the reference the DIG gain is measured against.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from .dsmc import DSMC, synth_solve


def default_A(omega: float):
    """Heat-flux relaxation matrix whose conductivities are the modified Eucken
    values kappa_t = 15 mu / 4, kappa_r = (7 - 2 omega) mu / 5 (equation kappa_A);
    the paper notes A cannot be matched by the BL model in general."""
    return (2.0 / 3.0, 0.0, 0.0, 5.0 / (7.0 - 2.0 * omega))


def _cycle_change(new: torch.Tensor, old: torch.Tensor) -> float:
    """Relative change between two macroscopic solutions [>=6, C] (rows rho,
    ux, uy, uz, Tt, Tr), taken on the host: the larger of the L2 changes of
    the in-plane velocity and of Tt, each over its own norm."""
    a = new[0:6].double().cpu().numpy()
    b = old[0:6].double().cpu().numpy()
    du = np.linalg.norm(a[1:3] - b[1:3]) / max(np.linalg.norm(b[1:3]), 1e-300)
    dt = np.linalg.norm(a[4] - b[4]) / max(np.linalg.norm(b[4]), 1e-300)
    return float(max(du, dt))


class DIG:
    def __init__(self, w: dict, mode: str = "dig", ns: int = 50, n_m: int = 2000,
                 tol: float = 1e-5, kn_ref: float = 0.01, A=None, wall_mode: str = "dsmc",
                 closure=None, capacity: int | None = None, cfl: float | None = None,
                 nsf_init: bool = True, init_iters: int | None = None, graph: bool = True,
                 scheme: str = "explicit", n_min: float = 1.0, handoff: float | None = None,
                 **dsmc_kw):
        assert mode in ("dig", "dsmc")
        self.w = w
        self.mode = mode
        self.ns = ns
        self.n_m = n_m
        self.tol = tol
        self.kn_ref = kn_ref
        # cells holding on average fewer particles than this keep the NSF closure
        # (their extracted higher-order terms are sampling noise)
        self.n_min = n_min
        self.A = A if A is not None else default_A(w["omega"])
        self.wall_mode = wall_mode
        self.cfl = cfl  # None: the scheme's default
        self.scheme = scheme  # synthetic solve: "explicit" or "lusgs" (implicit)
        self.graph = graph
        # optional learned closure: (sim, fields, hot, mask, kn, smooth=...) -> hot, where
        # smooth holds the latest macroscopic solution in rows 0..5
        self.closure_fn = closure
        # hand-off: the change of the macroscopic solution between cycles
        # (relative L2 norm of the in-plane velocity or of the translational
        # temperature, the larger) falls while DIG converges and then levels
        # off at the level the sampling noise sets; once its mean over the last
        # HANDOFF_WINDOW cycles is above `handoff` times the mean over the
        # window before, later cycles are plain DSMC
        self.handoff = handoff
        self.handoff_at = None
        self.sim = DSMC(w, capacity=capacity, cap_factor=1.6, **dsmc_kw)
        self.ncell = self.sim.ncell
        self.cycle_no = 0
        self.log = []
        self._initialise(nsf_init, init_iters if init_iters is not None else n_m)

    def _initialise(self, nsf_init: bool, iters: int):
        f0 = self.sim.uniform_fields()
        m = torch.zeros((20, self.ncell), dtype=torch.float64, device=f0.device)
        m[0:6] = f0
        if nsf_init and self.mode == "dig":
            out, it, ch = synth_solve(self.w, m, None, None, self.A, cfl=self.cfl,
                                      wall_mode="wall", max_iter=iters, tol=self.tol,
                                      scheme=self.scheme)
            f0 = out
        # the latest macroscopic solution (inputs of a learned closure)
        self.m_prev = f0[0:6].clone()
        # counts by Iround(rho V / N_eff), equilibrium velocities, rotational energies
        self.sim.init(f0.contiguous(), ppc=0)

    HANDOFF_WINDOW = 10

    def _levelled_off(self) -> bool:
        ch = [r["cycle_change"] for r in self.log if "cycle_change" in r]
        n = self.HANDOFF_WINDOW
        if len(ch) < 2 * n:
            return False
        last, before = np.mean(ch[-n:]), np.mean(ch[-2 * n:-n])
        return last > self.handoff * before

    def cycle(self):
        """One DIG iteration (or N_s plain DSMC steps); returns the averaged field."""
        t0 = time.perf_counter()
        self.sim.reset_average()
        self.sim.step(self.ns, graph=self.graph)
        f = self.sim.sample("average")
        rec = {"cycle": self.cycle_no}
        if self.mode == "dig" and self.handoff_at is None:
            # cells left empty over the cycle start from the previous solution
            self.sim.fill_empty(f, self.m_prev)
            hot, mask, kn, _ = self.sim.closure(f, self.A, self.kn_ref, n_min=self.n_min)
            if self.closure_fn is not None:
                smooth = torch.zeros((20, self.ncell), dtype=torch.float64, device=f.device)
                smooth[0:6] = self.m_prev
                hot = self.closure_fn(self.sim, f, hot, mask, kn, smooth=smooth)
            m_next, it, ch = synth_solve(self.w, f, hot, mask, self.A, cfl=self.cfl,
                                         wall_mode=self.wall_mode, max_iter=self.n_m,
                                         tol=self.tol, scheme=self.scheme)
            self.sim.adjust(m_next, self.cycle_no)
            change = _cycle_change(m_next, self.m_prev)
            self.m_prev = m_next
            rec.update(synth_iters=it, synth_change=ch, cycle_change=change,
                       eq_fraction=float(mask.double().mean().item()))
        torch.cuda.synchronize()
        rec["seconds"] = time.perf_counter() - t0
        self.log.append(rec)
        if self.mode == "dig" and self.handoff is not None and self.handoff_at is None and \
                self._levelled_off():
            self.handoff_at = self.cycle_no
        self.cycle_no += 1
        return f
