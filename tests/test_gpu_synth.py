"""GPU synthetic-equation solve vs its FP64 oracle (same scheme, same number
of pseudo-time steps), and the converged 1D Fourier closed form on the GPU."""
import numpy as np
import pytest
import torch

import dig_workloads as wl
from gpu_common import np_, say
from oracle import synth
from paper_2501_10965_amd.dsmc import synth_solve

pytestmark = pytest.mark.gpu


def _case2d(n=10, seed=3):
    w = wl.cavity_2d(n=n, kn=0.05)
    rng = np.random.default_rng(seed)
    nc = n * n
    m = np.zeros((20, nc))
    m[0] = 1.0 + 0.05 * rng.standard_normal(nc)
    m[1] = 0.05 * rng.standard_normal(nc)
    m[2] = 0.05 * rng.standard_normal(nc)
    m[4] = 1.0 + 0.03 * rng.standard_normal(nc)
    m[5] = 1.0 + 0.03 * rng.standard_normal(nc)
    hot = 0.005 * rng.standard_normal((12, nc))
    mask = (rng.random(nc) < 0.3).astype(np.uint8)
    return w, m, hot, mask


@pytest.mark.parametrize("mode", ["dsmc", "wall"])
def test_synth_matches_oracle_fixed_steps(mode):
    w, m, hot, mask = _case2d()
    say(f"case synth 2d {mode}")
    ref, it, _ = synth.solve(w, m, hot=hot, mask=mask, max_iter=300, tol=0.0, wall_mode=mode)
    out, git, _ = synth_solve(w, torch.tensor(m, device="cuda"), torch.tensor(hot, device="cuda"),
                              torch.tensor(mask, device="cuda"), max_iter=300, tol=0.0,
                              wall_mode=mode)
    assert git == 300 and it == 300
    g = np_(out)
    np.testing.assert_allclose(g, ref, rtol=1e-9, atol=1e-12)
    assert abs(g[0].sum() - m[0].sum()) <= 1e-12 * m[0].sum()


def test_synth_full_grid_matches_oracle_on_every_call():
    """The 200 x 200 cavity grid (157 workgroups per launch).  The first
    pseudo-time step is the minimum of the cells' step bounds over the whole
    grid, so every call agrees with the oracle, whatever order the workgroups
    run in."""
    w, m, hot, mask = _case2d(n=200, seed=5)
    say("case synth full grid")
    ref, it, _ = synth.solve(w, m, hot=hot, mask=mask, max_iter=4, tol=0.0, wall_mode="dsmc")
    args = [torch.tensor(a, device="cuda") for a in (m, hot, mask)]
    for rep in range(3):
        out, git, _ = synth_solve(w, *args, max_iter=4, tol=0.0, wall_mode="dsmc")
        assert git == 4 and it == 4
        np.testing.assert_allclose(np_(out), ref, rtol=1e-9, atol=1e-12)


def test_synth_fourier_converges_to_closed_form():
    w = wl.fourier_1d(nx=32)
    say("case synth fourier")
    m = np.zeros((20, 32))
    m[0] = 1.0
    m[4:6] = 1.25
    out, it, ch = synth_solve(w, torch.tensor(m, device="cuda"), max_iter=400000, tol=1e-12,
                              wall_mode="wall", cfl=0.8)
    assert ch < 1e-12 and it < 400000
    g = np_(out)
    T, Tr = g[4], g[5]
    xc = (np.arange(32) + 0.5) / 32
    assert np.abs(T - Tr).max() < 1e-8
    assert np.abs(g[1:4]).max() < 1e-7
    Tp = T ** 1.74
    fit = np.polyfit(xc, Tp, 1)
    assert np.abs(Tp - np.polyval(fit, xc)).max() < 2e-5 * (Tp.max() - Tp.min())
