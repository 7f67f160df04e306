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


# ---------------------------------------------------------------------------
# implicit LU-SGS scheme


@pytest.mark.parametrize("mode,iters", [("dsmc", 1), ("dsmc", 60), ("wall", 60)])
def test_lusgs_matches_oracle_fixed_steps(mode, iters):
    w, m, hot, mask = _case2d()
    say(f"case lusgs 2d {mode} {iters}")
    ref, it, _ = synth.solve_lusgs(w, m, hot=hot, mask=mask, max_iter=iters, tol=0.0,
                                   wall_mode=mode)
    out, git, _ = synth_solve(w, torch.tensor(m, device="cuda"), torch.tensor(hot, device="cuda"),
                              torch.tensor(mask, device="cuda"), max_iter=iters, tol=0.0,
                              wall_mode=mode, scheme="lusgs")
    assert git == iters and it == iters
    g = np_(out)
    np.testing.assert_allclose(g, ref, rtol=1e-9, atol=1e-12)
    assert abs(g[0].sum() - m[0].sum()) <= 1e-12 * m[0].sum()


def test_lusgs_full_grid_and_odd_ragged_grids_match_oracle():
    """The 200 x 200 cavity (157 workgroups), a ragged 37 x 23 box and a 1D
    slab, a few implicit steps each."""
    cases = [(_case2d(n=200, seed=5), 3, "dsmc")]
    w, m, hot, mask = _case2d(n=24, seed=9)
    w2 = wl.box(2, 37, 23, lx=1.0, ly=0.62, kn=0.02, bc=w["bc"])
    rng = np.random.default_rng(11)
    m2 = np.zeros((20, 37 * 23))
    m2[0] = 1.0 + 0.04 * rng.standard_normal(37 * 23)
    m2[1:3] = 0.05 * rng.standard_normal((2, 37 * 23))
    m2[4:6] = 1.0 + 0.03 * rng.standard_normal((2, 37 * 23))
    cases.append(((w2, m2, 0.004 * rng.standard_normal((12, 37 * 23)),
                   (rng.random(37 * 23) < 0.5).astype(np.uint8)), 25, "wall"))
    w1 = wl.fourier_1d(nx=45)
    m1 = np.zeros((20, 45))
    m1[0] = 1.0
    m1[4:6] = 1.2 + 0.01 * rng.standard_normal((2, 45))
    cases.append(((w1, m1, None, None), 25, "wall"))
    for (wc, mc, hc, kc), iters, mode in cases:
        say(f"case lusgs {wc['nx']}x{wc.get('ny', 1)} {iters}")
        ref, it, _ = synth.solve_lusgs(wc, mc, hot=hc, mask=kc, max_iter=iters, tol=0.0,
                                       wall_mode=mode)
        args = [torch.tensor(a, device="cuda") if a is not None else None for a in (mc, hc, kc)]
        out, git, _ = synth_solve(wc, *args, max_iter=iters, tol=0.0, wall_mode=mode,
                                  scheme="lusgs")
        assert git == iters
        np.testing.assert_allclose(np_(out), ref, rtol=1e-9, atol=1e-12)


def test_lusgs_converges_to_the_explicit_steady_state():
    w, m, hot, mask = _case2d(n=12, seed=4)
    say("case lusgs vs explicit steady state")
    args = [torch.tensor(a, device="cuda") for a in (m, hot, mask)]
    a, ita, cha = synth_solve(w, *args, max_iter=200000, tol=1e-12, cfl=0.8, check_every=256)
    b, itb, chb = synth_solve(w, *args, max_iter=20000, tol=1e-12, scheme="lusgs",
                              check_every=16)
    assert cha < 1e-12 and chb < 1e-12 and itb < ita
    np.testing.assert_allclose(np_(b), np_(a), rtol=1e-8, atol=1e-10)
