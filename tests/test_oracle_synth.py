"""Oracle pins for the synthetic-equation solve: closed-form steady solutions
(Fourier conduction, isothermal Couette flow), exact mass conservation, and
invariance under a divergence-free (uniform) higher-order term."""
import numpy as np

import dig_workloads as wl
from oracle import synth


def _fields(nc, rho=1.0, T=1.25, uy=None):
    m = np.zeros((20, nc))
    m[0] = rho
    m[4] = T
    m[5] = T
    if uy is not None:
        m[2] = uy
    return m


def test_fourier_steady_state_closed_form():
    """HoT = 0, walls 1.0 / 1.5: u = 0, uniform p, Tr = Tt, and T^(1+w)
    linear because kappa_t and kappa_r both scale with mu ~ T^w."""
    w = wl.fourier_1d(nx=20)
    out, it, ch = synth.solve(w, _fields(20), max_iter=100000, tol=1e-12, wall_mode="wall",
                              cfl=0.8)
    assert ch < 1e-12
    T, Tr = out[4], out[5]
    xc = (np.arange(20) + 0.5) / 20
    assert np.abs(T - Tr).max() < 1e-8
    assert np.abs(out[1:4]).max() < 1e-7
    p = out[0] * T
    assert (p.max() - p.min()) / p.mean() < 1e-7
    Tp = T ** 1.74
    fit = np.polyfit(xc, Tp, 1)
    assert np.abs(Tp - np.polyval(fit, xc)).max() < 2e-5 * (Tp.max() - Tp.min())
    # the wall values bound the profile
    assert 1.0 < T.min() < T.max() < 1.5
    assert abs(out[0].mean() - 1.0) < 1e-13  # mass of the initial field


def test_isothermal_couette_linear_velocity():
    U = 0.02
    bc = [("diffuse", 1.0, (0, -U, 0)), ("diffuse", 1.0, (0, U, 0)), ("periodic", 1, (0, 0, 0)),
          ("periodic", 1, (0, 0, 0))]
    w = wl.box(1, 20, kn=0.05, bc=bc)
    out, it, ch = synth.solve(w, _fields(20, T=1.0), max_iter=100000, tol=1e-12,
                              wall_mode="wall", cfl=0.8)
    xc = (np.arange(20) + 0.5) / 20
    uy = out[2]
    np.testing.assert_allclose(uy, U * (2 * xc - 1), atol=2e-6 * U / U)
    assert np.abs(out[4] - 1.0).max() < 5e-3 * U / 0.02  # viscous heating is O(U^2)


def _cavity_case(n=8, seed=3):
    w = wl.cavity_2d(n=n, kn=0.05)
    rng = np.random.default_rng(seed)
    nc = n * n
    m = _fields(nc, T=1.0)
    m[0] = 1.0 + 0.05 * rng.standard_normal(nc)
    m[1] = 0.05 * rng.standard_normal(nc)
    m[2] = 0.05 * rng.standard_normal(nc)
    m[4] = 1.0 + 0.03 * rng.standard_normal(nc)
    m[5] = 1.0 + 0.03 * rng.standard_normal(nc)
    hot = 0.005 * rng.standard_normal((12, nc))
    return w, m, hot


def test_mass_is_conserved_exactly():
    w, m, hot = _cavity_case()
    out, it, ch = synth.solve(w, m, hot=hot, max_iter=300, tol=0.0)
    assert it == 300
    assert abs(out[0].sum() - m[0].sum()) <= 1e-12 * m[0].sum()


def test_uniform_hot_is_divergence_free():
    """A spatially uniform higher-order term adds the same flux on every face,
    so it must not change the solution (it cancels in every cell)."""
    w = wl.fourier_1d(nx=12)
    hot = np.zeros((12, 12))
    hot[6] = 0.01   # q_t,x
    hot[9] = -0.02  # q_r,x
    hot[3] = 0.003  # sigma_xy
    a, *_ = synth.solve(w, _fields(12), max_iter=400, tol=0.0, wall_mode="wall")
    b, *_ = synth.solve(w, _fields(12), hot=hot, max_iter=400, tol=0.0, wall_mode="wall")
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)
    # a masked HoT field is the NSF solution
    bump = np.zeros((12, 12))
    bump[6, 5] = 0.05
    c, *_ = synth.solve(w, _fields(12), hot=bump, mask=np.ones(12, np.uint8), max_iter=400,
                        tol=0.0, wall_mode="wall")
    np.testing.assert_allclose(a, c, rtol=1e-14, atol=1e-15)
    d, *_ = synth.solve(w, _fields(12), hot=bump, max_iter=400, tol=0.0, wall_mode="wall")
    assert np.abs(d - a).max() > 1e-6
