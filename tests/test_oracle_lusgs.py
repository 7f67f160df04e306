"""Pins of the implicit (LU-SGS) synthetic-equation oracle.

LU-SGS changes how the pseudo-time iterations approach the steady state, not
the steady discrete equations: its converged state must be the explicit
scheme's (same residual R = 0), to 1e-8, with higher-order terms and a mask,
in both wall modes.  It also reproduces the closed forms (Fourier
conduction, Couette flow) along x and along y, keeps the initial total mass
exactly, and needs fewer iterations than the explicit scheme.
Mistakes in the approximate implicit operator only slow it down or stop it
from converging: a viscous cavity and a supersonic periodic box (where the
inviscid off-diagonal terms dominate) bound the iteration counts, and each
mistake in PLANTED must break one of those bounds or the agreement with the
explicit state."""
import types

import numpy as np
import pytest

import dig_workloads as wl
from oracle import synth

PER = ("periodic", 1.0, (0.0, 0.0, 0.0))


def _fields(nc, T=1.0):
    m = np.zeros((20, nc))
    m[0] = 1.0
    m[4] = T
    m[5] = T
    return m


def _cavity_case(n=8, seed=3, kn=0.05):
    w = wl.cavity_2d(n=n, kn=kn)
    rng = np.random.default_rng(seed)
    nc = n * n
    m = _fields(nc)
    m[0] = 1.0 + 0.05 * rng.standard_normal(nc)
    m[1:4] = 0.05 * rng.standard_normal((3, nc))
    m[4] = 1.0 + 0.03 * rng.standard_normal(nc)
    m[5] = 1.0 + 0.03 * rng.standard_normal(nc)
    hot = 0.003 * rng.standard_normal((12, nc))
    mask = (rng.random(nc) < 0.3).astype(np.uint8)
    return w, m, hot, mask


def agreement(S=synth, wall_mode="dsmc"):
    """(largest difference from the explicit steady state, LU-SGS iterations)."""
    w, m, hot, mask = _cavity_case()
    ref, it_e, ch_e = synth.solve(w, m, hot=hot, mask=mask, max_iter=200000, tol=1e-13,
                                  cfl=0.8, wall_mode=wall_mode)
    assert ch_e < 1e-13
    out, it, ch = S.solve_lusgs(w, m, hot=hot, mask=mask, max_iter=5000, tol=1e-13,
                                wall_mode=wall_mode)
    if not ch < 1e-13:
        return np.inf, it
    return np.abs(out - ref).max(), it


@pytest.mark.parametrize("wall_mode", ["dsmc", "wall"])
def test_converged_state_equals_the_explicit_scheme(wall_mode):
    diff, it = agreement(wall_mode=wall_mode)
    assert diff < 1e-8, diff
    assert it < 800, it


def convective(S=synth):
    """A periodic box with a Mach 1.6 mean flow at Kn = 0.001 (inviscid
    fluxes dominate): (converged, iterations, largest deviation of the
    result from uniform).  The steady states of a periodic box are uniform."""
    n = 16
    w = wl.box(2, n, n, kn=1e-3, bc=[PER] * 4)
    rng = np.random.default_rng(4)
    m = _fields(n * n)
    m[0] += 0.02 * rng.standard_normal(n * n)
    m[1] = 1.5 + 0.02 * rng.standard_normal(n * n)
    m[2] = 0.5 + 0.02 * rng.standard_normal(n * n)
    m[4] += 0.02 * rng.standard_normal(n * n)
    m[5] = m[4]
    with np.errstate(all="ignore"):
        out, it, ch = S.solve_lusgs(w, m, max_iter=1500, tol=1e-10)
    dev = np.abs(out - out.mean(axis=1, keepdims=True)).max()
    return bool(ch < 1e-10), it, dev


def test_convective_box_converges_to_a_uniform_state():
    ok, it, dev = convective()
    assert ok and dev < 1e-8, (it, dev)


def test_fourier_closed_form_along_x_and_y():
    w = wl.fourier_1d(nx=20)
    out, it, ch = synth.solve_lusgs(w, _fields(20, T=1.25), max_iter=5000, tol=1e-12,
                                    wall_mode="wall")
    assert ch < 1e-12
    xc = (np.arange(20) + 0.5) / 20
    T = out[4]
    Tp = T ** (1.0 + wl.OMEGA_N2)
    fit = np.polyfit(xc, Tp, 1)
    assert np.abs(Tp - np.polyval(fit, xc)).max() < 2e-5 * (Tp.max() - Tp.min())
    assert np.abs(T - out[5]).max() < 1e-8 and np.abs(out[1:4]).max() < 1e-7
    assert abs(out[0].mean() - 1.0) < 1e-13
    bc = [PER, PER, ("diffuse", 1.0, (0, 0, 0)), ("diffuse", 1.5, (0, 0, 0))]
    w2 = wl.box(2, 2, 20, kn=0.05, bc=bc)
    out2, it2, ch2 = synth.solve_lusgs(w2, _fields(40, T=1.25), max_iter=5000, tol=1e-12,
                                       wall_mode="wall")
    assert ch2 < 1e-12
    np.testing.assert_allclose(out2[4].reshape(20, 2)[:, 0], T, rtol=1e-9)


def test_couette_closed_form_along_y():
    U = 0.02
    bc = [PER, PER, ("diffuse", 1.0, (-U, 0, 0)), ("diffuse", 1.0, (U, 0, 0))]
    w = wl.box(2, 2, 20, kn=0.05, bc=bc)
    out, it, ch = synth.solve_lusgs(w, _fields(40), max_iter=5000, tol=1e-12, wall_mode="wall")
    assert ch < 1e-12
    yc = (np.arange(20) + 0.5) / 20
    np.testing.assert_allclose(out[1].reshape(20, 2), (U * (2 * yc - 1))[:, None].repeat(2, 1),
                               atol=2e-6)


def test_total_mass_is_kept_every_iteration():
    w, m, hot, mask = _cavity_case(n=10, seed=8)
    for k in (1, 2, 7):
        out, it, ch = synth.solve_lusgs(w, m, hot=hot, mask=mask, max_iter=k, tol=0.0)
        assert it == k
        assert abs(out[0].sum() - m[0].sum()) <= 1e-13 * m[0].sum()


def test_fewer_iterations_than_explicit():
    """On this low-Mach viscous cavity LU-SGS needs about half the explicit
    iterations (measured 672 against 1290 to a change of 1e-6)."""
    w, m, hot, mask = _cavity_case(n=16, seed=2, kn=0.01)
    _, it_l, ch_l = synth.solve_lusgs(w, m, hot=hot, mask=mask, max_iter=20000, tol=1e-6)
    _, it_e, ch_e = synth.solve(w, m, hot=hot, mask=mask, max_iter=20000, tol=1e-6)
    assert ch_l < 1e-6 and ch_e < 1e-6
    assert 1.5 * it_l < it_e, (it_l, it_e)


def test_periodic_axis_with_odd_count_is_refused():
    w = wl.box(2, 5, 4, kn=0.05, bc=[PER] * 4)
    with pytest.raises(ValueError):
        synth.solve_lusgs(w, _fields(20), max_iter=1)


def variant(edits):
    text = open(synth.__file__, encoding="utf-8").read()
    for old, new in edits:
        assert text.count(old) == 1, old
        text = text.replace(old, new)
    mod = types.ModuleType("synth_variant")
    exec(compile(text, "synth_variant", "exec"), mod.__dict__)
    return mod


PLANTED = {
    "neighbour_flux_sign": ("t = side * dF - r[a] * dW", "t = -side * dF - r[a] * dW"),
    "upper_sweep_sign": ("dW[:, first] = dW[:, first] - corr[:, first] / D[:, first]",
                         "dW[:, first] = dW[:, first] + corr[:, first] / D[:, first]"),
    "viscous_radius_dropped": ("r = {a: np.abs(u[a]) + c + 2.0 * nu / h[a] for a in axes}",
                               "r = {a: np.abs(u[a]) + c for a in axes}"),
    "same_colour_order": ("first = ((ii + jj) % 2 == 0)", "first = (ii >= 0)"),
}


@pytest.mark.parametrize("name", list(PLANTED))
def test_planted_mistake_is_caught(name):
    S = variant([PLANTED[name]])
    with np.errstate(all="ignore"):
        diff, it = agreement(S)
    viscous_ok = diff < 1e-8 and it < 800
    conv_ok, it_c, dev = convective(S)
    assert not (viscous_ok and conv_ok and dev < 1e-8), (name, diff, it, it_c, dev)
