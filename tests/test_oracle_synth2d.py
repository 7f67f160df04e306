"""Pins of the synthetic-equation oracle in two dimensions (equation
macroscopic_equation with the closure of equations ns_constitutive, kappa_A,
full_constitutive).

* Closed forms along y: steady Fourier conduction between walls at
  y = 0 and y = 1 (T^(1+omega) linear, Tr = Tt, uniform pressure, no flow) and
  isothermal Couette flow (u_x linear in y).
* Face fluxes on linear fields: central and one-sided differences are exact
  there, so the viscous part of every interior face flux (total flux minus
  the flux of the same fields with zero viscosity) equals the NSF stress,
  the work term sigma.u and the two heat fluxes evaluated at the face centre.
* Equivariance: a field rotated by 90 degrees (scalars moved, vectors and the
  higher-order stress and heat-flux terms rotated, walls permuted) gives the
  rotated solution.
* A uniform flow on a periodic box is steady, and a periodic box conserves
  mass, momentum and total energy to rounding.

PLANTED lists plausible mistakes; each is applied to a copy of the oracle
module and must fail at least one of these checks.
"""
import types

import numpy as np
import pytest

import dig_workloads as wl
from oracle import synth

OMEGA = wl.OMEGA_N2
PER = ("periodic", 1.0, (0.0, 0.0, 0.0))


def _fields(nc, rho=1.0, T=1.25):
    m = np.zeros((20, nc))
    m[0] = rho
    m[4] = T
    m[5] = T
    return m


# ------------------------------------------------------------------ closed forms
def fourier_y_error(S=synth):
    """Deviation from the closed form of steady conduction along y."""
    bc = [PER, PER, ("diffuse", 1.0, (0, 0, 0)), ("diffuse", 1.5, (0, 0, 0))]
    w = wl.box(2, 3, 20, kn=0.05, bc=bc)
    out, it, ch = S.solve(w, _fields(60), max_iter=20000, tol=1e-12, wall_mode="wall", cfl=0.8)
    T = out[4].reshape(20, 3)
    Tr = out[5].reshape(20, 3)
    yc = (np.arange(20) + 0.5) / 20
    p = (out[0] * out[4]).reshape(20, 3)
    Tp = T[:, 0] ** (1.0 + OMEGA)
    fit = np.polyfit(yc, Tp, 1)
    errs = [
        0.0 if ch < 1e-12 else 1.0,
        np.abs(T - Tr).max() / 1e-8,
        np.abs(out[1:4]).max() / 1e-7,
        (p.max() - p.min()) / p.mean() / 1e-7,
        np.abs(Tp - np.polyval(fit, yc)).max() / (2e-5 * (Tp.max() - Tp.min())),
        np.abs(T - T[:, :1]).max() / 1e-13,
        0.0 if 1.0 < T.min() < T.max() < 1.5 else 1.0,
        abs(out[0].mean() - 1.0) / 1e-13,
    ]
    return max(errs)  # below 1 when every closed-form property holds


def test_fourier_along_y_closed_form():
    assert fourier_y_error() < 1.0


def couette_y_error(S=synth):
    U = 0.02
    bc = [PER, PER, ("diffuse", 1.0, (-U, 0, 0)), ("diffuse", 1.0, (U, 0, 0))]
    w = wl.box(2, 2, 20, kn=0.05, bc=bc)
    out, it, ch = S.solve(w, _fields(40, T=1.0), max_iter=20000, tol=1e-12, wall_mode="wall",
                          cfl=0.8)
    yc = (np.arange(20) + 0.5) / 20
    ux = out[1].reshape(20, 2)
    return max(np.abs(ux - (U * (2 * yc - 1))[:, None]).max() / 2e-6,
               np.abs(out[2]).max() / 1e-9,
               np.abs(out[4] - 1.0).max() / 5e-3,
               0.0 if ch < 1e-12 else 1.0)


def test_couette_along_y_linear_velocity():
    assert couette_y_error() < 1.0


# ------------------------------------------------------------------ face fluxes
NXF, NYF, LXF, LYF = 6, 5, 1.0, 1.3
G = np.array([[0.3, -0.2], [0.45, 0.1], [-0.3, 0.7]])   # d u_i / d x_j, i = x, y, z
U0 = np.array([0.5, -0.2, 0.1])
GT, GR = np.array([0.2, -0.1]), np.array([-0.05, 0.3])
A_EUCKEN = (2.0 / 3.0, 0.0, 0.0, 5.0 / (7.0 - 2.0 * OMEGA))


def _flux_workload(kn):
    walls = [("diffuse", 1.0, (0, 0, 0))] * 4
    return wl.box(2, NXF, NYF, lx=LXF, ly=LYF, kn=kn, bc=walls)


def _linear_state(x, y):
    x, y = np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64)
    u = np.stack([U0[i] + G[i, 0] * x + G[i, 1] * y for i in range(3)])
    return u, 1.0 + GT[0] * x + GT[1] * y, 0.9 + GR[0] * x + GR[1] * y


def flux_error(S=synth):
    """Largest deviation of the interior viscous face fluxes from the closed
    form, relative to the largest closed-form entry."""
    kn = 0.05
    k = np.arange(NXF * NYF)
    xc, yc = (k % NXF + 0.5) * LXF / NXF, (k // NXF + 0.5) * LYF / NYF
    u, tt, tr = _linear_state(xc, yc)
    f = _fields(NXF * NYF)
    f[1:4], f[4], f[5] = u, tt, tr
    mu0 = kn * np.sqrt(2.0 / np.pi)
    worst = 0.0
    for axis in (0, 1):
        V = S.face_fluxes(_flux_workload(kn), f, axis, A=A_EUCKEN) - \
            S.face_fluxes(_flux_workload(0.0), f, axis, A=A_EUCKEN)
        if axis == 0:
            ii, jj = np.meshgrid(np.arange(1, NXF), np.arange(NYF))
            xf, yf = ii * LXF / NXF, (jj + 0.5) * LYF / NYF
            Vi = V[:, :, 1:NXF]
        else:
            ii, jj = np.meshgrid(np.arange(NXF), np.arange(1, NYF))
            xf, yf = (ii + 0.5) * LXF / NXF, jj * LYF / NYF
            Vi = V[:, 1:NYF, :]
        uf, tf, _ = _linear_state(xf, yf)
        mu = mu0 * tf ** OMEGA
        kt, kr = 15.0 / 4.0 * mu, (7.0 - 2.0 * OMEGA) / 5.0 * mu
        g3 = np.zeros((3, 3))
        g3[:, :2] = G
        div = G[0, 0] + G[1, 1]
        sig = [-mu * (g3[axis, j] + g3[j, axis] - (2.0 / 3.0 * div if j == axis else 0.0))
               for j in range(3)]
        ref = np.zeros_like(Vi)
        for j in range(3):
            ref[1 + j] = sig[j]
        qt, qr = -kt * GT[axis], -kr * GR[axis]
        ref[4] = sig[0] * uf[0] + sig[1] * uf[1] + sig[2] * uf[2] + qt + qr
        ref[5] = qr
        worst = max(worst, np.abs(Vi - ref).max() / np.abs(ref).max())
    return worst


def test_interior_face_fluxes_equal_closed_form():
    assert flux_error() < 1e-12


# ------------------------------------------------------------------ equivariance
def _rotate(m, hot, n):
    """Rotation by +90 degrees about the centre of the unit square:
    (x, y) -> (1 - y, x); cell (i, j) -> (n - 1 - j, i)."""
    i, j = np.meshgrid(np.arange(n), np.arange(n))   # [j][i]
    src = (j * n + i).ravel()                        # old cell index of each (j, i)
    dst = (i * n + (n - 1 - j)).ravel()              # its new index
    mr = np.zeros_like(m)
    mr[:, dst] = m[:, src]
    ux, uy = mr[1].copy(), mr[2].copy()
    mr[1], mr[2] = -uy, ux
    hr = None
    if hot is not None:
        h = np.zeros_like(hot)
        h[:, dst] = hot[:, src]
        hr = h.copy()
        hr[0], hr[1], hr[3] = h[1], h[0], -h[3]          # xx, yy, xy
        hr[4], hr[5] = -h[5], h[4]                       # (xz, yz) as a vector
        hr[6], hr[7] = -h[7], h[6]                       # q_t
        hr[9], hr[10] = -h[10], h[9]                     # q_r
    return mr, hr


def _rotated_walls(bc):
    rot = lambda U: (-U[1], U[0], U[2])
    # old x- -> new y-, old x+ -> new y+, old y- -> new x+, old y+ -> new x-
    return [(bc[3][0], bc[3][1], rot(bc[3][2])), (bc[2][0], bc[2][1], rot(bc[2][2])),
            (bc[0][0], bc[0][1], rot(bc[0][2])), (bc[1][0], bc[1][1], rot(bc[1][2]))]


def rotation_error(S=synth, wall_mode="dsmc"):
    n = 8
    rng = np.random.default_rng(11)
    bc = [("diffuse", 1.1, (0, 0.05, 0)), ("diffuse", 0.9, (0, -0.02, 0.01)),
          ("diffuse", 1.0, (0.03, 0, 0)), ("diffuse", 1.2, (0.3, 0, -0.01))]
    w = wl.box(2, n, n, kn=0.05, bc=bc)
    wr = wl.box(2, n, n, kn=0.05, bc=_rotated_walls(bc))
    m = _fields(n * n, T=1.0)
    m[0] = 1.0 + 0.05 * rng.standard_normal(n * n)
    m[1:4] = 0.1 * rng.standard_normal((3, n * n))
    m[4] = 1.0 + 0.05 * rng.standard_normal(n * n)
    m[5] = 1.0 + 0.05 * rng.standard_normal(n * n)
    hot = 0.004 * rng.standard_normal((12, n * n))
    hot[2] = -(hot[0] + hot[1])
    hot[8] = hot[11] = 0.0
    mask = (rng.random(n * n) < 0.3).astype(np.uint8)
    out, *_ = S.solve(w, m, hot=hot, mask=mask, max_iter=60, tol=0.0, wall_mode=wall_mode)
    mr, hr = _rotate(m, hot, n)
    maskr = np.zeros_like(mask)
    maskr[:] = _rotate(mask[None, :].astype(float).repeat(20, 0), None, n)[0][0]
    outr, *_ = S.solve(wr, mr, hot=hr, mask=maskr, max_iter=60, tol=0.0, wall_mode=wall_mode)
    expect, _ = _rotate(np.vstack([out, np.zeros((14, n * n))]), None, n)
    return np.abs(outr - expect[:6]).max()


@pytest.mark.parametrize("wall_mode", ["dsmc", "wall"])
def test_rotation_by_90_degrees(wall_mode):
    assert rotation_error(wall_mode=wall_mode) < 1e-12


# ------------------------------------------------------------------ periodic box
def _periodic(n=8):
    return wl.box(2, n, n, kn=0.05, bc=[PER] * 4)


def test_uniform_flow_is_steady():
    n = 8
    m = _fields(n * n, rho=1.3, T=1.1)
    m[1], m[2], m[3] = 0.3, -0.2, 0.1
    out, it, ch = synth.solve(_periodic(n), m, max_iter=30, tol=0.0)
    np.testing.assert_allclose(out, m[:6], rtol=1e-14, atol=1e-15)


def _totals(out, dr=2):
    rho, u, tt, tr = out[0], out[1:4], out[4], out[5]
    E = rho * (0.5 * (3 * tt + dr * tr) + 0.5 * (u ** 2).sum(axis=0))
    return np.array([rho.sum(), *(rho * u).sum(axis=1), E.sum()])


def conservation_error(S=synth):
    n = 8
    rng = np.random.default_rng(5)
    m = _fields(n * n, T=1.0)
    m[0] = 1.0 + 0.05 * rng.standard_normal(n * n)
    m[1:4] = 0.1 * rng.standard_normal((3, n * n))
    m[4] = 1.0 + 0.05 * rng.standard_normal(n * n)
    m[5] = 1.0 + 0.08 * rng.standard_normal(n * n)
    hot = 0.004 * rng.standard_normal((12, n * n))
    out, *_ = S.solve(_periodic(n), m, hot=hot, max_iter=200, tol=0.0)
    a, b = _totals(m[:6]), _totals(out)
    scale = np.array([a[0], a[0], a[0], a[0], a[4]])
    return np.abs(b - a).max() / 1e-12 / scale.min()


def test_periodic_box_conserves_mass_momentum_energy():
    assert conservation_error() < 1.0


# ------------------------------------------------------------------ planted mistakes
def variant(edits):
    """A copy of the synthetic-solve oracle with textual edits applied."""
    text = open(synth.__file__, encoding="utf-8").read()
    for old, new in edits:
        assert text.count(old) == 1, old
        text = text.replace(old, new)
    mod = types.ModuleType("synth_variant")
    exec(compile(text, "synth_variant", "exec"), mod.__dict__)
    return mod


PLANTED = {
    "tangential_axis_swapped": (
        "dt_ = [0.5 * (dul[i][1 - axis] + dur[i][1 - axis]) for i in range(3)]",
        "dt_ = [0.5 * (dul[i][axis] + dur[i][axis]) for i in range(3)]"),
    "work_term_dropped": (
        "V[4] = sig[0] * uf[0] + sig[1] * uf[1] + sig[2] * uf[2] + qt + qr",
        "V[4] = qt + qr"),
    "conductivity_factor_2": (
        "kt = 0.5 * mu * (arr * 5.0 - atr * dr) / det", "kt = mu * (arr * 5.0 - atr * dr) / det"),
    "y_plus_wall_from_y_minus_cells": (
        "            idx = (ny - 1, slice(None))", "            idx = (0, slice(None))"),
    "pressure_on_x_momentum_only": (
        "F[1 + k] = Wc[1 + k] * un + (p if k == axis else 0.0)",
        "F[1 + k] = Wc[1 + k] * un + (p if k == 0 else 0.0)"),
    "y_difference_with_x_spacing": (
        "            R -= (F[:, 1:, :] - F[:, :-1, :]) / h",
        "            R -= (F[:, 1:, :] - F[:, :-1, :]) / P[\"hx\"]"),
}


def _all_errors(S):
    return {"flux": flux_error(S) / 1e-12, "rot_dsmc": rotation_error(S, "dsmc") / 1e-12,
            "rot_wall": rotation_error(S, "wall") / 1e-12,
            "conservation": conservation_error(S)}


@pytest.mark.parametrize("name", list(PLANTED))
def test_planted_mistake_is_caught(name):
    S = variant([PLANTED[name]])
    errs = _all_errors(S)
    if max(errs.values()) < 1.0:  # the cheap checks pass: the closed forms must fail
        errs["fourier_y"] = fourier_y_error(S)
        errs["couette_y"] = couette_y_error(S)
    assert max(errs.values()) > 1.0, f"planted mistake {name} not caught: {errs}"
