"""Closed-form pins of the oracle's gradient-length local Knudsen number
(Section 3.1) and of the NSF terms it is built with.

On fields that are linear in x and y, the central and one-sided differences
of the closure are exact, so Kn_GLL has a closed form: the mean free path
lambda = mu(Tt)/(rho Tt) sqrt(pi Tt/2) (the same form as the Knudsen number's
definition in Section 2) times the largest of |grad rho|/rho,
|grad |u||/max(|u|, sqrt(gamma Tt)), |grad Tt|/Tt and |grad Tr|/Tr.  The five
field sets below make each ratio the largest in turn in every cell, the speed
ratio once above and once below the sound-speed floor, with Tt varying so
that lambda's temperature dependence is exercised.

Each plausible mistake listed in PLANTED is compiled into a copy of the
oracle; the same closed-form check must reject every one of them.
"""
import numpy as np
import pytest

import dig_workloads as wl
import oracle

NX, NY, LX, LY = 7, 6, 1.0, 1.5
OMEGA = wl.OMEGA_N2
GAMMA = 7.0 / 5.0  # (5 + d_r)/(3 + d_r), d_r = 2
A_EUCKEN = [2.0 / 3.0, 0.0, 0.0, 5.0 / (7.0 - 2.0 * OMEGA)]


def _workload():
    walls = [("diffuse", 1.0, (0, 0, 0))] * 4
    return wl.box(2, NX, NY, lx=LX, ly=LY, kn=0.05, bc=walls)


def _centres():
    k = np.arange(NX * NY)
    return (k % NX + 0.5) * LX / NX, (k // NX + 0.5) * LY / NY


def _linear(c0, cx, cy):
    x, y = _centres()
    return c0 + cx * x + cy * y, np.array([cx, cy], dtype=np.float64)


# (rho, speed, Tt, Tr) as (c0, cx, cy); the flow direction is fixed at 30 deg
CASES = {
    "density": dict(rho=(1.0, 0.6, 0.2), s=(0.2, 0.01, 0.0), tt=(1.0, 0.0, 0.02),
                    tr=(1.0, 0.03, 0.0)),
    "speed_above_sound": dict(rho=(1.0, 0.0, 0.01), s=(3.0, 2.0, 1.0), tt=(1.0, 0.02, 0.0),
                              tr=(1.0, 0.0, 0.02)),
    "speed_below_sound": dict(rho=(1.0, 0.01, 0.0), s=(0.1, 0.0, 0.6), tt=(1.2, 0.01, 0.0),
                              tr=(1.0, 0.02, 0.0)),
    "translational_T": dict(rho=(1.0, 0.0, 0.02), s=(0.3, 0.01, 0.0), tt=(1.0, 0.9, 0.3),
                            tr=(1.2, 0.05, 0.0)),
    "rotational_T": dict(rho=(1.0, 0.01, 0.0), s=(0.3, 0.0, 0.01), tt=(1.1, 0.02, 0.0),
                         tr=(0.8, 0.0, 1.2)),
}
WINNER = {"density": 0, "speed_above_sound": 1, "speed_below_sound": 1, "translational_T": 2,
          "rotational_T": 3}


def _fields(case):
    p = CASES[case]
    rho, grho = _linear(*p["rho"])
    s, gs = _linear(*p["s"])
    tt, gtt = _linear(*p["tt"])
    tr, gtr = _linear(*p["tr"])
    th = np.pi / 6.0
    f = np.zeros((20, NX * NY))
    f[0], f[1], f[2], f[4], f[5] = rho, s * np.cos(th), s * np.sin(th), tt, tr
    return f, dict(rho=rho, grho=grho, s=s, gs=gs, tt=tt, gtt=gtt, tr=tr, gtr=gtr)


def closed_form_kn(w, g):
    """Kn_GLL of Section 3.1 on linear fields, written out from its definition."""
    mu = oracle.mu0(w) * g["tt"] ** OMEGA
    lam = mu / (g["rho"] * g["tt"]) * np.sqrt(np.pi * g["tt"] / 2.0)
    ratios = np.stack([
        np.linalg.norm(g["grho"]) / g["rho"],
        np.linalg.norm(g["gs"]) / np.maximum(g["s"], np.sqrt(GAMMA * g["tt"])),
        np.linalg.norm(g["gtt"]) / g["tt"],
        np.linalg.norm(g["gtr"]) / g["tr"],
    ])
    return lam * ratios.max(axis=0), ratios


def kn_error():
    """Largest relative deviation of the oracle's Kn_GLL from the closed form
    over all cases and cells."""
    w = _workload()
    worst = 0.0
    for case in CASES:
        f, g = _fields(case)
        _, _, kn, _ = oracle.closure(w, f, A_EUCKEN, 0.0)
        ref, _ = closed_form_kn(w, g)
        worst = max(worst, float(np.max(np.abs(kn - ref) / ref)))
    return worst


@pytest.mark.parametrize("case", list(CASES))
def test_each_ratio_wins_where_intended(case):
    w = _workload()
    _, g = _fields(case)
    _, ratios = closed_form_kn(w, g)
    assert np.all(np.argmax(ratios, axis=0) == WINNER[case])
    if case == "speed_above_sound":
        assert np.all(g["s"] > np.sqrt(GAMMA * g["tt"]))
    if case == "speed_below_sound":
        assert np.all(g["s"] < np.sqrt(GAMMA * g["tt"]))


def test_kn_gll_equals_closed_form():
    assert kn_error() < 1e-12


def test_mask_is_the_threshold_of_the_closed_form():
    w = _workload()
    f, g = _fields("translational_T")
    ref, _ = closed_form_kn(w, g)
    kn_ref = float(np.median(ref))
    hot, mask, kn, nsf = oracle.closure(w, f, A_EUCKEN, kn_ref)
    np.testing.assert_array_equal(mask, (ref < kn_ref).astype(np.uint8))
    assert 0 < mask.sum() < mask.size
    assert np.all(hot[:, mask == 1] == 0.0)
    np.testing.assert_allclose(hot[:, mask == 0], -nsf[:, mask == 0], rtol=1e-13)


def test_nsf_terms_with_a_full_velocity_gradient():
    """sigma = -mu (grad u + grad u^T - 2/3 div u I) with all four in-plane
    gradient entries non-zero, and the heat fluxes of the Eucken-type A."""
    w = _workload()
    x, y = _centres()
    G = np.array([[0.3, -0.2], [0.45, 0.1]])  # G[i][j] = d u_i / d x_j
    f = np.zeros((20, NX * NY))
    f[0] = 1.0
    f[1] = 0.5 + G[0, 0] * x + G[0, 1] * y
    f[2] = -0.2 + G[1, 0] * x + G[1, 1] * y
    f[3] = 0.1 - 0.3 * x + 0.7 * y
    f[4] = 1.0 + 0.2 * x - 0.1 * y
    f[5] = 0.9 - 0.05 * x + 0.3 * y
    _, _, _, nsf = oracle.closure(w, f, A_EUCKEN, 0.0)
    mu = oracle.mu0(w) * f[4] ** OMEGA
    div = G[0, 0] + G[1, 1]
    np.testing.assert_allclose(nsf[0], -mu * (2 * G[0, 0] - 2 / 3 * div), rtol=1e-12)
    np.testing.assert_allclose(nsf[1], -mu * (2 * G[1, 1] - 2 / 3 * div), rtol=1e-12)
    np.testing.assert_allclose(nsf[2], -mu * (-2 / 3 * div), rtol=1e-12)
    np.testing.assert_allclose(nsf[3], -mu * (G[0, 1] + G[1, 0]), rtol=1e-12)
    np.testing.assert_allclose(nsf[4], -mu * -0.3, rtol=1e-12)
    np.testing.assert_allclose(nsf[5], -mu * 0.7, rtol=1e-12)
    kt, kr = 15.0 / 4.0 * mu, (7.0 - 2.0 * OMEGA) / 5.0 * mu
    np.testing.assert_allclose(nsf[6], -kt * 0.2, rtol=1e-12)
    np.testing.assert_allclose(nsf[7], -kt * -0.1, rtol=1e-12)
    np.testing.assert_allclose(nsf[9], -kr * -0.05, rtol=1e-12)
    np.testing.assert_allclose(nsf[10], -kr * 0.3, rtol=1e-12)
    assert np.all(nsf[8] == 0) and np.all(nsf[11] == 0)


# Plausible mistakes, each compiled into a copy of the oracle.
PLANTED = {
    "lambda_factor_2": ("double lam = mu / (rho[k] * tt[k])", "double lam = 2.0 * mu / (rho[k] * tt[k])"),
    "lambda_without_pi_over_2": ("sqrt(M_PI * tt[k] / 2.0)", "sqrt(tt[k])"),
    "speed_floor_dropped": ("/ (us > cs ? us : cs);", "/ us;"),
    "density_branch_dropped": ("double m = g;", "double m = 0.0;"),
    "rotational_ratio_over_tt": ("/ tr[k] : 0.0;", "/ tt[k] : 0.0;"),
    "speed_gradient_of_ux": ("grad_axis(c, speed, ix, iy, 0), grad_axis(c, speed, ix, iy, 1)",
                             "grad_axis(c, ux, ix, iy, 0), grad_axis(c, ux, ix, iy, 1)"),
}


@pytest.mark.parametrize("name", list(PLANTED))
def test_planted_mistake_is_caught(name, tmp_path):
    with oracle.variant([PLANTED[name]], str(tmp_path)):
        err = kn_error()
    assert err > 1e-3, f"planted mistake {name} not caught (error {err:.2e})"
    assert kn_error() < 1e-12  # the real oracle is back in place


def test_sparse_cells_are_treated_as_equilibrium():
    """Cells holding on average fewer than n_min particles (row 19) give no
    higher-order terms: mask 1 and HoT 0, Kn_GLL unchanged; the other cells
    are untouched, and n_min = 0 changes nothing."""
    import dig_workloads as wl
    w = wl.cavity_2d(n=8, kn=0.05)
    rng = np.random.default_rng(12)
    f = np.zeros((20, 64))
    f[0] = 1.0 + 0.2 * rng.random(64)
    f[1:4] = 0.1 * rng.standard_normal((3, 64))
    f[4] = 1.0 + 0.3 * rng.random(64)
    f[5] = 1.0 + 0.3 * rng.random(64)
    f[6:18] = 0.05 * rng.standard_normal((12, 64))
    f[19] = 0.5 + 3.0 * rng.random(64)
    A = (2.0 / 3.0, 0.0, 0.0, 5.0 / (7.0 - 2.0 * wl.OMEGA_N2))
    h0, m0, k0, n0 = oracle.closure(w, f, A, 0.001)
    hz, mz, kz, nz = oracle.closure(w, f, A, 0.001, n_min=0.0)
    assert np.array_equal(h0, hz) and np.array_equal(m0, mz)
    h1, m1, k1, n1 = oracle.closure(w, f, A, 0.001, n_min=1.5)
    sparse = f[19] < 1.5
    assert 0 < sparse.sum() < 64
    assert np.all(m1[sparse] == 1) and np.all(h1[:, sparse] == 0.0)
    np.testing.assert_array_equal(m1[~sparse], m0[~sparse])
    np.testing.assert_array_equal(h1[:, ~sparse], h0[:, ~sparse])
    np.testing.assert_array_equal(k1, k0)
    np.testing.assert_array_equal(n1, n0)


def test_fill_empty_takes_the_fallback_only_where_no_sample_is_usable():
    rng = np.random.default_rng(3)
    C = 40
    f = np.zeros((20, C))
    f[0] = 1.0 + rng.random(C)
    f[1:4] = rng.standard_normal((3, C))
    f[4] = 1.0 + rng.random(C)
    f[5] = 1.0 + rng.random(C)
    f[6:19] = rng.standard_normal((13, C))
    f[19] = 1.0 + 5.0 * rng.random(C)
    bad = {3: (19, 0.0), 7: (0, 0.0), 11: (4, 0.0), 15: (5, -0.1), 21: (2, np.nan),
           25: (4, np.inf)}
    for c, (row, v) in bad.items():
        f[row, c] = v
    fb = rng.random((6, C)) + 0.5
    out = oracle.fill_empty(f, fb, dr=2)
    good = np.ones(C, bool)
    good[list(bad)] = False
    np.testing.assert_array_equal(out[:, good], f[:, good])
    np.testing.assert_array_equal(out[0:6, ~good], fb[:, ~good])
    assert np.all(out[6:18, ~good] == 0.0) and np.all(out[19, ~good] == 0.0)
    np.testing.assert_allclose(out[18, ~good], (3 * fb[4, ~good] + 2 * fb[5, ~good]) / 5,
                               rtol=1e-15)
