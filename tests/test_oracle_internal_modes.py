"""Pins of the oracle's rotational modes beyond the paper's case d_r = 2:
Borgnakke-Larsen with Beta(d_r/2, 5/2 - omega) fractions and Gamma(d_r/2)
equilibrium energies for d_r = 3..6 (Section 2.2 writes the model and the
Jeans relaxation for a general d_r).

* Equilibrium rotational energies drawn at init, at diffuse walls and by the
  freestream have the Gamma(d_r/2, T) mean and variance.
* Collisions keep a gas with Tt = Tr in equilibrium, with Gamma(d_r/2) energies.
* Tr relaxes to T = (3 Tt + d_r Tr)/(3 + d_r) at the Jeans rate p/(mu Z).
* Each mistake in PLANTED breaks one of them."""
import math

import numpy as np
import pytest

import dig_workloads as wl
import oracle

OM = wl.OMEGA_N2


def zero_d(n, dr, Tt, Tr, zrot=5.0, seed=7, kn=0.1):
    w = wl.box(1, 1, kn=kn, zrot=zrot, ppc=n, seed=seed, Tt=Tt, Tr=Tr, dr=dr, tref=max(Tt, Tr))
    s = oracle.new_state(w, cap=n)
    return w, s


def temps(s, dr):
    n = s.n
    v = np.stack([s.vx[:n], s.vy[:n], s.vz[:n]])
    u = v.mean(axis=1, keepdims=True)
    return ((v - u) ** 2).sum(axis=0).mean() / 3.0, 2.0 * s.er[:n].mean() / dr


def gamma_ok(er, dr, T, k=5.0):
    """Mean and variance of er against Gamma(dr/2, T), within k standard errors."""
    n = len(er)
    a = 0.5 * dr
    mean, var = a * T, a * T * T
    se_mean = math.sqrt(var / n)
    se_var = math.sqrt((6.0 / a + 2.0) * var * var / n)  # Gamma: excess kurtosis 6/a
    return abs(er.mean() - mean) < k * se_mean and abs(er.var() - var) < k * se_var


@pytest.mark.parametrize("dr", [3, 4, 5, 6])
def test_initial_rotational_energies_are_gamma(dr):
    w, s = zero_d(40000, dr, 1.0, 1.3, seed=11 + dr)
    assert gamma_ok(s.er[: s.n], dr, 1.3)


@pytest.mark.parametrize("dr", [3, 5])
def test_wall_reemission_energies_are_gamma(dr):
    Tw = 1.4
    bc = [("diffuse", Tw, (0, 0, 0)), ("diffuse", 1.0, (0, 0, 0)), ("periodic", 1, (0, 0, 0)),
          ("periodic", 1, (0, 0, 0))]
    n = 100_000
    w = wl.box(1, 10, bc=bc, ppc=1, seed=9, dt=1e-3, dr=dr)
    s = oracle.State(w, n)
    s.load(np.full(n, 0.005), np.zeros(n), np.full(n, -1.0), np.zeros(n), np.zeros(n),
           np.zeros(n), np.arange(n, dtype=np.uint32), step=4)
    assert s.move() == n
    assert gamma_ok(s.er[:n], dr, Tw)


def equilibrium(dr, steps=120, n=20000, seed=5):
    w, s = zero_d(n, dr, 1.0, 1.0, seed=seed)
    for k in range(steps):
        s.step_no = k
        s.collide()
    Tt, Tr = temps(s, dr)
    return Tt, Tr, s.er[:n] / ((3 * Tt + dr * Tr) / (3 + dr))


@pytest.mark.parametrize("dr", [3, 4])
def test_collisions_keep_equilibrium(dr):
    Tt, Tr, er = equilibrium(dr)
    T = (3 * Tt + dr * Tr) / (3 + dr)
    assert abs(Tr - T) < 6.0 * T * math.sqrt(2.0 / (dr * len(er)))
    assert gamma_ok(er, dr, 1.0)


def relaxation_ratio(dr, zrot=5.0, n=150_000, seed=21):
    """Measured rate of Tr - T over the Jeans rate p / (mu Z) at T = 1."""
    Tt0 = 1.0 + 0.05
    Tr0 = (3.0 + dr - 3.0 * Tt0) / dr  # T = 1
    w, s = zero_d(n, dr, Tt0, Tr0, zrot=zrot, seed=seed)
    mu0 = oracle.mu0(w)
    ts, ys = [], []
    for step in range(60):
        Tt, Tr = temps(s, dr)
        T = (3 * Tt + dr * Tr) / (3 + dr)
        ts.append(step * w["dt"])
        ys.append(Tr - T)
        s.step_no = step
        s.collide()
    ts, ys = np.array(ts), np.array(ys)
    keep = np.abs(ys) > 0.012
    slope = np.polyfit(ts[keep], np.log(np.abs(ys[keep])), 1)[0]
    return -slope / (1.0 / (mu0 * zrot))


@pytest.mark.parametrize("dr", [3, 5])
def test_jeans_relaxation_rate(dr):
    """Two seeds averaged; the fit's own spread is a few per cent (d_r = 2
    gives 0.95 and 1.01 on two seeds), and the paper's P_inelastic, kept for
    every d_r, is derived for the double-relaxation scheme without a d_r
    factor, so 8 % is the bound."""
    ratio = 0.5 * (relaxation_ratio(dr, seed=21) + relaxation_ratio(dr, seed=22))
    assert abs(ratio - 1.0) < 0.08, ratio


PLANTED = {
    "odd_dof_as_even": [("if (c->dr >= 4) g += -log(orc_u01(w[0]));",
                         "if (c->dr >= 3) g += -log(orc_u01(w[0]));")],
    "beta_shape_off_by_half": [("double a = 0.5 * c->dr;", "double a = 0.5 * (c->dr - 1);")],
}


@pytest.mark.parametrize("name", list(PLANTED))
def test_planted_mistake_is_caught(name, tmp_path):
    with oracle.variant(PLANTED[name], str(tmp_path)):
        ok = []
        w, s = zero_d(40000, 3, 1.0, 1.3, seed=14)
        ok.append(gamma_ok(s.er[: s.n], 3, 1.3))
        Tt, Tr, er = equilibrium(3, steps=60)
        ok.append(gamma_ok(er, 3, 1.0))
    assert not all(ok), name
