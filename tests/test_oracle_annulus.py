"""Oracle pins for the annulus geometry with open boundaries (flow past a
cylinder): cell map against polar coordinates, cell areas, a closed annulus in
equilibrium, and the freestream inflow against the one-way flux of a drifting
Maxwellian (collisionless, so entering particles are counted exactly)."""
import math

import numpy as np
from scipy.special import erf

import dig_workloads as wl
import oracle


def small(outer="freestream", mach=2.0, kn=0.05, nth=48, nr=24, n_target=40_000, seed=11):
    return wl.cylinder(seed=seed, nth=nth, nr=nr, r_in=0.5, r_out=2.0, first=0.03, kn=kn,
                       mach=mach, n_target=n_target, outer=outer)


def test_cell_map_matches_polar_coordinates():
    w = small()
    rng = np.random.default_rng(1)
    n = 20000
    r = np.sqrt(rng.uniform(0.5 ** 2, 2.2 ** 2, n))
    th = rng.uniform(0, 2 * np.pi, n)
    x, y = r * np.cos(th), r * np.sin(th)
    faces = np.array([oracle.annulus_face(w, j) for j in range(w["ny"] + 1)])
    s = oracle.State(w, n)
    s.load(x, y, np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n), np.arange(n))
    cell = s.cells()
    dth = 2 * np.pi / w["nx"]
    i = np.floor(th / dth).astype(int)
    j = np.searchsorted(faces, r, side="right") - 1
    # away from faces (relative distance > 1e-5) the map is the polar one
    far = (np.abs(th / dth - np.round(th / dth)) > 1e-4) & \
        (np.min(np.abs(r[:, None] - faces[None, :]), axis=1) > 1e-5 * r)
    inside = r < faces[-1] * (1 - 1e-6)
    ok = far & inside
    np.testing.assert_array_equal(cell[ok], (i + w["nx"] * np.clip(j, 0, w["ny"] - 1))[ok])
    outside = r > faces[-1] * (1 + 1e-6)
    assert np.all(cell[outside] == -1)
    assert np.all(cell[inside] >= 0)
    # points on face directions belong to the sector that starts there
    k = np.arange(w["nx"])
    px, py = 1.0 * np.cos(k * dth), 1.0 * np.sin(k * dth)
    s.load(px, py, np.zeros(len(k)), np.zeros(len(k)), np.zeros(len(k)), np.zeros(len(k)), k)
    ck = s.cells() % w["nx"]
    assert np.all((ck == k) | (ck == (k - 1) % w["nx"]))


def test_cell_areas_sum_to_annulus_and_stretching():
    w = small()
    C = w["nx"] * w["ny"]
    v = np.array([oracle.cell_volume(w, c) for c in range(C)])
    assert abs(v.sum() - np.pi * (2.0 ** 2 - 0.5 ** 2)) < 1e-12
    f = np.array([oracle.annulus_face(w, j) for j in range(w["ny"] + 1)])
    assert abs(f[1] - f[0] - 0.03) < 1e-9 and abs(f[-1] - 2.0) < 1e-14
    ratios = np.diff(f)[1:] / np.diff(f)[:-1]
    np.testing.assert_allclose(ratios, w["q"], rtol=1e-9)


def test_closed_annulus_stays_in_equilibrium():
    """Diffuse inner and outer circles at T = 1 around gas at rest, T = 1:
    the particle count is conserved and the gas stays at T = 1 (particle
    moments averaged over the steps)."""
    w = small(outer="diffuse")
    s = oracle.new_state(w, cap_factor=1.2)
    n0 = s.n
    tt, tr, ux = [], [], []
    for _ in range(40):
        s.step()
        n = s.n
        tt.append((s.vx[:n] ** 2 + s.vy[:n] ** 2 + s.vz[:n] ** 2).mean() / 3.0)
        tr.append(s.er[:n].mean())
        ux.append(s.vx[:n].mean())
    assert s.n == n0
    # one step's estimate has standard deviation sqrt(2/(3n)) (Tt), 1/sqrt(n) (Tr)
    assert abs(np.mean(tt) - 1.0) < 4 * math.sqrt(2 / (3 * n0)), np.mean(tt)
    assert abs(np.mean(tr) - 1.0) < 4 / math.sqrt(n0), np.mean(tr)
    assert abs(np.mean(ux)) < 4 / math.sqrt(n0)


def _one_way_flux(U, T, rho, r, n=20000):
    """Particles per unit time entering a circle of radius r from a uniform
    drifting Maxwellian (U along +x) outside it: the integral over the circle
    of rho sqrt(T / 2 pi) (exp(-s^2) + sqrt(pi) s (1 + erf s)), s = U.n_in / sqrt(2T)."""
    th = (np.arange(n) + 0.5) * 2 * np.pi / n
    s = -U * np.cos(th) / math.sqrt(2 * T)  # n_in = -(cos, sin)
    f = rho * math.sqrt(T / (2 * math.pi)) * (np.exp(-s * s) + math.sqrt(math.pi) * s *
                                               (1 + erf(s)))
    return f.sum() * (2 * np.pi / n) * r


def test_inflow_matches_drifting_maxwellian_flux():
    """Collisionless (Kn = 50): particles that enter in a step are exactly the
    reservoir particles ending inside; their mean count is the one-way flux."""
    for mach in (0.0, 2.0):
        w = small(mach=mach, kn=50.0)
        w["dt"] = 0.01
        s = oracle.new_state(w, cap_factor=1.5)
        entered = []
        for _ in range(30):
            n0 = s.n
            s.inject()
            n1 = s.n
            s.move()
            cell = s.cells()
            entered.append(int((cell[n0:n1] >= 0).sum()))
            s.sort()
            s.step_no += 1
        U = mach * math.sqrt(1.4)
        expect = _one_way_flux(U, 1.0, 1.0, 2.0) * w["dt"] / w["weight"]
        got = np.mean(entered)
        assert abs(got - expect) < 4 * math.sqrt(expect / len(entered)) + 0.5, (mach, got,
                                                                                 expect)


def test_freestream_at_rest_keeps_density():
    """Gas at rest, T = 1, inside a freestream boundary at rest with the same
    state: what enters balances what leaves; density and count stay put."""
    w = small(mach=0.0)
    s = oracle.new_state(w, cap_factor=1.5)
    n0 = s.n
    for _ in range(30):
        s.step()
    assert abs(s.n - n0) < 5 * math.sqrt(n0 * 0.05) + 50
    f = s.fields()
    outer = slice(w["nx"] * (w["ny"] - 3), w["nx"] * w["ny"])
    rho = f[0][outer].mean()
    assert abs(rho - 1.0) < 0.03, rho
