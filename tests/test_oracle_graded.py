"""Pins of the oracle on graded grids (cells of different widths between
per-axis face tables, positions in physical units): the wall-refined grids
of the paper's DIG cavity (Section 4.1, Table 1: 100 x 100 cells, first cell
0.001 at the walls).

* A graded grid whose faces are uniform reproduces the uniform box: cell
  volumes, free flight and cell index, collisions, closure and both
  synthetic-solve schemes.
* Cell-centred gradients are exact for linear fields on any grid, so the NSF
  terms and Kn_GLL equal their closed forms at every cell, walls included.
* Cell location equals a search over the FP32 faces, positions exactly on a
  face included; initial and DIG-modified particle counts follow the cell
  volumes; positions stay in their cells.
* The synthetic solve keeps the total mass (sum of rho V) exactly, reproduces
  Couette flow (linear velocity in the cell-centre coordinate) on a strongly
  graded axis, and LU-SGS converges to the explicit scheme's state.
* Each mistake in PLANTED_C / PLANTED_SYNTH breaks one of these pins."""
import types

import numpy as np
import pytest

import dig_workloads as wl
import oracle
from oracle import synth

PER = ("periodic", 1.0, (0.0, 0.0, 0.0))


def uniform_twin(w):
    """The graded-geometry copy of a uniform box workload."""
    g = dict(w)
    g["geometry"] = "graded"
    g["xfaces"] = list(np.linspace(0.0, w["lx"], w["nx"] + 1))
    g["yfaces"] = list(np.linspace(0.0, w["ly"], w["ny"] + 1)) if w["dim"] == 2 else [0.0, 1.0]
    return g


def graded_cavity(n=12, first=0.01, kn=0.05, ppc=30, seed=21):
    f = wl.wall_refined_faces(n, 1.0, first)
    w = wl.cavity_graded(seed=seed, n=n, first=first, ppc=ppc, kn=kn)
    assert np.allclose(w["xfaces"], f)
    return w


def random_fields(nc, seed, lin=None):
    rng = np.random.default_rng(seed)
    m = np.zeros((20, nc))
    m[0] = 1.0 + 0.1 * rng.random(nc)
    m[1:4] = 0.1 * rng.standard_normal((3, nc))
    m[4] = 1.0 + 0.1 * rng.random(nc)
    m[5] = 1.0 + 0.1 * rng.random(nc)
    m[6:18] = 0.01 * rng.standard_normal((12, nc))
    return m


# ----------------------------------------------------------------------------- C oracle
def test_uniform_faces_reproduce_the_box_step():
    w = wl.cavity_2d(seed=31, n=8, ppc=20, kn=0.05)
    g = uniform_twin(w)
    h = 1.0 / 8
    for k in range(64):
        assert oracle.cell_volume(g, k) == pytest.approx(oracle.cell_volume(w), rel=1e-15)
    st = wl.random_sorted_state(w, 5)
    start = st.pop("start")
    n = len(st["x"])
    sg = np.full(64, oracle.sgmax_default(w), np.float32)
    a, b = oracle.State(w, 2 * n), oracle.State(g, 2 * n)
    args = [st[k] for k in ("x", "y", "vx", "vy", "vz", "er", "id")]
    a.load(*args, start=start, sgmax=sg, step=2)
    args[0] = st["x"].astype(np.float64) * h
    args[1] = st["y"].astype(np.float64) * h
    b.load(*args, start=start, sgmax=sg.copy(), step=2)
    a.move()
    b.move()
    np.testing.assert_allclose(b.x[:n], a.x[:n] * h, rtol=0, atol=1e-12)
    np.testing.assert_allclose(b.y[:n], a.y[:n] * h, rtol=0, atol=1e-12)
    for k in ("vx", "vy", "vz", "er"):
        np.testing.assert_array_equal(getattr(b, k)[:n], getattr(a, k)[:n])
    # cells agree away from FP32 ties at the faces
    far = (np.abs(a.x[:n] - np.round(a.x[:n])) > 1e-5) & (np.abs(a.y[:n] - np.round(a.y[:n])) > 1e-5)
    assert far.mean() > 0.99
    np.testing.assert_array_equal(a.cells()[far], b.cells()[far])
    if far.all():
        a.sort()
        b.sort()
        ra, rb = a.collide(), b.collide()
        assert ra == rb
        for k in ("vx", "vy", "vz", "er"):
            np.testing.assert_array_equal(getattr(b, k)[: b.n], getattr(a, k)[: a.n])


def test_uniform_faces_reproduce_the_box_closure():
    w = wl.cavity_2d(seed=31, n=9, ppc=20, kn=0.05)
    g = uniform_twin(w)
    m = random_fields(81, 3)
    A = (2.0 / 3.0, 0.0, 0.0, 5.0 / (7.0 - 2.0 * wl.OMEGA_N2))
    for x, y in zip(oracle.closure(w, m, A, 0.01), oracle.closure(g, m, A, 0.01)):
        np.testing.assert_allclose(y, x, rtol=1e-12, atol=1e-14)


def _linear_fields(w, cx, cy):
    """Fields linear in the cell-centre coordinates of a graded grid."""
    nx, ny = w["nx"], w["ny"]
    X = np.tile(cx, ny)
    Y = np.repeat(cy, nx)
    m = np.zeros((20, nx * ny))
    m[0] = 1.0 + 0.2 * X - 0.1 * Y
    m[1] = 0.05 + 0.3 * X + 0.2 * Y
    m[2] = -0.1 * X + 0.25 * Y
    m[3] = 0.05 * X - 0.04 * Y
    m[4] = 1.0 + 0.3 * X + 0.1 * Y
    m[5] = 1.1 - 0.2 * X + 0.3 * Y
    return m, X, Y


def gradient_error(S=None):
    """Largest deviation of the oracle's NSF terms and Kn_GLL from their
    closed forms for linear fields on a strongly graded 2D grid."""
    fx = wl.wall_refined_faces(11, 1.0, 0.01)
    fy = wl.wall_refined_faces(9, 1.0, 0.004)
    w = wl.graded_box(2, fx, fy, kn=0.05, bc=[wl._bc("diffuse")] * 4)
    cx, cy = 0.5 * (fx[1:] + fx[:-1]), 0.5 * (fy[1:] + fy[:-1])
    m, X, Y = _linear_fields(w, cx, cy)
    A = (2.0 / 3.0, 0.0, 0.0, 5.0 / (7.0 - 2.0 * wl.OMEGA_N2))
    hot, mask, kn, nsf = oracle.closure(w, m, A, 0.0)
    om = wl.OMEGA_N2
    mu = 0.05 * np.sqrt(2 / np.pi) * m[4] ** om
    dux, duy, dvx, dvy, dwx, dwy = 0.3, 0.2, -0.1, 0.25, 0.05, -0.04
    div = dux + dvy
    det = A[0] * A[3] - A[1] * A[2]
    kt = 0.5 * mu * (A[3] * 5 - A[1] * 2) / det
    kr = 0.5 * mu * (-A[2] * 5 + A[0] * 2) / det
    ref = np.array([-mu * (2 * dux - 2 / 3 * div), -mu * (2 * dvy - 2 / 3 * div),
                    -mu * (-2 / 3 * div), -mu * (duy + dvx), -mu * dwx, -mu * dwy,
                    -kt * 0.3, -kt * 0.1, 0 * mu, -kr * -0.2, -kr * 0.3, 0 * mu])
    err = np.abs(nsf - ref).max() / np.abs(ref).max()
    lam = mu / (m[0] * m[4]) * np.sqrt(np.pi * m[4] / 2)
    sp = np.sqrt(m[1] ** 2 + m[2] ** 2 + m[3] ** 2)
    # |grad |u|| from the linear speed field is not linear: compare the other
    # three ratios, which bound Kn_GLL from below, and equality where they win
    g_rho = np.hypot(0.2, -0.1) / m[0]
    g_t = np.hypot(0.3, 0.1) / m[4]
    g_r = np.hypot(-0.2, 0.3) / m[5]
    lower = lam * np.maximum(np.maximum(g_rho, g_t), g_r)
    kerr = max(0.0, np.max((lower - kn) / lower))
    return err, kerr


def test_gradients_are_exact_for_linear_fields():
    err, kerr = gradient_error()
    assert err < 1e-10, err
    assert kerr < 1e-12, kerr


def test_cell_location_equals_a_search_over_fp32_faces():
    fx = wl.wall_refined_faces(13, 1.0, 0.003)
    fy = wl.wall_refined_faces(7, 1.0, 0.02)
    w = wl.graded_box(2, fx, fy, kn=0.05, bc=[wl._bc("diffuse")] * 4)
    rng = np.random.default_rng(4)
    f32x, f32y = fx.astype(np.float32), fy.astype(np.float32)
    x = np.concatenate([rng.random(3000), f32x, np.nextafter(f32x, np.float32(-1)),
                        np.nextafter(f32x, np.float32(2))]).astype(np.float32)
    y = np.concatenate([rng.random(3000), np.resize(f32y, 14), np.resize(f32y, 14),
                        np.resize(f32y, 14)]).astype(np.float32)
    y = np.resize(y, len(x))
    x = np.clip(x, 0, 1)
    y = np.clip(y, 0, 1)
    s = oracle.State(w, len(x))
    s.load(x, y, np.zeros(len(x)), np.zeros(len(x)), np.zeros(len(x)), np.zeros(len(x)),
           np.arange(len(x), dtype=np.uint32))
    cells = s.cells()
    ix = np.clip(np.searchsorted(f32x, x, side="right") - 1, 0, 12)
    iy = np.clip(np.searchsorted(f32y, y, side="right") - 1, 0, 6)
    np.testing.assert_array_equal(cells, ix + 13 * iy)


def init_check(S=None):
    """(largest |count - rho V / N_eff|, particles outside their cell) after
    initialisation of a graded cavity with a density gradient."""
    w = graded_cavity(n=10, first=0.02, ppc=40)
    nc = 100
    f = np.zeros((6, nc))
    rng = np.random.default_rng(9)
    f[0] = 0.5 + rng.random(nc)
    f[4] = f[5] = 1.0
    s = oracle.State(w, 20000)
    s.init(f, 0, 1.0)
    counts = np.diff(s.start)
    fx, fy = np.asarray(w["xfaces"]), np.asarray(w["yfaces"])
    vol = np.outer(np.diff(fy), np.diff(fx)).ravel()    # from the faces, not the oracle
    dev = np.abs(counts - f[0] * vol / w["weight"]).max()
    cell = np.repeat(np.arange(nc), counts)
    ix, iy = cell % 10, cell // 10
    xs, ys = s.x[: s.n], s.y[: s.n]
    outside = np.sum((xs < fx[ix]) | (xs > fx[ix + 1]) | (ys < fy[iy]) | (ys > fy[iy + 1]))
    return dev, int(outside)


def test_initial_counts_follow_cell_volumes():
    dev, outside = init_check()
    assert dev < 1.0 and outside == 0, (dev, outside)


def test_dig_modification_counts_follow_cell_volumes():
    w = graded_cavity(n=8, first=0.03, ppc=40)
    s = oracle.new_state(w, cap_factor=3.0)
    for _ in range(3):
        s.step()
    t = np.zeros((6, 64))
    rng = np.random.default_rng(2)
    t[0] = 0.8 + 0.4 * rng.random(64)
    t[4] = t[5] = 1.0
    assert s.adjust(t, 1) == 0
    counts = np.diff(s.start)
    fx, fy = np.asarray(w["xfaces"]), np.asarray(w["yfaces"])
    vol = np.outer(np.diff(fy), np.diff(fx)).ravel()
    assert np.abs(counts - t[0] * vol / w["weight"]).max() < 1.0
    cell = np.repeat(np.arange(64), counts)
    ix, iy = cell % 8, cell // 8
    xs, ys = s.x[: s.n], s.y[: s.n]
    assert np.all((xs >= fx[ix]) & (xs <= fx[ix + 1]) & (ys >= fy[iy]) & (ys <= fy[iy + 1]))


# ----------------------------------------------------------------------------- synthetic solve
def _fields(nc, T=1.0):
    m = np.zeros((20, nc))
    m[0] = 1.0
    m[4] = T
    m[5] = T
    return m


@pytest.mark.parametrize("scheme", ["explicit", "lusgs"])
def test_uniform_faces_reproduce_the_box_solve(scheme):
    w = wl.cavity_2d(seed=1, n=8, kn=0.05)
    g = uniform_twin(w)
    m = random_fields(64, 7)
    hot = m[6:18] * 0.1
    fn = synth.solve if scheme == "explicit" else synth.solve_lusgs
    a, ia, _ = fn(w, m, hot=hot, max_iter=30, tol=0.0)
    b, ib, _ = fn(g, m, hot=hot, max_iter=30, tol=0.0)
    assert ia == ib == 30
    np.testing.assert_allclose(b, a, rtol=1e-11, atol=1e-13)


def couette_error(S=synth):
    """Largest deviation of the converged Couette velocity from the linear
    profile through the cell centres (strongly graded y axis)."""
    U = 0.02
    fy = wl.wall_refined_faces(16, 1.0, 0.005)
    bc = [PER, PER, ("diffuse", 1.0, (-U, 0, 0)), ("diffuse", 1.0, (U, 0, 0))]
    w = wl.graded_box(2, np.linspace(0, 1, 3), fy, kn=0.05, bc=bc)
    out, it, ch = S.solve_lusgs(w, _fields(32), max_iter=8000, tol=1e-12, wall_mode="wall")
    assert ch < 1e-12, (it, ch)
    yc = 0.5 * (fy[1:] + fy[:-1])
    return np.abs(out[1].reshape(16, 2) - (U * (2 * yc - 1))[:, None]).max()


def test_couette_closed_form_on_a_graded_axis():
    assert couette_error() < 2e-6


def mass_drift(S=synth, scheme="explicit"):
    """Relative change of sum(rho V) over 40 steps on a graded periodic box
    with a non-uniform start."""
    fx = wl.wall_refined_faces(12, 1.0, 0.02)
    fy = wl.wall_refined_faces(10, 1.0, 0.03)
    w = wl.graded_box(2, fx, fy, kn=0.05, bc=[PER] * 4)
    m = random_fields(120, 11)
    vol = np.outer(np.diff(fy), np.diff(fx)).ravel()
    fn = S.solve if scheme == "explicit" else S.solve_lusgs
    out, it, _ = fn(w, m, max_iter=40, tol=0.0)
    return abs((out[0] * vol).sum() / (m[0] * vol).sum() - 1.0)


@pytest.mark.parametrize("scheme", ["explicit", "lusgs"])
def test_total_mass_is_kept_on_a_graded_grid(scheme):
    assert mass_drift(scheme=scheme) < 1e-13


def test_lusgs_converges_to_the_explicit_state_on_a_graded_cavity():
    w = graded_cavity(n=8, first=0.06, kn=0.1)
    m = random_fields(64, 5)
    m[0] = 1.0
    mask = (np.random.default_rng(1).random(64) < 0.3).astype(np.uint8)
    ref, _, che = synth.solve(w, m, hot=m[6:18] * 0.1, mask=mask, max_iter=400000, tol=1e-13,
                              cfl=0.8)
    out, _, chl = synth.solve_lusgs(w, m, hot=m[6:18] * 0.1, mask=mask, max_iter=20000,
                                    tol=1e-13)
    assert che < 1e-13 and chl < 1e-13
    assert np.abs(out - ref).max() < 1e-8


# ----------------------------------------------------------------------------- planted mistakes
PLANTED_C = {
    "volume_of_a_uniform_cell": [("double w = c->xf[i + 1] - c->xf[i];",
                                  "double w = c->lx / c->nx;")],
    "gradient_over_cell_width": [("double d = centre(c, axis, b) - centre(c, axis, a);",
                                  "double d = 2.0 * (centre(c, axis, b) - (axis == 0 ? c->xf : c->yf)[b]);")],
    "strict_face_comparison": [("if (fx[i] <= xs) ix = i;", "if (fx[i] < xs) ix = i;")],
    "uniform_init_positions": [(
        "x[n] = c->xf[ix] + orc_u01(a[0]) * (c->xf[ix + 1] - c->xf[ix]);",
        "x[n] = c->xf[ix] + orc_u01(a[0]) * (c->lx / c->nx);")],
}


@pytest.mark.parametrize("name", list(PLANTED_C))
def test_planted_c_mistake_is_caught(name, tmp_path):
    with oracle.variant(PLANTED_C[name], str(tmp_path)):
        broken = []
        err, kerr = gradient_error()
        broken.append(err > 1e-10 or kerr > 1e-12)
        dev, outside = init_check()
        broken.append(dev >= 1.0 or outside > 0)
        try:
            test_cell_location_equals_a_search_over_fp32_faces()
            broken.append(False)
        except AssertionError:
            broken.append(True)
    assert any(broken), name


def synth_variant(edits):
    text = open(synth.__file__, encoding="utf-8").read()
    for old, new in edits:
        assert text.count(old) == 1, old
        text = text.replace(old, new)
    mod = types.ModuleType("synth_variant")
    exec(compile(text, "synth_variant", "exec"), mod.__dict__)
    return mod


PLANTED_SYNTH = {
    "face_gap_is_a_cell_width": ("gap[1:-1] = c[1:] - c[:-1]", "gap[1:-1] = width[1:]"),
    "wall_gap_of_the_next_face": ("gap[0] = c[0] - f[0]", "gap[0] = c[1] - c[0]"),
    "divergence_over_face_gap": ("            R -= (F[:, 1:, :] - F[:, :-1, :]) / h",
                                 "            R -= (F[:, 1:, :] - F[:, :-1, :]) / P[\"gap\"][1][1:]"),
}


@pytest.mark.parametrize("name", list(PLANTED_SYNTH))
def test_planted_synth_mistake_is_caught(name):
    S = synth_variant([PLANTED_SYNTH[name]])
    with np.errstate(all="ignore"):
        try:
            cerr = couette_error(S)
        except AssertionError:
            cerr = np.inf
        drift = mass_drift(S)
    assert not (cerr < 2e-6 and drift < 1e-13), (name, cerr, drift)


def test_network_inputs_are_exact_for_linear_fields():
    """The learned closure's inputs (scaled gradients) on a graded grid equal
    the closed form for linear fields, wall cells included."""
    from oracle import learn
    fx = wl.wall_refined_faces(9, 1.0, 0.01)
    fy = wl.wall_refined_faces(7, 1.0, 0.02)
    w = wl.graded_box(2, fx, fy, kn=0.05, bc=[wl._bc("diffuse")] * 4)
    cx, cy = 0.5 * (fx[1:] + fx[:-1]), 0.5 * (fy[1:] + fy[:-1])
    m, X, Y = _linear_fields(w, cx, cy)
    kn = np.full(63, 0.1)
    unit = {"x_mean": [0.0] * 9, "x_std": [1.0] * 9, "y_mean": [0.0] * 7, "y_std": [1.0] * 7}
    f, _ = learn.features(w, m, kn, unit)
    mu = 0.05 * np.sqrt(2 / np.pi) * m[4] ** wl.OMEGA_N2
    lam = mu / (m[0] * m[4]) * np.sqrt(np.pi * m[4] / 2)
    su, st = lam / np.sqrt(m[4]), lam / m[4]
    ref = np.stack([su * 0.3, su * 0.2, su * -0.1, su * 0.25, st * 0.3, st * 0.1, st * -0.2,
                    st * 0.3, kn], axis=1)
    np.testing.assert_allclose(f, ref, rtol=1e-10, atol=1e-14)
