"""GPU vs oracle on graded grids (cells of different widths between per-axis
face tables, positions in physical units): the wall-refined grids of the
paper's DIG cavity (Section 4.1, Table 1).

Same contracts as on uniform grids: cell indices, sort permutations, starts
and candidate counts bit-exact; moved positions within 1e-5; post-collision
state within 1e-5 (decision-margin cells aside); initial and DIG-modified
particles (ids, starts bit-exact, positions 1e-6, velocities 2e-6); closure
1e-11; network inputs 2e-6; synthetic solve (both schemes) 1e-9."""
import numpy as np
import pytest
import torch

import dig_workloads as wl
import oracle
from gpu_common import DSMC, gpu_state, np_, oracle_state, rel_close, say
from oracle import learn as olearn
from oracle import synth
from paper_2501_10965_amd import learn
from paper_2501_10965_amd.dsmc import synth_solve
from test_gpu_dig_closure import injected, random_target
from test_gpu_step_parity import run_stage_parity

pytestmark = pytest.mark.gpu

PER = ("periodic", 1.0, (0.0, 0.0, 0.0))


def graded_cases():
    cav = wl.cavity_graded(seed=301, n=24, first=0.004, ppc=40, kn=0.05)
    cav["dt"] *= 2.0  # more wall hits: particles cross several thin cells per step
    fx = wl.wall_refined_faces(30, 1.0, 0.005)
    slab = wl.graded_box(1, fx, kn=0.05, ppc=40, seed=302,
                         bc=[("diffuse", 1.0, (0, 0, 0)), ("diffuse", 1.5, (0, 0, 0)), PER, PER])
    fy = wl.wall_refined_faces(14, 0.7, 0.01)
    per = wl.graded_box(2, wl.wall_refined_faces(12, 1.0, 0.03), fy, kn=0.05, ppc=40, seed=303,
                        bc=[PER, PER, ("diffuse", 1.0, (-0.3, 0, 0)),
                            ("diffuse", 1.2, (0.3, 0, 0))])
    return {"cavity": cav, "slab1d": slab, "periodic_x": per}


CASES = graded_cases()


@pytest.mark.parametrize("name", list(CASES))
def test_graded_step_stage_parity(name):
    say(f"case graded step {name}")
    res, nbad = run_stage_parity(CASES[name], seed=11)
    assert res["accepted"] > 0
    say(f"  candidates={res['candidates']} accepted={res['accepted']} flipped={nbad}")


def test_graded_init_matches_oracle():
    w = CASES["cavity"]
    say("case graded init")
    sim = DSMC(w)
    sim.init()
    g = gpu_state(sim)
    o = oracle.new_state(w)
    om = o.arrays()
    assert len(g["x"]) == o.n
    np.testing.assert_array_equal(g["id"], om["id"])
    np.testing.assert_array_equal(np_(sim.array("start")), o.start)
    for k in ("x", "y"):
        assert rel_close(g[k], om[k], 1e-6).all(), k
    for k in ("vx", "vy", "vz", "er"):
        assert rel_close(g[k], om[k], 1e-5).all(), k
    # every particle lies in its cell by the kernels' own rule
    gc = np.repeat(np.arange(w["nx"] * w["ny"]), np.diff(np_(sim.array("start"))))
    s = oracle.State(w, len(g["x"]))
    s.load(g["x"], g["y"], g["vx"], g["vy"], g["vz"], g["er"], g["id"])
    np.testing.assert_array_equal(s.cells(), gc)


def test_graded_adjust_matches_oracle():
    w = CASES["cavity"]
    say("case graded adjust")
    sim, arrays, start, sg, n = injected(w, seed=7)
    rng = np.random.default_rng(3)
    t = random_target(w, rng)
    t[0, :2] = 0.0
    o = oracle_state(w, arrays, start, sg, 3, cap=4 * n, next_id=n + 17)
    assert o.adjust(t, dig_iter=4) == 0
    sim.adjust(torch.tensor(t, device="cuda"), 4)
    c = sim.counters()
    assert c["n"] == o.n and c["next_id"] == o.next_id
    np.testing.assert_array_equal(np_(sim.array("start")), o.start)
    g = gpu_state(sim)
    om = o.arrays()
    np.testing.assert_array_equal(g["id"], om["id"])
    for k in ("x", "y"):
        assert rel_close(g[k], om[k], 1e-6).all(), k
    for k in ("vx", "vy", "vz", "er"):
        assert rel_close(g[k], om[k], 2e-6).all(), k
    # refill the emptied cells, both sides from the GPU's FP32 state (cells
    # of a few particles amplify the FP32-vs-FP64 difference of the inputs
    # through their sample temperature)
    t2 = t.copy()
    t2[0, :2] = 1.0
    o = oracle_state(w, g, np_(sim.array("start")), np_(sim.array("sgmax")), 3, cap=4 * n,
                     next_id=c["next_id"])
    assert o.adjust(t2, dig_iter=5) == 0
    sim.adjust(torch.tensor(t2, device="cuda"), 5)
    g = gpu_state(sim)
    om = o.arrays()
    np.testing.assert_array_equal(g["id"], om["id"])
    for k in ("x", "y", "vx", "vy", "vz", "er"):
        assert rel_close(g[k], om[k], 2e-6).all(), k


def _smooth_fields(w, seed):
    nx, ny = w["nx"], w["ny"]
    fx = np.asarray(w["xfaces"])
    fy = np.asarray(w["yfaces"]) if w["dim"] == 2 else np.array([0.0, 1.0])
    xc = np.tile(0.5 * (fx[1:] + fx[:-1]), ny)
    yc = np.repeat(0.5 * (fy[1:] + fy[:-1]), nx)
    rng = np.random.default_rng(seed)
    C = nx * ny
    f = np.zeros((20, C))
    f[0] = 1.0 + 0.2 * np.sin(3 * xc) * np.cos(2 * yc)
    f[1] = 0.3 * yc ** 2
    f[2] = -0.1 * np.sin(4 * xc)
    f[3] = 0.02 * xc
    f[4] = 1.0 + 0.3 * xc * yc
    f[5] = 0.9 + 0.2 * np.cos(3 * yc)
    f[6:18] = 0.01 * rng.standard_normal((12, C))
    f[19] = 20.0 + 40.0 * rng.random(C)
    return f


@pytest.mark.parametrize("name", ["cavity", "periodic_x", "slab1d"])
def test_graded_closure_matches_oracle(name):
    w = CASES[name]
    say(f"case graded closure {name}")
    f = _smooth_fields(w, 4)
    A = [2.0 / 3.0, 0.05, 0.02, 5.0 / (7 - 2 * 0.74)]
    # n_min 30: the cells holding on average fewer than 30 particles (row 19
    # ranges over 20..60) keep the NSF closure
    hot, mask, kn, nsf = oracle.closure(w, f, A, 0.01, n_min=30.0)
    assert 0 < (f[19] < 30).sum() < len(f[19])
    sim = DSMC(w)
    gh, gm, gk, gn = sim.closure(torch.tensor(f, device="cuda"), A, 0.01, with_nsf=True,
                                 n_min=30.0)
    np.testing.assert_array_equal(np_(gm), mask)
    np.testing.assert_allclose(np_(gk), kn, rtol=1e-12)
    np.testing.assert_allclose(np_(gh), hot, rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(np_(gn), nsf, rtol=1e-11, atol=1e-15)


def test_graded_network_inputs_and_judge_match_oracle():
    w = CASES["cavity"]
    say("case graded features + blend")
    F = _smooth_fields(w, 6)
    A = learn.default_A(w["omega"])
    hot, mask, kn = oracle.closure(w, F, A, 0.02)[:3]
    rng = np.random.default_rng(2)
    sc = {"x_mean": rng.standard_normal(9) * 0.01, "x_std": 0.5 + rng.random(9),
          "y_mean": rng.standard_normal(7) * 0.01, "y_std": 0.5 + rng.random(7)}
    xo, to = olearn.features(w, F, kn, sc, hot)
    sim = DSMC(w)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), device="cuda")  # noqa: E731
    x, t = sim.features(dev(F), dev(kn), sc, hot=dev(hot))
    np.testing.assert_allclose(np_(x), xo, rtol=2e-6, atol=1e-6)
    np.testing.assert_allclose(np_(t), to, rtol=2e-6, atol=1e-6)
    C = F.shape[1]
    yo = (to + np.where(np.arange(C)[:, None] % 2 == 0, 0.01, 5.0)
          * rng.standard_normal((C, 7))).astype(np.float32)
    kn_lo, kn_hi = float(np.quantile(kn, 0.2)), float(np.quantile(kn, 0.8))
    ref, src_ref = olearn.blend(w, F, kn, mask, yo.astype(np.float64), sc, A, hot, kn_lo,
                                kn_hi, 3.0, 0.1, 5.0)
    h = dev(hot)
    src = sim.blend(dev(F), dev(kn), dev(mask), dev(yo), sc, h, kn_lo, kn_hi, 3.0, 0.1, 5.0,
                    A=A)
    np.testing.assert_array_equal(np_(src), src_ref)
    np.testing.assert_allclose(np_(h), ref, rtol=1e-12, atol=1e-15)


def _synth_case(w, seed):
    C = w["nx"] * w["ny"]
    rng = np.random.default_rng(seed)
    m = np.zeros((20, C))
    m[0] = 1.0 + 0.05 * rng.standard_normal(C)
    m[1] = 0.05 * rng.standard_normal(C)
    m[2] = 0.05 * rng.standard_normal(C) if w["dim"] == 2 else 0.0
    m[4] = 1.0 + 0.03 * rng.standard_normal(C)
    m[5] = 1.0 + 0.03 * rng.standard_normal(C)
    hot = 0.005 * rng.standard_normal((12, C))
    mask = (rng.random(C) < 0.3).astype(np.uint8)
    return m, hot, mask


@pytest.mark.parametrize("scheme,mode,iters", [("explicit", "dsmc", 200), ("explicit", "wall", 200),
                                               ("lusgs", "dsmc", 40), ("lusgs", "wall", 40)])
@pytest.mark.parametrize("name", ["cavity", "periodic_x", "slab1d"])
def test_graded_synth_matches_oracle(name, scheme, mode, iters):
    w = CASES[name]
    say(f"case graded synth {name} {scheme} {mode}")
    m, hot, mask = _synth_case(w, 8)
    fn = synth.solve if scheme == "explicit" else synth.solve_lusgs
    ref, it, _ = fn(w, m, hot=hot, mask=mask, max_iter=iters, tol=0.0, wall_mode=mode)
    out, git, _ = synth_solve(w, torch.tensor(m, device="cuda"), torch.tensor(hot, device="cuda"),
                              torch.tensor(mask, device="cuda"), max_iter=iters, tol=0.0,
                              wall_mode=mode, scheme=scheme)
    assert git == iters and it == iters
    g = np_(out)
    np.testing.assert_allclose(g, ref, rtol=1e-9, atol=1e-12)
    fx = np.diff(np.asarray(w["xfaces"]))
    fy = np.diff(np.asarray(w["yfaces"])) if w["dim"] == 2 else np.ones(1)
    vol = np.outer(fy, fx).ravel()
    assert abs((g[0] * vol).sum() / (m[0] * vol).sum() - 1.0) <= 1e-12


def test_graded_checkpoint_round_trip():
    w = CASES["cavity"]
    say("case graded checkpoint")
    sim = DSMC(w)
    sim.init()
    sim.step(5)
    img = sim.save()
    sim.step(5)
    a = {k: np.array(v, copy=True) for k, v in gpu_state(sim).items()}
    sim.load(img)
    sim.step(5)
    b = {k: np.array(v, copy=True) for k, v in gpu_state(sim).items()}
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def test_fill_empty_matches_oracle():
    w = CASES["cavity"]
    say("case fill empty")
    C = w["nx"] * w["ny"]
    f = _smooth_fields(w, 9)
    rng = np.random.default_rng(10)
    idx = rng.choice(C, 40, replace=False)
    f[19, idx[:10]] = 0.0
    f[0, idx[10:20]] = 0.0
    f[4, idx[20:30]] = 0.0
    f[5, idx[30:35]] = np.nan
    f[5, idx[35:]] = -1.0
    fb = 0.5 + rng.random((6, C))
    ref = oracle.fill_empty(f, fb, dr=2)
    sim = DSMC(w)
    g = torch.tensor(f, device="cuda")
    sim.fill_empty(g, torch.tensor(fb, device="cuda"))
    np.testing.assert_array_equal(np_(g), ref)
