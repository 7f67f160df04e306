"""GPU (HIP, through the C ABI) vs FP64 oracle: one DSMC step, stage by stage,
from a common injected state.

Contract: cell indices, sort permutations, cell starts and candidate counts
bit-exact; positions after the move within 1e-5 relative; post-collision
velocities and rotational energies within 1e-5 of max(|v|, 1) except in cells
whose oracle decision margin (|u - ratio| or |u - P|) is below 1e-5, which
must stay rare; FP64 moment sums within 1e-10 relative.
"""
import zlib

import numpy as np
import pytest

import dig_workloads as wl
import oracle
from gpu_common import (DSMC, STAGES, cells_of, gpu_buffer, gpu_state, np_, oracle_state,
                        rel_close, say, sorted_arrays)

pytestmark = pytest.mark.gpu

WALLS = [("diffuse", 1.0, (0, 0, 0))] * 4


def case_workloads():
    fourier = wl.fourier_1d(seed=101, nx=40, ppc=30)
    couette = wl.batch_1d(n_inst=2, seed_base=700, scale=0.05)[1]
    cav = wl.cavity_2d(seed=202, n=24, ppc=40, kn=0.05)
    cav["dt"] *= 4.0  # more wall hits and collisions per step
    spec = wl.box(2, 10, 7, lx=1.0, ly=0.7, kn=0.05, ppc=30, seed=9,
                  bc=[("specular", 1, (0, 0, 0)), ("diffuse", 1.3, (0, 0.2, 0)),
                      ("periodic", 1, (0, 0, 0)), ("periodic", 1, (0, 0, 0))])
    big = wl.box(1, 3, kn=0.2, ppc=3000, seed=31,
                 bc=[("diffuse", 1.0, (0, 0, 0)), ("diffuse", 1.5, (0, 0, 0)),
                     ("periodic", 1, (0, 0, 0)), ("periodic", 1, (0, 0, 0))])
    vss = wl.cavity_2d(seed=203, n=24, ppc=40, kn=0.05)
    vss["alpha"] = 1.6  # VSS scattering
    vss["dt"] *= 4.0
    return {"fourier1d": fourier, "couette1d": couette, "cavity2d": cav, "specular2d": spec,
            "bigcells1d": big, "vss2d": vss}


CASES = case_workloads()


def run_stage_parity(w, seed, step=5, group=(0, 0), sg_scale=1.0, transverse=1.0):
    arrays = wl.random_sorted_state(w, seed)
    start = arrays.pop("start")
    # transverse < 1: relative velocities nearly along x (VSS rotation frame)
    for k in ("vy", "vz"):
        arrays[k] = (arrays[k] * np.float32(transverse)).astype(np.float32)
    n = len(arrays["x"])
    nc = w["nx"] * w["ny"]
    sg = np.full(nc, oracle.sgmax_default(w) * sg_scale, np.float32)
    sim = DSMC(w, capacity=int(n * 1.2) + 1024, group_particles=group[0], group_cells=group[1])
    sim.inject(arrays, start, step=step, next_id=n, sgmax=sg)
    c0 = sim.counters()
    assert c0["n"] == n and c0["step"] == step

    # ---- move ---------------------------------------------------------------
    say(f"  move: n={n} cells={nc}")
    sim.stage(STAGES["move"])
    gm = gpu_buffer(sim, c0["cur"], n)
    o = oracle_state(w, arrays, start, sg, step)
    o.move()
    om = o.arrays()
    for k in ("x", "y") if w["dim"] == 2 else ("x",):
        bad = ~rel_close(gm[k], om[k], 1e-5)
        assert bad.sum() <= max(1, n // 100000), (k, bad.sum())
    hit = np.abs(om["vx"] - arrays["vx"]) + np.abs(om["vy"] - arrays["vy"]) > 0
    for k in ("vx", "vy", "vz", "er"):
        bad = ~rel_close(gm[k], om[k], 1e-5)
        assert bad.sum() <= max(1, n // 100000), (k, bad.sum(), hit.sum())
    np.testing.assert_array_equal(gm["id"], arrays["id"])

    # ---- index + stable sort: bit-exact given the GPU's stored positions ----
    say("  sort")
    sim.stage(STAGES["sort"])
    gcell = np_(sim.array("cell"))[:n]
    gperm = np_(sim.array("perm"))[:n]
    gstart = np_(sim.array("start"))
    o2 = oracle_state(w, gm, start, sg, step)
    ocell = o2.cells()
    np.testing.assert_array_equal(gcell, ocell)
    operm = o2.sort()
    np.testing.assert_array_equal(gperm, operm)
    np.testing.assert_array_equal(gstart, o2.start)

    # ---- collide + sample ------------------------------------------------------
    say("  collide")
    pre = sorted_arrays(gm, gperm)
    o3 = oracle_state(w, pre, gstart, sg, step)
    res = o3.collide(with_obs=True)
    sim.stage(STAGES["collide"])
    c1 = sim.counters()
    assert c1["cur"] == 1 - c0["cur"] and c1["step"] == step + 1
    gc = gpu_state(sim)
    oc = o3.arrays()
    np.testing.assert_array_equal(gc["id"], oc["id"])
    np.testing.assert_array_equal(gc["x"], pre["x"])
    if w["dim"] == 2:
        np.testing.assert_array_equal(gc["y"], pre["y"])
    # candidate counts are bit-exact (FP64 Iround on identical inputs)
    assert c1["candidates"] - c0["candidates"] == res["candidates"]
    cells = cells_of(gstart)
    bad = np.zeros(n, bool)
    for k in ("vx", "vy", "vz", "er"):
        bad |= ~rel_close(gc[k], oc[k], 1e-5)
    bad_cells = np.unique(cells[bad])
    margin = res["margin"]
    assert np.all(margin[bad_cells] < 1e-5), (bad_cells, margin[bad_cells])
    decisions = 3 * res["candidates"]
    assert len(bad_cells) <= max(1, 1e-4 * decisions), (len(bad_cells), decisions)
    acc_gpu = c1["accepted"] - c0["accepted"]
    assert abs(acc_gpu - res["accepted"]) <= len(bad_cells) * 5
    gsg = np_(sim.array("sgmax"))
    ok = np.ones(nc, bool)
    ok[bad_cells] = False
    assert np.all(rel_close(gsg[ok], o3.sgmax[ok], 2e-6, floor=0.0))

    # accumulated FP64 sums of the step = sums of the GPU's post-collision state
    o4 = oracle_state(w, gc, gstart, gsg, step + 1)
    osum = o4.sums()
    gacc = np_(sim.array("acc")).reshape(nc, 17)
    scale = np.abs(osum).max(axis=0, keepdims=True) + 1e-300
    assert np.all(np.abs(gacc - osum) <= 1e-10 * scale)
    ginst = np_(sim.sample("instant"))
    ofld = o4.fields(osum, 1)
    fscale = np.abs(ofld).max(axis=1, keepdims=True) + 1e-300
    assert np.all(np.abs(ginst - ofld) <= 1e-9 * fscale)
    return res, len(bad_cells)


@pytest.mark.parametrize("name", list(CASES))
def test_single_step_stage_parity(name):
    seed = zlib.crc32(name.encode()) % 1000
    say(f"case {name} seed {seed}")
    res, nbad = run_stage_parity(CASES[name], seed=seed)
    assert res["accepted"] > 0
    say(f"  candidates={res['candidates']} accepted={res['accepted']} flipped_cells={nbad}")


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_vss_relative_velocities_near_an_axis(seed):
    """VSS with every relative velocity within a few milliradians of the x
    axis: the rotation frame of the deflection must stay well conditioned
    (post-collision states to 1e-5 like any other case)."""
    say(f"case vss near-axis seed {seed}")
    res, nbad = run_stage_parity(CASES["vss2d"], seed=100 + seed, transverse=3e-3)
    assert res["accepted"] > 0
    say(f"  candidates={res['candidates']} accepted={res['accepted']} flipped_cells={nbad}")


def test_stage_parity_small_groups_and_empty_cells():
    """Group size 256 particles / 32 cells (many groups, ragged tails), and a
    sparse state with empty and single-particle cells."""
    w = wl.cavity_2d(seed=77, n=30, ppc=3, kn=0.05)
    say("case sparse cavity, small groups")
    run_stage_parity(w, seed=5, group=(256, 32), sg_scale=8.0)


def test_init_matches_oracle():
    for name, w in (("fourier", wl.fourier_1d(seed=4, nx=50, ppc=20)),
                    ("cavity", wl.cavity_2d(seed=5, n=16, ppc=25))):
        say(f"case init {name}")
        sim = DSMC(w)
        sim.init()
        g = gpu_state(sim)
        o = oracle.new_state(w)
        om = o.arrays()
        assert len(g["x"]) == o.n
        np.testing.assert_array_equal(g["id"], om["id"])
        for k in ("x", "y") if w["dim"] == 2 else ("x",):
            assert rel_close(g[k], om[k], 1e-6).all()
        for k in ("vx", "vy", "vz", "er"):
            assert rel_close(g[k], om[k], 1e-5).all(), k
        np.testing.assert_array_equal(np_(sim.array("start")), o.start)
        np.testing.assert_array_equal(np_(sim.array("sgmax")), o.sgmax)


def test_init_iround_counts_match_oracle():
    w = wl.cavity_2d(seed=6, n=20, ppc=10)
    w["weight"] *= 10 / 6.37
    say("case init iround")
    sim = DSMC(w, capacity=20 * 20 * 12)
    sim.init(ppc=0)
    o = oracle.State(w, 20 * 20 * 12)
    o.init(wl.fields_uniform(w), 0, oracle.sgmax_default(w))
    np.testing.assert_array_equal(np_(sim.array("start")), o.start)
    g = gpu_state(sim)
    assert rel_close(g["vx"], o.vx[: o.n], 1e-5).all()


def test_library_constants_match_oracle():
    w = wl.fourier_1d()
    sim = DSMC(w)
    c = sim.constants()
    assert c["csigma"] == pytest.approx(oracle.csigma(w), rel=1e-15)
    assert c["pinelastic"] == pytest.approx(oracle.pinelastic(w), rel=1e-15)
    assert c["mu0"] == pytest.approx(oracle.mu0(w), rel=1e-15)
    assert c["volume"] == oracle.cell_volume(w)
    assert np.float32(c["sgmax_default"]) == np.float32(oracle.sgmax_default(w))
