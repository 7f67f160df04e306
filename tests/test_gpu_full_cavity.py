"""The lid-driven cavity at full size (200 x 200 cells, 50 particles per cell,
about 2M particles, Kn 0.01), in the launch configuration the benchmark times:
the autotuned cell groups, full steps in which the collide orders each cell
group itself (no ordering pass), graph-captured step sequences and the DIG
particle modification (Section 3.2).

The oracle runs the whole state at this size in seconds, so every particle and
every cell is compared, from seeded cell-sorted states:

* one full step, stage by stage (the oracle sorts and collides the GPU's moved
  positions): the move within 1e-5 relative, the stable sort and the cell
  starts exactly, candidate counts exactly, post-collision velocities and
  energies within 1e-5 outside cells whose oracle decision margin is below
  1e-5, the step's FP64 moment sums within 1e-10;
* the particle modification toward a per-cell target: counts, ids and order
  exactly, positions within 1e-6, velocities within 2e-6;
* 50 steps launched as captured graphs equal the same steps launched eagerly,
  bit for bit;
* whole DIG cycles repeat bit for bit in fresh device memory and under another
  launch configuration."""
import numpy as np
import pytest
import torch

import dig_workloads as wl
import oracle
from gpu_common import DSMC, cells_of, gpu_buffer, gpu_state, np_, oracle_state, rel_close, say

pytestmark = pytest.mark.gpu

STEP0 = 7


@pytest.fixture(scope="module")
def tuned():
    """The workload and the configuration the autotuner picks for it."""
    w = wl.cavity_2d()
    sim = DSMC(w)
    sim.init()
    t = sim.autotune(steps_per_trial=5)
    say(f"case full cavity: autotuned {t}")
    del sim
    return w, t


def _context(w, t, arrays, start, sg, capacity):
    sim = DSMC(w, capacity=capacity)
    sim.tuning(t["group_particles"], t["group_cells"], t["seq_max"], t["big_stage_kib"])
    sim.inject(arrays, start, step=STEP0, next_id=len(arrays["x"]), sgmax=sg)
    sim.reset_average()
    return sim


def _seeded(w, seed):
    arrays = wl.random_sorted_state(w, seed)
    start = arrays.pop("start")
    sg = np.full(w["nx"] * w["ny"], oracle.sgmax_default(w), np.float32)
    return arrays, start, sg


def test_full_size_step_matches_oracle(tuned):
    w, t = tuned
    arrays, start, sg = _seeded(w, 2002)
    n = len(arrays["x"])
    nc = w["nx"] * w["ny"]
    say(f"  full step: {n} particles, {nc} cells")
    sim = _context(w, t, arrays, start, sg, int(n * 1.2) + 1024)
    c0 = sim.counters()
    sim.step(1)
    c1 = sim.counters()
    assert c1["step"] == STEP0 + 1 and c1["n"] == n and c1["err"] == 0
    assert c1["cur"] == 1 - c0["cur"]
    moved = gpu_buffer(sim, c0["cur"], n)
    post = gpu_state(sim)
    gstart = np_(sim.array("start")).copy()
    gsg = np_(sim.array("sgmax")).copy()
    gacc = np_(sim.array("acc")).reshape(nc, 17).copy()

    # move: positions, and the velocities of particles that hit a wall
    o = oracle_state(w, arrays, start, sg, STEP0)
    o.move()
    om = o.arrays()
    for k in ("x", "y", "vx", "vy", "vz", "er"):
        bad = ~rel_close(moved[k], om[k], 1e-5)
        assert bad.sum() <= max(1, n // 100000), (k, bad.sum())
    np.testing.assert_array_equal(moved["id"], arrays["id"])

    # stable sort of the GPU's moved positions: exact
    o2 = oracle_state(w, moved, start, sg, STEP0)
    o2.sort()
    np.testing.assert_array_equal(gstart, o2.start)
    np.testing.assert_array_equal(post["id"], o2.id[:n])
    np.testing.assert_array_equal(post["x"], o2.x[:n])
    np.testing.assert_array_equal(post["y"], o2.y[:n])

    # collide
    res = o2.collide(with_obs=True)
    assert c1["candidates"] - c0["candidates"] == res["candidates"]
    say(f"  {res['candidates']} candidates, {res['accepted']} accepted")
    cells = cells_of(gstart)
    bad = np.zeros(n, bool)
    for k in ("vx", "vy", "vz", "er"):
        bad |= ~rel_close(post[k], getattr(o2, k)[:n], 1e-5)
    bad_cells = np.unique(cells[bad])
    assert np.all(res["margin"][bad_cells] < 1e-5), bad_cells
    assert len(bad_cells) <= max(1, 1e-4 * 3 * res["candidates"]), len(bad_cells)
    ok = np.ones(nc, bool)
    ok[bad_cells] = False
    assert np.all(rel_close(gsg[ok], o2.sgmax[ok], 2e-6, floor=0.0))

    # the step's FP64 sums are those of the GPU's post-collision state
    osum = oracle_state(w, post, gstart, gsg, STEP0 + 1).sums()
    scale = np.abs(osum).max(axis=0, keepdims=True) + 1e-300
    assert np.all(np.abs(gacc - osum) <= 1e-10 * scale)


def _target(w, seed):
    """Per-cell (rho, ux, uy, uz, Tt, Tr) around the cavity's initial state."""
    rng = np.random.default_rng(seed)
    nc = w["nx"] * w["ny"]
    t = np.empty((6, nc))
    t[0] = 1.0 + 0.1 * rng.standard_normal(nc)
    t[1:4] = 0.05 * rng.standard_normal((3, nc))
    t[4] = 1.0 + 0.05 * rng.standard_normal(nc)
    t[5] = 1.0 + 0.05 * rng.standard_normal(nc)
    return t


def test_full_size_modification_then_graph_steps(tuned):
    w, t = tuned
    arrays, start, sg = _seeded(w, 2003)
    n = len(arrays["x"])
    tgt = _target(w, 2004)
    say(f"  modification: {n} particles")
    o = oracle_state(w, arrays, start, sg, STEP0, cap=3 * n, next_id=n)
    assert o.adjust(tgt, 3) == 0
    sims = []
    for _ in range(2):
        sim = _context(w, t, arrays, start, sg, int(n * 1.5))
        sim.adjust(torch.tensor(tgt, device="cuda"), 3)
        sims.append(sim)
    c = sims[0].counters()
    assert c["n"] == o.n and c["next_id"] == o.next_id and c["err"] == 0
    np.testing.assert_array_equal(np_(sims[0].array("start")), o.start)
    g = gpu_state(sims[0])
    om = o.arrays()
    np.testing.assert_array_equal(g["id"], om["id"])
    for k in ("x", "y"):
        assert rel_close(g[k], om[k], 1e-6).all(), k
    for k in ("vx", "vy", "vz", "er"):
        assert rel_close(g[k], om[k], 2e-6).all(), k

    say("  50 steps, eager and graph-captured")
    sims[0].step(50)
    sims[1].step(50, graph=True)
    ca, cb = sims[0].counters(), sims[1].counters()
    assert ca == cb
    assert ca["n"] == o.n and ca["err"] == 0 and ca["step"] == STEP0 + 50
    sa, sb = gpu_state(sims[0]), gpu_state(sims[1])
    for k in sa:
        np.testing.assert_array_equal(sa[k], sb[k], err_msg=k)
    for name in ("start", "sgmax", "acc"):
        np.testing.assert_array_equal(np_(sims[0].array(name)), np_(sims[1].array(name)),
                                      err_msg=name)


def test_full_size_dig_cycles_repeat_bit_for_bit():
    """DIG cycles (50 steps, closure, synthetic solve of 2000 pseudo-time
    steps, modification) on the full cavity give the same particles on a rerun
    in fresh device memory and under another launch configuration."""
    from paper_2501_10965_amd.dig import DIG

    def run(tune):
        d = DIG(wl.cavity_2d())
        if tune:
            d.sim.tuning(*tune)
        out = []
        for _ in range(3):
            d.cycle()
            out.append((gpu_state(d.sim), d.sim.counters()["n"]))
        return out

    say("  DIG cycles: default, rerun, other tuning")
    a = run(None)
    for other in (run(None), run((512, 128, 0))):
        for (sa, na), (sb, nb) in zip(a, other):
            assert na == nb
            for k in sa:
                np.testing.assert_array_equal(sa[k], sb[k], err_msg=k)
