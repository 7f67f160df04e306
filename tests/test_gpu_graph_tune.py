"""Captured step graphs, the launch-configuration autotuner, and the full-size
64-instance batch (13.7M particles) advanced by graph replays, with sampled
instances checked stage by stage against their own oracles."""
import os

import numpy as np
import pytest
import torch

import dig_workloads as wl
import oracle
from gpu_common import DSMC, STAGES, gpu_buffer, gpu_state, np_, oracle_state, rel_close, say

pytestmark = pytest.mark.gpu


def _full(sim):
    st = gpu_state(sim)
    st["start"] = np_(sim.array("start")).copy()
    st["sgmax"] = np_(sim.array("sgmax")).copy()
    st["acc"] = np_(sim.array("acc")).copy()
    c = sim.counters()
    st["ctr"] = {k: c[k] for k in ("n", "step", "nsamp", "next_id", "candidates", "accepted",
                                   "inelastic", "saturated", "wall_hits", "err")}
    return st


def _assert_same(a, b):
    assert a["ctr"] == b["ctr"]
    for k in a:
        if k != "ctr":
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def _pair(w, **kw):
    sims = []
    for _ in range(2):
        s = DSMC(w, **kw)
        s.init()
        sims.append(s)
    return sims


@pytest.mark.parametrize("nsteps", [10, 3, 150])
def test_graph_steps_match_eager(nsteps):
    """Replays of one captured graph, with eager work and synchronisation in
    between, give bit-identical states to the same steps run eagerly."""
    w = wl.cavity_2d(seed=301, n=24, ppc=30, kn=0.02)
    say(f"case graph vs eager, {nsteps} steps per graph")
    eager, graph = _pair(w)
    for rep in range(3):
        eager.step(nsteps)
        graph.step(nsteps, graph=True)
        # eager work between replays
        fe = np_(eager.sample("instant"))
        fg = np_(graph.sample("instant"))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(fe, fg)
        _assert_same(_full(eager), _full(graph))
    assert graph.counters()["step"] == 3 * nsteps


def test_graph_after_adjust_recaptures():
    """A particle-count change (DIG adjust) gives a new graph for the new size."""
    w = wl.cavity_2d(seed=302, n=16, ppc=25, kn=0.02)
    say("case graph after adjust")
    eager, graph = _pair(w)
    rng = np.random.default_rng(4)
    t = np.zeros((6, 256))
    t[0] = 1.0 + 0.2 * rng.random(256)
    t[4] = 1.0 + 0.1 * rng.random(256)
    t[5] = 1.0
    tgt = torch.tensor(t, device="cuda")
    for s, g in ((eager, False), (graph, True)):
        s.step(4, graph=g)
        s.adjust(tgt, 0)
        s.step(4, graph=g)
    _assert_same(_full(eager), _full(graph))


def test_autotune_is_result_invariant_and_cached(tmp_path):
    w = wl.cavity_2d(seed=303, n=40, ppc=30, kn=0.02)
    say("case autotune")
    a, b = _pair(w)
    cache = str(tmp_path / "tune.txt")
    t = a.autotune(steps_per_trial=2, cache_path=cache)
    assert t["group_particles"] in (512, 1024, 2048, 4096, 8192)
    assert t["group_cells"] in (32, 64, 128, 256)
    assert t["seq_max"] in (0, 64, 128, 192, 384)
    assert t["ms_per_step"] > 0
    assert a.tuning() == {**t, "ms_per_step": 0.0}
    taken = a.counters()["step"]
    assert taken >= 2 * 15
    # the tuning steps are ordinary steps: the default configuration gives the
    # same state after the same number of steps
    b.step(taken)
    _assert_same(_full(a), _full(b))
    # a second context of the same size class reads the cache without trials
    c = DSMC(w)
    c.init()
    t2 = c.autotune(steps_per_trial=2, cache_path=cache)
    assert c.counters()["step"] == 0
    assert (t2["group_particles"], t2["group_cells"], t2["seq_max"], t2["big_stage_kib"]) == \
        (t["group_particles"], t["group_cells"], t["seq_max"], t["big_stage_kib"])
    assert open(cache).read().count("\n") == 1


def test_tuning_rejects_out_of_range():
    w = wl.fourier_1d(nx=20, ppc=10)
    s = DSMC(w)
    s.init()
    from paper_2501_10965_amd import _lib as L
    for bad in (dict(group_particles=128), dict(group_cells=512), dict(seq_max=5000),
                dict(big_stage_kib=20), dict(big_stage_kib=200)):
        with pytest.raises(L.DigError):
            s.tuning(**bad)
    assert s.tuning()["group_particles"] == 1024


def _instance_parity(w, pre, start, sg, step, moved, gperm, gstart, post):
    """One step of one instance: move within 1e-5, sort exact, collide within
    1e-5 outside near-tie cells.  Arrays are the instance's own slices."""
    n = len(pre["x"])
    o = oracle_state(w, pre, start, sg, step)
    o.move()
    assert rel_close(moved["x"], o.x[:n], 1e-5).sum() >= n - max(1, n // 100000)
    o2 = oracle_state(w, moved, start, sg, step)
    operm = o2.sort()
    if gperm is not None:  # a full step keeps no permutation: the ids below check the order
        np.testing.assert_array_equal(gperm, operm)
    np.testing.assert_array_equal(gstart, o2.start)
    res = o2.collide(with_obs=True)
    np.testing.assert_array_equal(post["id"], o2.id[:n])
    cells = np.repeat(np.arange(len(gstart) - 1), np.diff(gstart))
    bad = np.zeros(n, bool)
    for k in ("vx", "vy", "vz", "er"):
        bad |= ~rel_close(post[k], getattr(o2, k)[:n], 1e-5)
    badc = np.unique(cells[bad])
    assert np.all(res["margin"][badc] < 1e-5)
    assert len(badc) <= max(1, 1e-4 * 3 * res["candidates"])
    return res


def test_full_batch_graph_and_sampled_instance_parity():
    """The 64-instance batch at full size: exact initial counts, 50 graph-captured
    steps with the autotuned configuration (particles never leave an instance),
    then one staged step and one full step (the collide ordering its cell
    groups itself, as timed) compared with the oracle on four instances from
    the smallest (2k particles) to the largest (2M)."""
    ws = wl.batch_1d(64)
    ncs = np.array([w["nx"] for w in ws])
    ppcs = np.array([w["ppc"] for w in ws])
    total = int((ncs * ppcs).sum())
    say(f"case full batch: {total} particles, {ncs.sum()} cells")
    assert total == 13_671_119
    sim = DSMC(ws, cap_factor=1.02)
    sim.init_batch()
    cell0 = np.concatenate([[0], np.cumsum(ncs)])
    st = np_(sim.array("start"))
    np.testing.assert_array_equal(np.diff(st), np.repeat(ppcs, ncs))
    t = sim.autotune(steps_per_trial=2)
    say(f"  autotuned {t}")
    sim.step(50, graph=True)
    c = sim.counters()
    assert c["n"] == total and c["err"] == 0
    st = np_(sim.array("start"))
    np.testing.assert_array_equal(st[cell0], np.concatenate([[0], np.cumsum(ncs * ppcs)]))
    # one staged step, compared per instance
    pre = gpu_state(sim)
    sg = np_(sim.array("sgmax")).copy()
    step = c["step"]
    cur = c["cur"]
    sim.stage(STAGES["move"] | STAGES["sort"])
    moved = gpu_buffer(sim, cur, total)
    gperm = np_(sim.array("perm"))[:total].copy()
    gstart = np_(sim.array("start")).copy()
    sim.stage(STAGES["collide"])
    post = gpu_state(sim)
    for i in (0, 9, 54, 63):
        w = ws[i]
        c0, c1 = cell0[i], cell0[i + 1]
        p0, p1 = st[c0], st[c1]
        assert (gstart[c0], gstart[c1]) == (p0, p1)
        say(f"  instance {i}: {p1 - p0} particles, {c1 - c0} cells")
        sl = lambda d: {k: v[p0:p1] for k, v in d.items()}  # noqa: E731
        res = _instance_parity(w, sl(pre), st[c0:c1 + 1] - p0, sg[c0:c1], step, sl(moved),
                               gperm[p0:p1] - p0, gstart[c0:c1 + 1] - p0, sl(post))
        assert res["candidates"] > 0
    # one full step as the benchmark times it (ordering inside the collide)
    pre = post
    sg = np_(sim.array("sgmax")).copy()
    start_pre = np_(sim.array("start")).copy()
    c = sim.counters()
    step, cur = c["step"], c["cur"]
    sim.step(1)
    assert sim.counters()["err"] == 0
    moved = gpu_buffer(sim, cur, total)
    gstart = np_(sim.array("start")).copy()
    post = gpu_state(sim)
    for i in (0, 9, 54, 63):
        c0, c1 = cell0[i], cell0[i + 1]
        p0, p1 = st[c0], st[c1]
        say(f"  full step, instance {i}")
        sl = lambda d: {k: v[p0:p1] for k, v in d.items()}  # noqa: E731
        res = _instance_parity(ws[i], sl(pre), start_pre[c0:c1 + 1] - p0, sg[c0:c1], step,
                               sl(moved), None, gstart[c0:c1 + 1] - p0, sl(post))
        assert res["candidates"] > 0


def test_graph_steps_refused_while_profiling():
    """Per-kernel event timing needs eager launches: a graph step with
    profiling enabled is refused and changes nothing."""
    from paper_2501_10965_amd import _lib as L
    w = wl.cavity_2d(seed=304, n=20, ppc=20, kn=0.02)
    eager, graph = _pair(w)
    graph.profile("on")
    with pytest.raises(L.DigError) as e:
        graph.step(5, graph=True)
    assert e.value.code == L.DIG_ERR_STATE
    graph.step(5)
    prof = graph.profile("read")
    graph.profile("off")
    for k in ("move", "scan", "place", "collide"):
        assert prof[k][1] == 5 and prof[k][0] > 0, (k, prof[k])
    assert prof["order"][1] == 0  # a full step orders inside the collide kernels
    eager.step(5, graph=True)
    _assert_same(_full(eager), _full(graph))


def test_profiling_a_subset_of_kernel_kinds():
    """Events only around the chosen kinds; the others run untimed."""
    from paper_2501_10965_amd import _lib as L
    w = wl.cavity_2d(seed=305, n=20, ppc=20, kn=0.02)
    s = DSMC(w)
    s.init()
    s.profile("on", kinds=["collide"])
    s.step(4)
    prof = s.profile("read")
    s.profile("off")
    assert prof["collide"][1] == 4 and prof["collide"][0] > 0
    assert all(prof[k] == (0.0, 0) for k in prof if k != "collide")
    s.profile("on")  # back to every kind
    s.step(2)
    prof = s.profile("read")
    s.profile("off")
    assert all(prof[k][1] == 2 for k in ("move", "scan", "place", "collide"))
    s.profile("on", kinds=["collide", "move"], every=3)  # launches 0, 3, 6 of each
    s.step(7)
    prof = s.profile("read")
    s.profile("off")
    assert prof["collide"][1] == 3 and prof["move"][1] == 3 and prof["scan"][1] == 0
    with pytest.raises(L.DigError):
        L.check(s.lib.dsmc_profile_kinds(s.ctx, 1 << len(L.KERNELS), 1))
    with pytest.raises(L.DigError):
        L.check(s.lib.dsmc_profile_kinds(s.ctx, 1, 0))
