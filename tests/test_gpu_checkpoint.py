"""Checkpoint and resume through the C ABI (dsmc_save / dsmc_load).

A run that is saved, loaded into a fresh context (another capacity) and
stepped on must equal the uninterrupted run bit for bit: particle arrays,
cell starts, majorants, time-average accumulator and counters.  Covered: the
DIG cavity after a modification, a batch of uneven 1D instances, and the
annulus with freestream inflow (the particle count changes every step);
eager and graph-captured steps after the load.  Corrupted, truncated and
mismatched images, and images larger than the capacity, are rejected before
any device work and leave the state unchanged."""
import numpy as np
import pytest
import torch

import dig_workloads as wl
from gpu_common import DSMC, np_, say
from paper_2501_10965_amd import _lib as L

pytestmark = pytest.mark.gpu


def snapshot(sim: DSMC) -> dict:
    """Everything later steps read, copied to the host."""
    torch.cuda.synchronize()
    c = sim.counters()
    n = c["n"]
    out = {k: np_(v).copy().view(np.uint32) for k, v in sim.state(n).items()}
    out["start"] = np_(sim.array("start")).copy()
    out["sgmax"] = np_(sim.array("sgmax")).copy().view(np.uint32)
    out["acc"] = np_(sim.array("acc")).copy().view(np.uint64)
    for k in ("n", "step", "nsamp", "next_id", "candidates", "accepted", "inelastic",
              "saturated", "wall_hits", "removed", "injected", "err"):
        out["ctr_" + k] = c[k]
    return out


def assert_same(a: dict, b: dict, what: str):
    assert a.keys() == b.keys()
    for k in a:
        if isinstance(a[k], np.ndarray):
            if k == "y" and a[k].dtype == np.uint32 and len(a[k]) and what.startswith("1d"):
                continue  # a 1D state has no y
            assert np.array_equal(a[k], b[k]), f"{what}: {k} differs"
        else:
            assert a[k] == b[k], f"{what}: {k} {a[k]} != {b[k]}"


def _cavity():
    w = wl.cavity_2d(seed=77, n=48, ppc=40, kn=0.02)
    sim = DSMC(w)
    sim.init()
    sim.step(30)
    f = sim.sample("average")
    sim.adjust(f[0:6], 0)       # ids handed out, counts changed
    sim.reset_average()
    sim.step(17)
    return w, sim


def _resume_case(make, steps, graph, what, cap_scale=1.5):
    w, sim = make()
    image = sim.save()
    say(f"case {what}: image {len(image)} bytes, n={sim.counters()['n']}")
    sim.step(steps, graph=graph)
    ref = snapshot(sim)
    # a fresh context with another capacity
    other = DSMC(w, capacity=int(sim.capacity * cap_scale))
    other.load(image)
    other.step(steps, graph=graph)
    assert_same(ref, snapshot(other), what + " (fresh context)")
    # the same context rewound to the image
    sim.load(image)
    sim.step(steps, graph=graph)
    assert_same(ref, snapshot(sim), what + " (rewound)")


@pytest.mark.parametrize("graph", [False, True])
def test_cavity_resume_is_bit_exact(graph):
    _resume_case(_cavity, 23, graph, f"cavity graph={graph}")


def _batch():
    ws = wl.batch_1d(8, scale=0.05)
    sim = DSMC(ws)
    sim.init_batch()
    sim.step(12)
    return ws, sim


def test_batch_resume_is_bit_exact():
    _resume_case(_batch, 20, True, "1d batch")


def _annulus():
    w = wl.cylinder(seed=31, nth=64, nr=32, r_in=0.5, r_out=2.0, first=0.02, kn=0.05, mach=3.0,
                    n_target=60_000)
    sim = DSMC(w, cap_factor=2.0)
    sim.init()
    sim.step(15)
    return w, sim


def test_annulus_inflow_resume_is_bit_exact():
    _resume_case(_annulus, 25, False, "annulus inflow", cap_scale=1.0)


def _rejects(sim, image, code, what):
    before = sim.save()
    with pytest.raises(L.DigError) as e:
        sim.load(image)
    assert e.value.code == code, what
    assert sim.save() == before, f"{what}: state changed by a rejected load"


def test_bad_images_are_rejected_and_leave_the_state_unchanged():
    w, sim = _cavity()
    image = sim.save()
    sim.step(5)
    n = len(image)
    bad = bytearray(image)
    bad[n // 2] ^= 0x40                                  # one bit in the particle state
    _rejects(sim, bytes(bad), L.DIG_ERR_INVALID, "flipped bit")
    bad = bytearray(image)
    bad[0] ^= 1                                          # magic
    _rejects(sim, bytes(bad), L.DIG_ERR_INVALID, "magic")
    _rejects(sim, image[:-8], L.DIG_ERR_INVALID, "truncated")
    _rejects(sim, image[:100], L.DIG_ERR_INVALID, "header only")
    _rejects(sim, image + b"\0" * 8, L.DIG_ERR_INVALID, "trailing bytes")
    # another configuration (other Knudsen number, same grid)
    w2 = wl.cavity_2d(seed=77, n=48, ppc=40, kn=0.03)
    sim2 = DSMC(w2)
    sim2.init()
    _rejects(sim2, image, L.DIG_ERR_INVALID, "other configuration")
    # a capacity below the saved count
    small = DSMC(w, capacity=1000)
    with pytest.raises(L.DigError) as e:
        small.load(image)
    assert e.value.code == L.DIG_ERR_CAPACITY
    # the good image still loads after the rejections
    sim.load(image)


def test_inflow_overflow_leaves_the_particles_unchanged():
    """An inflow that does not fit the capacity enters not at all (no
    clamping): the particle count only drops by the outflow and the error
    bit is set."""
    w = wl.cylinder(seed=41, nth=64, nr=32, r_in=0.5, r_out=2.0, first=0.02, kn=0.05, mach=3.0,
                    n_target=60_000)
    probe = DSMC(w, cap_factor=2.0)
    probe.init()
    n0 = probe.counters()["n"]
    del probe
    sim = DSMC(w, capacity=n0 + 10)  # far less room than one step's inflow
    sim.init()
    c0 = sim.counters()
    assert c0["n"] == n0 and c0["err"] == 0
    sim.step(1)
    c1 = sim.counters()
    assert c1["err"] & L.EBIT_INFLOW
    assert c1["injected"] == c0["injected"]
    assert c1["next_id"] == c0["next_id"]
    assert c1["n"] == n0 - (c1["removed"] - c0["removed"])
