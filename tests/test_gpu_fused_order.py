"""A full step orders each cell group inside the collide kernel; the staged
path orders the whole permutation in a pass of its own.  Both must give
bit-identical states: small cells (ordered by counting ranks), cells above
that size in groups that fit the shared-memory stage (ordered from the move's
runs), groups too large for that stage but not for the oversize-group
kernel's, groups too large for both (ordered in global memory), and steps
where particles leave through an open boundary."""
import numpy as np
import pytest

import dig_workloads as wl
from gpu_common import DSMC, STAGES, np_, say

pytestmark = pytest.mark.gpu


def _snap(sim):
    st = {k: np_(v).copy() for k, v in sim.state().items()}
    if sim.workloads[0]["dim"] == 1:
        st.pop("y")  # not part of a 1D state
    st["start"] = np_(sim.array("start")).copy()
    st["sgmax"] = np_(sim.array("sgmax")).copy()
    st["acc"] = np_(sim.array("acc")).copy()
    c = sim.counters()
    st["ctr"] = [c[k] for k in ("n", "step", "nsamp", "candidates", "accepted", "inelastic")]
    return st


CASES = {
    "cavity": lambda: wl.cavity_2d(seed=401, n=32, ppc=40, kn=0.02),
    # cells of ~200 particles in groups that fit the LDS stage: ordered from
    # the move's runs (cells above the rank-counting size)
    "midcells": lambda: wl.box(1, 40, kn=0.05, ppc=200, seed=404,
                               bc=[("diffuse", 1.0, (0, 0, 0)), ("diffuse", 1.3, (0, 0, 0)),
                                   ("periodic", 1, (0, 0, 0)), ("periodic", 1, (0, 0, 0))]),
    # cells of ~700 particles: groups of two exceed the small-group stage and
    # are ordered and collided in the oversize-group kernel's LDS stage
    "stagecells": lambda: wl.box(1, 30, kn=0.1, ppc=700, seed=405,
                                 bc=[("diffuse", 1.0, (0, 0, 0)), ("diffuse", 1.2, (0, 0, 0)),
                                     ("periodic", 1, (0, 0, 0)), ("periodic", 1, (0, 0, 0))]),
    "bigcells": lambda: wl.box(1, 6, kn=0.2, ppc=3000, seed=402,
                               bc=[("diffuse", 1.0, (0, 0, 0)), ("diffuse", 1.5, (0, 0, 0)),
                                   ("periodic", 1, (0, 0, 0)), ("periodic", 1, (0, 0, 0))]),
    "cylinder": lambda: wl.cylinder(seed=403, nth=64, nr=32, r_in=0.5, r_out=2.0, first=0.02,
                                    kn=0.05, mach=3.0, n_target=60_000),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("group", [(0, 0), (256, 32)])
def test_fused_step_equals_staged_step(name, group):
    w = CASES[name]()
    say(f"case fused vs staged: {name} groups {group}")
    a = DSMC(w, group_particles=group[0], group_cells=group[1])
    b = DSMC(w, group_particles=group[0], group_cells=group[1])
    a.init()
    b.init()
    for _ in range(6):
        a.step(1)
        b.stage(STAGES["move"] | STAGES["sort"])
        b.stage(STAGES["collide"])
        sa, sb = _snap(a), _snap(b)
        assert sa["ctr"] == sb["ctr"]
        for k in sa:
            if k != "ctr":
                np.testing.assert_array_equal(sa[k], sb[k], err_msg=k)


@pytest.mark.parametrize("name", ["stagecells", "bigcells", "cylinder"])
def test_oversize_stage_budget_is_result_invariant(name):
    """The LDS budget of the oversize-group kernel (38 to 150 KiB) decides
    which groups it collides in LDS and which in HBM; every budget gives the
    same state, bit for bit."""
    w = CASES[name]()
    say(f"case oversize stage budgets: {name}")
    snaps = []
    for kib in (38, 50, 76, 150):
        s = DSMC(w, group_particles=4096, group_cells=64)
        s.tuning(big_stage_kib=kib)
        s.init()
        s.step(5)
        snaps.append(_snap(s))
    for other in snaps[1:]:
        assert other["ctr"] == snaps[0]["ctr"]
        for k in other:
            if k != "ctr":
                np.testing.assert_array_equal(other[k], snaps[0][k], err_msg=k)
