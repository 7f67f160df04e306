"""GPU vs oracle with rotational degrees of freedom other than 2 (d_r = 3..6:
Gamma(d_r/2) equilibrium energies, Borgnakke-Larsen fractions
Beta(d_r/2, 5/2 - omega) by acceptance-rejection), alone and with VSS
scattering: one step stage by stage (cell indices, permutations, candidate
counts bit-exact; post-collision state within 1e-5 outside decision-margin
cells), initialisation and the DIG modification's refill of empty cells."""
import zlib

import numpy as np
import pytest
import torch

import dig_workloads as wl
import oracle
from gpu_common import DSMC, gpu_state, np_, oracle_state, rel_close, say
from test_gpu_dig_closure import injected, random_target
from test_gpu_step_parity import run_stage_parity

pytestmark = pytest.mark.gpu


def cases():
    cav3 = wl.cavity_2d(seed=402, n=24, ppc=40, kn=0.05)
    cav3["dr"] = 3
    cav3["dt"] *= 4.0
    four5 = wl.fourier_1d(seed=403, nx=40, ppc=60)
    four5["dr"] = 5
    vss4 = wl.cavity_2d(seed=404, n=20, ppc=40, kn=0.05)
    vss4["dr"] = 4
    vss4["alpha"] = 1.5
    vss4["dt"] *= 4.0
    six = wl.fourier_1d(seed=405, nx=30, ppc=80)
    six["dr"] = 6
    return {"cavity_dr3": cav3, "fourier_dr5": four5, "vss_dr4": vss4, "fourier_dr6": six}


CASES = cases()


@pytest.mark.parametrize("name", list(CASES))
def test_stage_parity(name):
    seed = zlib.crc32(name.encode()) % 1000
    say(f"case {name} seed {seed}")
    res, nbad = run_stage_parity(CASES[name], seed=seed)
    assert res["accepted"] > 0 and res["inelastic"] > 0
    say(f"  candidates={res['candidates']} accepted={res['accepted']} "
        f"inelastic={res['inelastic']} flipped={nbad}")


@pytest.mark.parametrize("name", ["cavity_dr3", "fourier_dr5"])
def test_init_matches_oracle(name):
    w = dict(CASES[name])
    say(f"case init {name}")
    sim = DSMC(w)
    sim.init()
    g = gpu_state(sim)
    o = oracle.new_state(w)
    om = o.arrays()
    np.testing.assert_array_equal(g["id"], om["id"])
    np.testing.assert_array_equal(np_(sim.array("start")), o.start)
    for k in ("vx", "vy", "vz", "er"):
        assert rel_close(g[k], om[k], 1e-5).all(), k
    # Gamma(d_r/2) energies: mean (d_r/2) Tr
    dr = w["dr"]
    assert abs(g["er"].mean() / (0.5 * dr * w["init"]["Tr"]) - 1.0) < 0.02


def test_adjust_refill_matches_oracle():
    w = dict(CASES["cavity_dr3"])
    say("case adjust d_r 3")
    sim, arrays, start, sg, n = injected(w, seed=9)
    rng = np.random.default_rng(4)
    t = random_target(w, rng)
    t[0, :4] = 0.0
    o = oracle_state(w, arrays, start, sg, 3, cap=4 * n, next_id=n + 17)
    assert o.adjust(t, dig_iter=2) == 0
    sim.adjust(torch.tensor(t, device="cuda"), 2)
    g = gpu_state(sim)
    c = sim.counters()
    o = oracle_state(w, g, np_(sim.array("start")), np_(sim.array("sgmax")), 3, cap=4 * n,
                     next_id=c["next_id"])
    t2 = t.copy()
    t2[0, :4] = 1.0
    assert o.adjust(t2, dig_iter=3) == 0
    sim.adjust(torch.tensor(t2, device="cuda"), 3)
    g = gpu_state(sim)
    om = o.arrays()
    np.testing.assert_array_equal(g["id"], om["id"])
    np.testing.assert_array_equal(np_(sim.array("start")), o.start)
    for k in ("x", "y", "vx", "vy", "vz", "er"):
        assert rel_close(g[k], om[k], 2e-6).all(), k
