"""Host arithmetic of bench.py's roofline (no GPU): the algorithmic bytes per
particle and per cell of the collide stage, the achieved and traffic rates of
one launch, and the counter summaries' digest guard and per-particle scaling."""
import math

import bench

N, C = 2_000_000, 40_000


def test_algorithmic_bytes_of_the_collide_stage():
    # per particle: provisional source 4 B + the state read unsorted and written
    # sorted (2 x 28 B in 2D, 2 x 24 B in 1D); per cell: start pair 4, majorant
    # read + write 8, instance 4, 17 FP64 sums read + written
    assert bench.collide_particle_bytes(2) == 4 + 2 * 28
    assert bench.collide_particle_bytes(1) == 4 + 2 * 24
    assert bench.PER_CELL_BYTES == 4 + 8 + 4 + 2 * 17 * 8 == 288
    # the network's forward flops per sample (unpadded 9-128-128-128-7)
    assert bench.MLP_FWD_FLOP == 69632 and bench.MLP_TRAIN_FLOP == 3 * 69632


def test_roofline_rates_of_one_launch():
    prof = {"collide": (0.75, 10), "move": (0.2, 10)}  # ms over 10 launches
    bd = {"collide": (0.75, 10), "move": (0.2, 10)}
    r = bench.roofline(prof, bd, N, C, "no-such-workload", 2)
    alg = 60 * N + 288 * C
    avg_s = 0.075e-3
    assert r["algorithmic_bytes_per_launch"] == alg
    assert math.isclose(r["achieved"], round(alg / avg_s / 1e9, 1))
    assert math.isclose(r["frac"], round(alg / avg_s / 1e9 / 8000.0, 4))
    assert r["traffic"] is None and "traffic_frac" not in r  # no counter summary


def test_traffic_fields_follow_the_counter_summary():
    prof = bd = {"collide": (0.75, 10)}
    r = bench.roofline(prof, bd, N, C, "cavity", 2)
    t = bench.pmc_traffic("collide", "cavity", N)
    assert r["traffic"] == t
    if t is None:  # kernel sources changed since the counters were taken
        return
    avg_s = 0.075e-3
    assert math.isclose(r["traffic_GBs"], round(t / avg_s / 1e9, 1))
    assert math.isclose(r["traffic_frac"], round(t / avg_s / 1e9 / 8000.0, 4))
    assert math.isclose(r["traffic_over_algorithmic"],
                        round(t / r["algorithmic_bytes_per_launch"], 3))


def test_cylinder_traffic_scales_per_particle():
    a = bench.pmc_traffic("collide", "cylinder", 50_000_000)
    b = bench.pmc_traffic("collide", "cylinder", 100_000_000)
    if a is None:
        assert b is None
        return
    assert abs(b - 2 * a) <= 2
