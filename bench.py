#!/usr/bin/env python
"""DSMC + DIG hot-path benchmark on one MI355X.

Default workload (--workload cylinder): the largest single-GPU
configuration, Mach 5 flow of a diatomic gas past a cylinder (annulus
0.5 < r < 5.5, 500 x 400 stretched polar cells, about 50M particles at the
freestream density, Kn 0.01, freestream inflow and outflow every step, plain
DSMC), timed after an untimed pre-roll from the start at rest that lets the
bow shock form.  Its working set (about 3 GB) is far beyond the 256 MB
last-level cache, so the collide roofline is an HBM figure.

--workload cavity: the DIG-coupled 2D lid-driven cavity (200 x 200 cells, 50
particles per cell = 2,000,000 particles, Kn = 0.01, lid Ma = 0.3,
omega = 0.74, Z = 5, N_s = 50).  A timed "step" is one DSMC step (move + walls,
cell index + stable sort, NTC/VHS/BL collide, FP64 sampling); every N_s steps
the DIG cycle runs (time-averaged fields, closure assembly, particle
modification).  Inside the timed region the kernels are launched eagerly,
with HIP events around one collide launch in every ten (the dominant kernel,
whose average duration gives the roofline; timing-only events without a
system fence), and the modification target is the
time-averaged DSMC field.  The per-kernel breakdown comes from a shorter,
untimed run of the same loop with events around every kernel.  Two more regions follow
and are reported beside it: the same loop with the N_s steps as one captured
HIP graph ("graph_replay"), and the full DIG loop with the synthetic-equation
solve as the target ("dig_loop").

--workload batch: 64 uneven 1D instances (13,671,119 particles) advanced
together by graph replays, plain DSMC.

--workload sweep: the cavity family from 1M to 100M particles, showing where
the step leaves the last-level cache and becomes HBM-bound.

--workload synth: the synthetic-equation solve alone on the 200 x 200 cavity
grid (LU-SGS and explicit, fixed iteration counts).

Prints one JSON line: particle-steps/s, the roofline of the dominant kernel
(HIP events around every kernel inside the timed region), and the FP64 oracle
timed on the host for a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DSMC particle-steps/s; time-to-steady-state at fixed error, learned vs plain"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per particle-step of the whole step: state (x[, y], v, er,
# id) read once and written once
STATE_BYTES = {1: 24, 2: 28}
# collide kernel (stable order of each cell group, gather, collisions,
# sampling): per particle its provisional source index (4 B) read, the state
# read from the unsorted buffer and written to the sorted one; per cell the
# start pair (4 B), majorant read + write (8 B), instance tag (4 B) and the
# FP64 accumulator of 17 sums read + written
def collide_particle_bytes(dim):
    return 4 + 2 * STATE_BYTES[dim]


PER_CELL_BYTES = 4 + 8 + 4 + 2 * 17 * 8
# DIG cycles of the untimed per-kernel breakdown run (cavity)
BREAKDOWN_CYCLES = 4
# inside the timed region, HIP events around one collide launch in every 10
PROFILE_EVERY = 10
KERNEL_SOURCES = ("paper_2501_10965_amd/csrc/dig_kernels.hip",
                  "paper_2501_10965_amd/csrc/dig_internal.h")


def default_A(omega):
    return [2.0 / 3.0, 0.0, 0.0, 5.0 / (7.0 - 2.0 * omega)]


def source_digest() -> str:
    """Hash of the kernel sources' code (comments and whitespace removed), so
    that counters taken on the same code stay valid across comment edits."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def pmc_traffic(kernel: str, workload: str, n_avg: float):
    """HBM bytes per dispatch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    when there is none or the kernel sources changed since it was taken.
    Where the summary records its particle count, the bytes are scaled per
    particle to n_avg (the cylinder's count grows over a long window)."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_digest:\s*(\w+)", text)
    f = re.search(r"fetch_bytes_per_dispatch:\s*([\d.eE+]+)", text)
    w = re.search(r"write_bytes_per_dispatch:\s*([\d.eE+]+)", text)
    if not (m and f and w) or m.group(1) != source_digest():
        return None
    t = float(f.group(1)) + float(w.group(1))
    n = re.search(r"particles_per_dispatch:\s*([\d.eE+]+)", text)
    return round(t * n_avg / float(n.group(1))) if n else t


def roofline(prof, breakdown, n_avg, ncell, workload, dim):
    """Roofline of the kernel that dominates the breakdown, from its events in
    the timed region (prof)."""
    name = max(breakdown.items(), key=lambda kv: kv[1][0])[0]
    ms, launches = prof[name]
    avg_s = ms / max(launches, 1) / 1e3
    if name != "collide":
        return {"bound": "hbm", "kernel": name, "achieved": None, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": None, "traffic": None,
                "avg_launch_us": round(avg_s * 1e6, 2)}
    alg = collide_particle_bytes(dim) * n_avg + PER_CELL_BYTES * ncell
    ach = alg / avg_s / 1e9
    traffic = pmc_traffic("collide", workload, n_avg)
    out = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
           "kernel": "k_collide + k_collide_big (collide stage, one launch each per step)",
           "avg_launch_us": round(avg_s * 1e6, 2),
           "algorithmic_bytes_per_launch": int(alg)}
    if traffic:
        # the rate of the measured HBM bytes beside the algorithmic one: what the
        # memory system actually moves (partial sectors, re-reads) per launch
        out["traffic_GBs"] = round(traffic / avg_s / 1e9, 1)
        out["traffic_frac"] = round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4)
        out["traffic_over_algorithmic"] = round(traffic / alg, 3)
    return out


def summarise(prof, breakdown, psteps, sec, nsteps, n_avg, ncell, dim, workload):
    """prof: events of the timed region (the collide only); breakdown: events
    around every kernel of a separate, untimed run of the same loop."""
    step_bytes = STATE_BYTES[dim] * 2 + PER_CELL_BYTES * ncell / n_avg
    step_alg = step_bytes * psteps / sec / 1e9
    return dict(
        value=psteps / sec, ms_per_step=sec / nsteps * 1e3,
        roofline=roofline(prof, breakdown, n_avg, ncell, workload, dim),
        kernels_us={k: round(v[0] / max(v[1], 1) * 1e3, 2) for k, v in breakdown.items()
                    if v[1]},
        kernel_launches={k: v[1] for k, v in breakdown.items() if v[1]},
        step_roofline={"achieved_algorithmic_GBs": round(step_alg, 1),
                       "frac": round(step_alg / HBM_PEAK_GBS, 4),
                       "bytes_per_particle_step": round(step_bytes, 2)})


def run_cavity(args):
    import torch

    import dig_workloads as wl
    from paper_2501_10965_amd.dsmc import DSMC, synth_solve

    w = wl.cavity_2d(seed=2001)
    ns = w["ns"]
    sim = DSMC(w, group_particles=args.group_particles, group_cells=args.group_cells)
    if args.seq_max >= 0:
        sim.tuning(seq_max=args.seq_max)
    sim.init()
    A = default_A(w["omega"])
    state = {"step": 0, "cycle": 0, "n": sim.counters()["n"]}

    def dig_cycle(target=None):
        f = sim.sample("average")
        hot, mask, _, _ = sim.closure(f, A, 0.01, n_min=1.0)
        if target == "synth":
            tgt, it, ch = synth_solve(w, f, hot, mask, A, wall_mode="dsmc",
                                      max_iter=args.synth_iters, tol=1e-5,
                                      scheme=args.synth_scheme)
        else:
            tgt, it = f[0:6], 0
        sim.adjust(tgt, state["cycle"])
        sim.reset_average()
        state["cycle"] += 1
        state["n"] = sim.counters()["n"]
        return it

    def run(nsteps, counts, target=None, graph=False):
        done = 0
        its = []
        while done < nsteps:
            k = min(ns - state["step"] % ns, nsteps - done)
            sim.step(k, graph=graph)
            counts.append((k, state["n"]))
            state["step"] += k
            done += k
            if state["step"] % ns == 0:
                its.append(dig_cycle(target))
        return its

    tuning = None
    if not args.no_autotune:
        tuning = sim.autotune(steps_per_trial=5)
        taken = sim.counters()["step"]
        state["step"] = taken
    # warm up to a cycle boundary at or after the requested warmup
    tgt = -(-max(args.warmup, state["step"]) // ns) * ns
    run(tgt - state["step"], [], graph=True)
    # per-kernel breakdown: events around every kernel, outside the timed region
    sim.profile("on")
    run(BREAKDOWN_CYCLES * ns, [])
    breakdown = sim.profile("read")
    sim.profile("off")
    torch.cuda.synchronize()
    sim.profile("on", kinds=["collide"], every=PROFILE_EVERY)
    counts = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step0 = state["step"]
    cycles_timed = len(run(args.steps, counts))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile("read")
    sim.profile("off")
    ctr = sim.counters()
    psteps = sum(k * n for k, n in counts)
    n_avg = psteps / max(args.steps, 1)
    out = summarise(prof, breakdown, psteps, t1 - t0, args.steps, n_avg, w["nx"] * w["ny"], 2,
                    "cavity")
    # the same loop with graph-captured steps
    run((-state["step"]) % ns, [], graph=True)
    torch.cuda.synchronize()
    cg = []
    tg0 = time.perf_counter()
    run(args.steps, cg, graph=True)
    torch.cuda.synchronize()
    tg1 = time.perf_counter()
    out["graph_replay"] = {"value": sum(k * n for k, n in cg) / (tg1 - tg0),
                           "unit": "particle-steps/s", "steps": args.steps,
                           "ms_per_step": (tg1 - tg0) / args.steps * 1e3}
    # the full DIG loop: N_s steps + closure + synthetic solve + modification
    dig = None
    if args.dig_cycles > 0:
        run((-state["step"]) % ns, [], graph=True)
        torch.cuda.synchronize()
        c2 = []
        t2 = time.perf_counter()
        its = run(args.dig_cycles * ns, c2, target="synth", graph=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        ps2 = sum(k * n for k, n in c2)
        dig = {"value": ps2 / (t3 - t2), "unit": "particle-steps/s", "cycles": args.dig_cycles,
               "synth_iterations": its, "ms_per_cycle": (t3 - t2) / args.dig_cycles * 1e3,
               "dsmc_ms_per_cycle": ns * out["ms_per_step"]}
    dig_what = ("no DIG cycle falls inside it" if cycles_timed == 0 else
                f"{cycles_timed} DIG cycle(s) (closure + modification toward the "
                f"time-averaged field) fall inside it")
    out.update(particles=int(n_avg), cells=w["nx"] * w["ny"], err_bits=ctr["err"],
               collisions_per_particle_step=ctr["accepted"] * 2 / max(ctr["step"] * n_avg, 1),
               tuning=tuning, dig_loop=dig, dig_cycles_timed=cycles_timed,
               timed_steps=[step0, step0 + args.steps],
               workload=f"{w['name']} 200x200 cells, 50 ppc (2M particles, working set inside "
                        f"the 256 MB last-level cache), Kn 0.01, lid Ma 0.3, DIG every 50 "
                        f"steps; the timed window is steps {step0}-{step0 + args.steps} and "
                        f"{dig_what}")
    return out, w


def run_batch(args):
    import torch

    import dig_workloads as wl
    from paper_2501_10965_amd.dsmc import DSMC

    ws = wl.batch_1d(64)
    sim = DSMC(ws, cap_factor=1.02, group_particles=args.group_particles,
               group_cells=args.group_cells)
    if args.seq_max >= 0:
        sim.tuning(seq_max=args.seq_max)
    sim.init_batch()
    n = sim.counters()["n"]
    tuning = None if args.no_autotune else sim.autotune(steps_per_trial=10)
    graph = 50
    k0 = sim.counters()["step"]
    sim.step(max(args.warmup - k0, 0) // graph * graph + graph, graph=True)
    sim.profile("on")
    sim.step(2 * graph)
    breakdown = sim.profile("read")
    sim.profile("off")
    torch.cuda.synchronize()
    sim.profile("on", kinds=["collide"], every=PROFILE_EVERY)
    steps = max(graph, args.steps // graph * graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // graph):
        sim.step(graph)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile("read")
    sim.profile("off")
    ctr = sim.counters()
    ncell = sim.ncell
    out = summarise(prof, breakdown, n * steps, t1 - t0, steps, n, ncell, 1, "batch")
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    for _ in range(steps // graph):
        sim.step(graph, graph=True)
    torch.cuda.synchronize()
    tg1 = time.perf_counter()
    out["graph_replay"] = {"value": n * steps / (tg1 - tg0), "unit": "particle-steps/s",
                           "steps": steps, "ms_per_step": (tg1 - tg0) / steps * 1e3}
    out.update(particles=n, cells=ncell, err_bits=ctr["err"], tuning=tuning, dig_loop=None,
               steps_run=steps,
               collisions_per_particle_step=ctr["accepted"] * 2 / max(ctr["step"] * n, 1),
               workload="64 uneven 1D Couette/Fourier instances, 13,671,119 particles, Kn "
                        "1e-3..1, plain DSMC, 50-step graphs")
    args.steps = steps
    return out, ws[63]


# closure network: multiply-adds of the real (unpadded) layers per sample
MLP_FWD_FLOP = 2 * (9 * 128 + 128 * 128 + 128 * 128 + 128 * 7)
MLP_TRAIN_FLOP = 3 * MLP_FWD_FLOP
MFMA_BF16_PEAK_TFLOPS = 2500.0


def run_mlp(args):
    """Closure-network training (batch 65,536, Adam) and inference throughput
    (2^20 samples)."""
    import numpy as np
    import torch

    import dig_workloads as wl
    from paper_2501_10965_amd.mlp import MLP

    batch, n_inf = 65536, 1 << 20
    net = MLP(wl.mlp_init(7), max_batch=batch)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    x = torch.randn((batch, 9), device="cuda", generator=g)
    t = torch.tanh(x[:, :7]).contiguous()
    xi = torch.randn((n_inf, 9), device="cuda", generator=g)
    yi = torch.empty((n_inf, 7), device="cuda")
    for _ in range(max(args.warmup, 10)):
        net.train_step(x, t, 1e-3)
        net.forward(xi, out=yi)
    steps = max(args.steps, 10)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e[0].record()
    for _ in range(steps):
        net.train_step(x, t, 1e-3)
    e[1].record()
    for _ in range(steps):
        net.forward(xi, out=yi)
    e[2].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    train_s = e[0].elapsed_time(e[1]) / 1e3 / steps
    inf_s = e[1].elapsed_time(e[2]) / 1e3 / steps
    train_tf = MLP_TRAIN_FLOP * batch / train_s / 1e12
    inf_tf = MLP_FWD_FLOP * n_inf / inf_s / 1e12
    return {
        "value": batch * steps / (e[0].elapsed_time(e[1]) / 1e3), "unit": "samples/s",
        "metric": "closure-network training samples/s (batch 65536, Adam)",
        "ms_per_step": train_s * 1e3, "steps": steps,
        "roofline": {"bound": "mfma", "achieved": round(inf_tf, 2),
                     "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(inf_tf / MFMA_BF16_PEAK_TFLOPS, 5), "traffic": None,
                     "kernel": "k_mlp_infer (inference, 2^20 samples)",
                     "avg_launch_us": round(inf_s * 1e6, 2),
                     "algorithmic_flop_per_launch": MLP_FWD_FLOP * n_inf},
        "training_tflops": round(train_tf, 3),
        "training_frac": round(train_tf / MFMA_BF16_PEAK_TFLOPS, 5),
        "inference_samples_per_s": n_inf / inf_s,
        "wall_s": t1 - t0,
    }


def run_synth(args):
    """Synthetic-equation solve on the 200 x 200 cavity grid (Kn 0.01): a
    seeded state near rest at unit density and temperature with small
    perturbations, masked higher-order terms of the size the DSMC extracts,
    fixed iteration counts (LU-SGS --synth-iters, explicit 2000), timed with
    HIP events over whole solves."""
    import numpy as np
    import torch

    import dig_workloads as wl
    from paper_2501_10965_amd.dsmc import synth_solve

    n = 200
    w = wl.cavity_2d(n=n, kn=0.01)
    rng = np.random.default_rng(5)
    nc = n * n
    m = np.zeros((20, nc))
    m[0] = 1.0 + 0.05 * rng.standard_normal(nc)
    m[1:3] = 0.05 * rng.standard_normal((2, nc))
    m[4:6] = 1.0 + 0.03 * rng.standard_normal((2, nc))
    hot = 0.005 * rng.standard_normal((12, nc))
    mask = (rng.random(nc) < 0.3).astype(np.uint8)
    dev = [torch.tensor(a, device="cuda") for a in (m, hot, mask)]
    out = {}
    solves = max(1, min(args.steps, 20))
    for scheme, iters in (("lusgs", args.synth_iters), ("explicit", 2000)):
        synth_solve(w, *dev, max_iter=20, tol=0.0, scheme=scheme)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(solves):
            synth_solve(w, *dev, max_iter=iters, tol=0.0, scheme=scheme)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / solves
        out[scheme] = {"iterations": iters, "ms_per_solve": round(ms, 3),
                       "us_per_iteration": round(1e3 * ms / iters, 2)}
        progress(f"synth {scheme}: {ms:.2f} ms per solve of {iters} iterations")
    return out, solves


def run_cylinder(args):
    """Mach 5 flow past a cylinder: 500 x 400 stretched polar cells, ~50M
    particles at the freestream density, freestream inflow and outflow every
    step, plain DSMC.  The gas starts at rest (as in the paper); `preroll`
    steps (graph replays, untimed) let the freestream cross the domain and the
    bow shock form before the autotuner, the breakdown and the timed window."""
    import torch

    import dig_workloads as wl
    from paper_2501_10965_amd.dsmc import DSMC

    w = wl.cylinder()
    # the bow shock and the inflow reservoir raise the count from the initial
    # 50M to about 81M by the end of the pre-roll
    sim = DSMC(w, cap_factor=2.2, group_particles=args.group_particles,
               group_cells=args.group_cells)
    if args.seq_max >= 0:
        sim.tuning(seq_max=args.seq_max)
    sim.init()
    progress(f"cylinder: {sim.counters()['n']} particles at rest; pre-roll {args.preroll} steps")
    graphs = not args.no_graphs
    sim.step(args.preroll, graph=graphs)
    tuning = None if args.no_autotune else sim.autotune(steps_per_trial=10)
    k0 = sim.counters()["step"]
    sim.step(max(args.warmup, 1), graph=graphs)
    sim.profile("on")
    sim.step(10)
    breakdown = sim.profile("read")
    sim.profile("off")
    torch.cuda.synchronize()
    steps = args.steps
    c0 = sim.counters()
    sim.profile("on", kinds=["collide"], every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile("read")
    sim.profile("off")
    c1 = sim.counters()
    n_avg = 0.5 * (c0["n"] + c1["n"])
    out = summarise(prof, breakdown, n_avg * steps, t1 - t0, steps, n_avg, sim.ncell, 2,
                    "cylinder")
    c2 = c1
    out["graph_replay"] = None
    if graphs:
        torch.cuda.synchronize()
        tg0 = time.perf_counter()
        sim.step(steps, graph=True)
        torch.cuda.synchronize()
        tg1 = time.perf_counter()
        c2 = sim.counters()
        ng = 0.5 * (c1["n"] + c2["n"])
        out["graph_replay"] = {"value": ng * steps / (tg1 - tg0), "unit": "particle-steps/s",
                               "steps": steps, "ms_per_step": (tg1 - tg0) / steps * 1e3}
    out.update(particles=int(n_avg), cells=sim.ncell, err_bits=c2["err"], tuning=tuning,
               dig_loop=None, timed_steps=[c0["step"], c1["step"]],
               inflow_per_step=(c1["injected"] - c0["injected"]) / steps,
               removed_per_step=(c1["removed"] - c0["removed"]) / steps,
               collisions_per_particle_step=(c1["accepted"] - c0["accepted"]) * 2 /
               max(n_avg * steps, 1),
               workload=f"{w['name']}: Mach 5 flow past a cylinder, Kn 0.01, 500x400 "
                        f"stretched polar cells, {n_avg / 1e6:.1f}M particles, freestream "
                        f"inflow/outflow every step, plain DSMC (move, sort, collide, sample); "
                        f"timed steps {c0['step']}-{c1['step']} of a start from rest "
                        f"(pre-roll {args.preroll} steps, then {k0 - args.preroll} autotuner "
                        f"steps: the freestream has crossed the domain, the bow shock "
                        f"stands)")
    return out, w


def run_sweep(args):
    """Cavity family at 1M to 100M particles (50 per cell): where the working
    set leaves the 256 MB last-level cache, the step becomes HBM-bound."""
    import math

    import torch

    import dig_workloads as wl
    from paper_2501_10965_amd.dsmc import DSMC

    rows = []
    for mp in args.sweep:
        n = int(round(math.sqrt(mp * 1e6 / 50)))
        w = wl.cavity_2d(seed=2001, n=n, ppc=50, kn=0.01 * 200 / n)
        sim = DSMC(w, cap_factor=1.05)
        sim.init()
        sim.step(20, graph=True)
        tuning = sim.autotune(steps_per_trial=5)
        sim.profile("on")
        sim.step(10)
        bd = sim.profile("read")
        sim.profile("off")
        torch.cuda.synchronize()
        c0 = sim.counters()
        t0 = time.perf_counter()
        sim.step(args.steps, graph=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        c1 = sim.counters()
        npart = 0.5 * (c0["n"] + c1["n"])
        state_mb = (2 * 28 + 16) * npart / 1e6 + (4 * 3 + 8 + 2 * 17 * 8) * n * n / 1e6
        us = {k: v[0] / max(v[1], 1) * 1e3 for k, v in bd.items() if v[1]}
        col = us["collide"] * 1e-6
        ach = (collide_particle_bytes(2) * npart + PER_CELL_BYTES * n * n) / col / 1e9
        row = {"particles": int(npart), "cells": n * n, "working_set_MB": round(state_mb, 1),
               "particle_steps_per_s": npart * args.steps / (t1 - t0),
               "ms_per_step": (t1 - t0) / args.steps * 1e3,
               "collide_us": round(us["collide"], 1), "move_us": round(us["move"], 1),
               "collide_GBs": round(ach, 1), "collide_frac": round(ach / HBM_PEAK_GBS, 4),
               "tuning": tuning}
        progress(f"sweep {mp}M: {json.dumps(row)}")
        rows.append(row)
        del sim
        torch.cuda.empty_cache()
    return rows


def run_steady(args):
    """Time to steady state at a fixed centreline-velocity error on the
    cavity: plain DSMC, DIG with DSMC-extracted terms, DIG with the learned
    closure (trained here on the cavity family; its training time is reported
    separately), all on the same GPU; optionally also DIG with the explicit
    synthetic solve."""
    import math

    import torch

    import dig_workloads as wl
    from paper_2501_10965_amd import learn, steady
    from paper_2501_10965_amd.mlp import MLP

    from paper_2501_10965_amd.dsmc import DSMC

    w = wl.cavity_2d(seed=2001, ppc=args.steady_ppc)
    P, W, thr, cols = 20, args.steady_window, args.steady_threshold, args.steady_columns
    # one launch configuration for every arm, found once on a separate copy of
    # the workload (untimed; the results do not depend on it)
    tun = None
    if not args.no_autotune:
        progress("autotune")
        probe = DSMC(w)
        probe.init()
        tun = probe.autotune(10)
        del probe
        progress(f"tuning {tun}")
    progress("reference run")
    ref = steady.reference_profile(w, args.steady_ref_steps[0], args.steady_ref_steps[1], P, cols,
                                   tuning=tun, progress=progress)
    arms = {}
    progress("plain DSMC arm")
    tr = steady.run_plain(w, ref, w["ns"], args.dig_max_cycles * 4, W, thr, P, cols, tuning=tun)
    arms["dsmc"] = tr
    # DIG cycles of N_s steps; the sliding window covers the same number of
    # DSMC steps as the plain arm's
    ns = args.steady_dig_ns or w["ns"]
    Wd = max(1, W * w["ns"] // ns)
    dig_kw = dict(ns=ns, n_m=args.synth_iters, wall_mode=args.steady_wall_mode,
                  scheme=args.synth_scheme, columns=cols, handoff=args.steady_handoff or None,
                  tuning=tun)
    runs = {}
    progress(f"DIG arm (DSMC-extracted terms, {args.synth_scheme} synthetic solve, N_s {ns})")
    tr, runs["dig"] = steady.run_dig(w, ref, args.dig_max_cycles, Wd, thr, P, **dig_kw)
    arms["dig"] = tr
    if args.steady_explicit_arm:
        progress("DIG arm (explicit synthetic solve, 2000 iterations)")
        tr, _ = steady.run_dig(w, ref, args.dig_max_cycles, W, thr, P, ns=w["ns"], n_m=2000,
                               wall_mode="wall", scheme="explicit", columns=cols, tuning=tun)
        arms["dig_explicit"] = tr
    if args.steady_graded_arm:
        # the paper's DIG grid for this Kn (Section 4.1, Table 1): 100 x 100 cells refined
        # toward the walls (first cell 0.001), a larger time step, slip and jump from DSMC
        g = wl.cavity_graded(seed=2101, n=100, first=0.001, ppc=50, kn=w["kn"],
                             lid=w["bc"][3][2][0], dt_frac=0.5)
        progress("DIG arm on the wall-refined 100 x 100 grid")
        tr, _ = steady.run_dig(g, ref, args.dig_max_cycles, W, thr, P, ns=w["ns"],
                               n_m=args.synth_iters, wall_mode="dsmc", scheme=args.synth_scheme,
                               columns=2)
        arms["dig_graded_100"] = tr
    progress("closure-network training")
    KNS = [0.005, 0.01, 0.02, 0.05, 0.1, 0.2, 0.5]
    MAS = [0.1, 0.25, 0.5, 1.0]
    ws = [wl.cavity_2d(seed=4000 + i, n=100, ppc=50, kn=k, lid=m * math.sqrt(1.4))
          for i, (k, m) in enumerate((k, m) for k in KNS for m in MAS)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    from paper_2501_10965_amd.dsmc import DSMC
    batch = DSMC(ws, cap_factor=1.05)
    batch.init_batch()
    batch.step(2000, graph=True)
    x, t, _ = learn.collect(batch, windows=6, window_steps=1000)
    del batch
    sc = learn.fit_scaling(x, t)
    xs, ts = learn.standardise(x, t, sc)
    net = MLP(wl.mlp_init(7), max_batch=4096)
    learn.train(net, xs, ts, steps=3000, batch=4096, lr=2e-3, lr_final=1e-4)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    progress("DIG arm (learned closure)")
    hook = learn.LearnedClosure(net, sc, kn_lo=0.01, judge_sigma=3.0, judge_rel=0.1,
                                avg_steps=ns)
    tr, d = steady.run_dig(w, ref, args.dig_max_cycles, Wd, thr, P, closure=hook, **dig_kw)
    runs["dig_learned"] = d
    arms["dig_learned"] = tr
    res = {}
    for name, tr in arms.items():
        t = tr.time_to_steady()
        res[name] = {"seconds": None if t is None else round(t[0], 3),
                     "steps": None if t is None else t[1],
                     "final_err": round(tr.history[-1][2], 5) if tr.history else None,
                     "min_err": round(min(e[2] for e in tr.history), 5) if tr.history else None,
                     "seconds_to": {str(x): (None if tr.time_to_steady(x) is None
                                             else round(tr.time_to_steady(x)[0], 3))
                                    for x in (0.05, 0.03, 0.02, 0.01)},
                     # the same with the largest pointwise error of the profile
                     "final_err_max": round(tr.history[-1][3], 5) if tr.history else None,
                     "min_err_max": round(min(e[3] for e in tr.history), 5) if tr.history else None,
                     "seconds_to_max": {str(x): (None if tr.time_to_steady(x, "max") is None
                                                 else round(tr.time_to_steady(x, "max")[0], 3))
                                        for x in (0.05, 0.03, 0.02, 0.01)},
                     "err_at": [(round(e[0], 3), e[1], round(e[2], 5), round(e[3], 5))
                                for e in tr.history[::10]]}
    res["dig_learned"]["training_seconds"] = round(train_s, 2)
    for name, d in runs.items():
        ch = [r["cycle_change"] for r in d.log if "cycle_change" in r]
        res[name]["handoff_cycle"] = d.handoff_at
        res[name]["cycle_change"] = [round(c, 5) for c in ch[::5]]
    src = hook.last_src
    if src is not None:
        res["dig_learned"]["last_cycle_sources"] = {
            k: int((src == v).sum()) for k, v in (("nsf", 0), ("dsmc", 1), ("network", 2),
                                                  ("rejected", 3))}
    base = res["dsmc"]["seconds"]
    res["tuning"] = tun
    return res, base


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, usable


def _oracle_sample(w, steps, dig):
    """The oracle on one core: (particle-steps, seconds, final particle count)."""
    import oracle

    s = oracle.new_state(w)
    t0 = time.perf_counter()
    ps = 0
    A = default_A(w["omega"])
    it = 0
    ns = w.get("ns", 50)
    for done in range(1, steps + 1):
        ps += s.n
        s.step()
        if dig and done % ns == 0:
            f = s.fields()
            oracle.closure(w, f, A, 0.01)
            s.adjust(f[0:6].copy(), it)
            s.reset_average()
            it += 1
    return ps, time.perf_counter() - t0, s.n


def _oracle_worker(job):
    w, steps, dig = job
    return _oracle_sample(w, steps, dig)


def cpu_baseline(w, steps, dig: bool, par_steps=None):
    """The FP64 oracle (single-threaded C) on the host: one copy alone, then one
    copy per usable core (capped at 16, the host share of one GPU), each on
    its own seed, run at once; the all-core rate is the sum of their rates."""
    import multiprocessing as mp

    model, usable = host_cpu()
    progress(f"oracle baseline on {w['name']}, {steps} steps, one core")
    ps1, sec1, n1 = _oracle_sample(w, steps, dig)
    procs = max(1, min(usable, 16))
    par_steps = par_steps or steps
    jobs = [(dict(w, seed=w["seed"] + 7919 * (k + 1)), par_steps, dig) for k in range(procs)]
    progress(f"oracle baseline, {procs} processes at once, {par_steps} steps each")
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    agg = sum(ps / sec for ps, sec, _ in res)
    what = (f"{steps} DSMC steps with {steps // w.get('ns', 50)} DIG cycles (closure + "
            f"modification)" if dig else f"{steps} DSMC steps")
    return {"value": agg, "unit": "particle-steps/s", "cores": procs, "kind": "oracle",
            "sample": f"{w['name']}: {n1} particles, {what}, FP64; {procs} independent copies "
                      f"(seeds differ) of {par_steps} steps each, one per core, run at once; "
                      f"value = sum of their rates",
            "per_core_value": ps1 / sec1, "per_core_seconds": round(sec1, 2),
            "all_core_wall_seconds": round(wall, 2), "host_cpu_model": model,
            "host_usable_cores": usable, "host_nproc": os.cpu_count()}


def copy_calibration():
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch

    nbytes = 1 << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "dispatches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=150)
    ap.add_argument("--workload",
                    choices=["cylinder", "cavity", "batch", "mlp", "steady", "sweep", "synth"],
                    default="cylinder")
    ap.add_argument("--preroll", type=int, default=2000,
                    help="cylinder: untimed steps from the start at rest before the window")
    ap.add_argument("--sweep", type=float, nargs="+", default=[1, 2, 5, 10, 20, 50, 100],
                    help="sweep: particle counts in millions")
    ap.add_argument("--steady-threshold", type=float, default=0.01)
    ap.add_argument("--steady-window", type=int, default=40,
                    help="steady: cycles in the sliding average of the observable")
    ap.add_argument("--steady-columns", type=int, default=8,
                    help="steady: centre columns averaged into the centreline profile")
    ap.add_argument("--steady-explicit-arm", action="store_true")
    ap.add_argument("--steady-graded-arm", action="store_true",
                    help="steady: also DIG on the wall-refined 100 x 100 grid")
    ap.add_argument("--synth-scheme", choices=["explicit", "lusgs"], default="lusgs")
    ap.add_argument("--steady-wall-mode", choices=["wall", "dsmc"], default="wall",
                    help="steady: wall faces of the DIG arms' synthetic solve: the walls' "
                         "values, or the DSMC slip and jump of the wall-adjacent cells")
    ap.add_argument("--steady-handoff", type=float, default=0.95,
                    help="steady: DIG arms continue as plain DSMC once the mean change of "
                         "the macroscopic solution between cycles over 10 cycles exceeds this "
                         "fraction of the mean over the 10 before (it has levelled off; 0: never)")
    ap.add_argument("--steady-ppc", type=int, default=50,
                    help="steady: particles per cell of the cavity")
    ap.add_argument("--steady-ref-steps", type=int, nargs=2, default=[60000, 120000],
                    help="steady: transient and averaged steps of the reference run")
    ap.add_argument("--steady-dig-ns", type=int, default=0,
                    help="steady: DSMC steps per DIG cycle (N_s) of the DIG arms "
                         "(0: the workload's 50)")
    ap.add_argument("--dig-max-cycles", type=int, default=400)
    ap.add_argument("--cpu-steps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--dig-cycles", type=int, default=2)
    ap.add_argument("--synth-iters", type=int, default=400,
                    help="synthetic-solve iterations per DIG cycle (N_m)")
    ap.add_argument("--group-particles", type=int, default=0)
    ap.add_argument("--group-cells", type=int, default=0)
    ap.add_argument("--seq-max", type=int, default=-1,
                    help="cells up to this size run their candidates on one lane "
                         "(with --no-autotune; -1 keeps the library default)")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-graphs", action="store_true",
                    help="cylinder: every step launched eagerly (for counter collection)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU only (the DSMC domain decomposition "
              "across GPUs is a design, not an implementation); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    progress(f"workload {args.workload}")
    if args.workload == "steady":
        res, base = run_steady(args)
        tun = res.pop("tuning")
        learned = res["dig_learned"]["seconds"]
        line = {"metric": "time-to-steady-state at fixed error, learned vs plain",
                "value": learned, "unit": "s", "n_gpus": 1, "steps": None,
                "warmup": 0, "ms_per_step": None, "higher_is_better": False,
                "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                "config": {"workload": f"cavity 200x200, {args.steady_ppc} particles per cell "
                           f"({args.steady_ppc * 40000 / 1e6:g}M), Kn 0.01, lid Ma 0.3; "
                           f"centreline u_x ({args.steady_columns} centre columns, 20 block "
                           f"averages), window {args.steady_window} cycles of 50 steps, "
                           f"RMS error <= {args.steady_threshold} of the reference range "
                           "(the largest pointwise error reported beside it); "
                           f"reference {args.steady_ref_steps[0]} + {args.steady_ref_steps[1]} "
                           "plain-DSMC steps; DIG synthetic solve "
                           f"{args.synth_scheme}, N_m = {args.synth_iters}, N_s = "
                           f"{args.steady_dig_ns or 50}"
                           + (f", DIG hands off to plain DSMC once its cycle-to-cycle change "
                              f"levels off (ratio {args.steady_handoff} over 10-cycle means)"
                              if args.steady_handoff else ""),
                           "tuning": tun},
                "plain_dsmc_seconds": base, "arms": res}
        print(json.dumps(line), flush=True)
        return
    if args.workload == "mlp":
        res = run_mlp(args)
        line = {"metric": res["metric"], "value": res["value"], "unit": res["unit"],
                "n_gpus": 1, "steps": res["steps"], "warmup": args.warmup,
                "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
                "config": {"workload": "closure network 9-128-128-128-7, training batch "
                           "65536, inference over 2^20 samples"},
                "roofline": res["roofline"], "cpu_baseline": None,
                "training_tflops": res["training_tflops"],
                "training_frac": res["training_frac"],
                "inference_samples_per_s": res["inference_samples_per_s"]}
        print(json.dumps(line), flush=True)
        return
    if args.workload == "synth":
        res, solves = run_synth(args)
        lu = res["lusgs"]
        print(json.dumps({"metric": "synthetic-solve iterations/s (200x200 cavity grid, LU-SGS)",
                          "value": 1e6 / lu["us_per_iteration"], "unit": "iterations/s",
                          "n_gpus": 1, "steps": solves, "warmup": 1,
                          "ms_per_step": lu["ms_per_solve"], "higher_is_better": True,
                          "dtype": "f64", "data": "synthetic",
                          "config": {"workload": "synthetic equations on the 200x200 cavity "
                                     "grid, Kn 0.01, fixed iteration counts per solve"},
                          "schemes": res}), flush=True)
        return
    if args.workload == "sweep":
        rows = run_sweep(args)
        print(json.dumps({"metric": "DSMC particle-steps/s vs particle count (cavity, 50 "
                                    "particles per cell)", "unit": "particle-steps/s",
                          "steps": args.steps, "rows": rows}), flush=True)
        return
    if args.workload == "batch":
        res, wcpu = run_batch(args)
        cpu = None if args.no_cpu_baseline else cpu_baseline(wcpu, 300, dig=False)
    elif args.workload == "cylinder":
        res, wcpu = run_cylinder(args)
        # bounded sample: the same geometry and flow with 4M particles, from rest
        import dig_workloads as wl
        wsmall = wl.cylinder(n_target=4_000_000)
        cpu = None if args.no_cpu_baseline else cpu_baseline(wsmall, 40, dig=False,
                                                             par_steps=20)
    else:
        res, wcpu = run_cavity(args)
        cpu = None if args.no_cpu_baseline else cpu_baseline(wcpu, args.cpu_steps, dig=True)
    line = {
        "metric": METRIC, "value": res["value"], "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": res["workload"], "particles": res["particles"],
                   "cells": res["cells"], "parallelism": "single GPU",
                   "tuning": res["tuning"]},
        "roofline": res["roofline"], "cpu_baseline": cpu,
        "step_roofline": res["step_roofline"], "kernels_us": res["kernels_us"],
        "kernel_launches": res["kernel_launches"], "err_bits": res["err_bits"],
        "collisions_per_particle_step": res["collisions_per_particle_step"],
        "graph_replay": res["graph_replay"], "dig_loop": res["dig_loop"],
        "kernel_source_digest": source_digest(),
    }
    for k in ("timed_steps", "inflow_per_step", "removed_per_step", "dig_cycles_timed"):
        if k in res:
            line[k] = res[k]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
