"""Helpers shared by the GPU parity tests: move states between the HIP library
(through its C ABI) and the oracle, and compare them."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from paper_2501_10965_amd import _lib as L
from paper_2501_10965_amd.dsmc import DSMC


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def np_(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def gpu_state(sim: DSMC, n: int | None = None) -> dict:
    st = sim.state(n)
    out = {k: np_(v).copy() for k, v in st.items()}
    out["id"] = out["id"].view(np.uint32)
    return out


def gpu_buffer(sim: DSMC, b: int, n: int) -> dict:
    st = sim.buffer(b, n)
    out = {k: np_(v).copy() for k, v in st.items()}
    out["id"] = out["id"].view(np.uint32)
    return out


def oracle_state(w, arrays, start, sgmax, step, cap=None, next_id=None):
    n = len(arrays["x"])
    s = oracle.State(w, cap or max(n, 1) * 2 + 64)
    # a 1D state has no y: the GPU buffer holds whatever was there before
    y = arrays["y"] if w["dim"] == 2 else np.zeros(n, np.float32)
    s.load(arrays["x"], y, arrays["vx"], arrays["vy"], arrays["vz"], arrays["er"],
           arrays["id"], start=start, sgmax=sgmax, step=step, next_id=next_id)
    return s


def rel_close(a, b, rel, floor=1.0):
    """|a - b| <= rel * max(|b|, floor), elementwise."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) <= rel * np.maximum(np.abs(b), floor)


def cells_of(start: np.ndarray) -> np.ndarray:
    counts = np.diff(start)
    return np.repeat(np.arange(len(counts)), counts)


def sorted_arrays(arrays: dict, perm: np.ndarray) -> dict:
    return {k: v[perm] for k, v in arrays.items()}


STAGES = dict(move=L.STAGE_MOVE, sort=L.STAGE_SORT, collide=L.STAGE_COLLIDE)
