"""synth_solve_static (the synthetic-equation solve for callers that cannot
allocate device memory) through the C ABI, against synth_solve with a
caller workspace: two calls in a row on one GPU, the second on a smaller
grid (the static scratch keeps the first call's contents), must give the
same solution, iteration count and last change, bit for bit; a grid whose
scratch exceeds the static array is rejected."""
import ctypes as C

import numpy as np
import pytest
import torch

import dig_workloads as wl
from paper_2501_10965_amd import _lib as L
from paper_2501_10965_amd.dsmc import _ptr, _stream, synth_solve

pytestmark = pytest.mark.gpu


def _case(n, seed):
    w = wl.cavity_2d(seed=seed, n=n, kn=0.05)
    rng = np.random.default_rng(seed)
    nc = n * n
    m = np.zeros((20, nc))
    m[0] = 1.0 + 0.05 * rng.standard_normal(nc)
    m[1:4] = 0.05 * rng.standard_normal((3, nc))
    m[4] = 1.0 + 0.03 * rng.standard_normal(nc)
    m[5] = 1.0 + 0.03 * rng.standard_normal(nc)
    hot = 0.005 * rng.standard_normal((12, nc))
    mask = (rng.random(nc) < 0.4).astype(np.uint8)
    dev = torch.device("cuda")
    return (w, torch.tensor(m, device=dev), torch.tensor(hot, device=dev),
            torch.tensor(mask, device=dev))


def _opts(w, cfl=0.5, wall_mode=1, check_every=32):
    o = L.DigSynthOpts()
    om = w["omega"]
    for k, v in enumerate((2.0 / 3.0, 0.0, 0.0, 5.0 / (7.0 - 2.0 * om))):
        o.A[k] = v
    o.cfl = cfl
    o.wall_mode = wall_mode
    o.check_every = check_every
    return o


def static_solve(w, m, hot, mask, max_iter, tol):
    lib = L.load()
    cfg = L.make_config(w)
    out = torch.empty((6, w["nx"] * w["ny"]), dtype=torch.float64, device=m.device)
    it, ch = C.c_int32(0), C.c_double(0.0)
    rc = lib.synth_solve_static(C.byref(cfg), C.byref(_opts(w)), _ptr(m), _ptr(hot), _ptr(mask),
                                _ptr(out), int(max_iter), float(tol), C.byref(it),
                                C.byref(ch), _stream())
    return rc, out, it.value, ch.value


@pytest.mark.parametrize("order", ["large_then_small"])
def test_static_scratch_solve_equals_workspace_solve(order):
    for n, seed, iters, tol in ((96, 3, 300, 0.0), (40, 4, 5000, 1e-6)):
        w, m, hot, mask = _case(n, seed)
        print(f"case synth_solve_static {n}x{n} max_iter {iters}", flush=True)
        rc, out_s, it_s, ch_s = static_solve(w, m, hot, mask, iters, tol)
        assert rc == L.DIG_OK, L.load().dig_last_error()
        out_w, it_w, ch_w = synth_solve(w, m, hot, mask, wall_mode="dsmc", max_iter=iters,
                                        tol=tol, check_every=32)
        torch.cuda.synchronize()
        assert it_s == it_w and ch_s == ch_w
        assert torch.equal(out_s, out_w), (out_s - out_w).abs().max().item()
        assert torch.isfinite(out_s).all()


def test_grid_beyond_the_static_scratch_is_rejected():
    lib = L.load()
    w = wl.cavity_2d(seed=1, n=400, kn=0.05)
    cfg = L.make_config(w)
    assert lib.dig_synth_workspace_bytes(C.byref(cfg)) > L.SYNTH_STATIC_BYTES
    dev = torch.device("cuda")
    m = torch.zeros((20, 4), dtype=torch.float64, device=dev)
    out = torch.zeros((6, 4), dtype=torch.float64, device=dev)
    it, ch = C.c_int32(0), C.c_double(0.0)
    rc = lib.synth_solve_static(C.byref(cfg), C.byref(_opts(w)), _ptr(m), None, None, _ptr(out),
                                10, 0.0, C.byref(it), C.byref(ch), _stream())
    assert rc == L.DIG_ERR_INVALID
    assert b"static" in lib.dig_last_error()
    assert torch.count_nonzero(out) == 0
