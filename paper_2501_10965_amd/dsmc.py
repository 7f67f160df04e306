"""Python face of libdig: device memory and streams from PyTorch, every step of
the method in the library's HIP kernels.

    sim = DSMC(workload)            # or a list of workloads (batched instances)
    sim.init()                      # equilibrium start from the workload's fields
    sim.step(50)                    # DSMC steps, time averaging on
    f = sim.sample("average")       # [20, C] float64 fields on the device
    sim.adjust(target, dig_iter)    # DIG particle modification toward target [6, C]
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

FIELD_NAMES = ["rho", "ux", "uy", "uz", "Tt", "Tr", "sxx", "syy", "szz", "sxy", "sxz", "syz",
               "qtx", "qty", "qtz", "qrx", "qry", "qrz", "T", "N"]
HOT_NAMES = ["sxx", "syy", "szz", "sxy", "sxz", "syz", "qtx", "qty", "qtz", "qrx", "qry", "qrz"]


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    assert t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


class DSMC:
    """A context of one or more simulation instances on one GPU."""

    def __init__(self, workloads, capacity: int | None = None, cap_factor: float = 1.3,
                 group_particles: int = 0, group_cells: int = 0, device="cuda"):
        self.lib = L.load()
        self.workloads = list(workloads) if isinstance(workloads, (list, tuple)) else [workloads]
        self.n_inst = len(self.workloads)
        # the configuration objects own the face tables the array points to
        self._cfg_objs = [L.make_config(w) for w in self.workloads]
        self.cfgs = (L.DigConfig * self.n_inst)(*self._cfg_objs)
        self.ncells = [w["nx"] * w.get("ny", 1) for w in self.workloads]
        self.ncell = int(sum(self.ncells))
        self.cell0 = np.concatenate([[0], np.cumsum(self.ncells)]).astype(np.int64)
        if capacity is None:
            est = sum(nc * w.get("ppc", 1) if w.get("ppc", 1) > 0 else w["n_target"]
                      for nc, w in zip(self.ncells, self.workloads))
            capacity = int(est * cap_factor) + 1024
        self.capacity = int(capacity)
        self.layout = L.DigLayout()
        L.check(self.lib.dig_plan(self.cfgs, self.n_inst, self.capacity, C.byref(self.layout)))
        self.device = torch.device(device)
        self.ws = torch.empty(self.layout.total_bytes, dtype=torch.uint8, device=self.device)
        self.ctx = C.c_void_p()
        L.check(self.lib.dsmc_create(self.cfgs, self.n_inst, self.capacity, _ptr(self.ws),
                                     self.layout.total_bytes, int(group_particles),
                                     int(group_cells), _stream(), C.byref(self.ctx)))

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.lib.dsmc_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # -- workspace views ----------------------------------------------------
    def _view(self, off: int, count: int, dtype) -> torch.Tensor:
        item = torch.empty((), dtype=dtype).element_size()
        return self.ws[off: off + count * item].view(dtype)

    def counters(self) -> dict:
        c = L.DigCounters()
        L.check(self.lib.dsmc_query(self.ctx, C.byref(c), _stream()))
        return c.as_dict()

    def save(self) -> bytes:
        """Checkpoint image of the current state (dsmc_save)."""
        need = C.c_size_t(0)
        L.check(self.lib.dsmc_save(self.ctx, None, C.byref(need), _stream()))
        buf = C.create_string_buffer(need.value)
        L.check(self.lib.dsmc_save(self.ctx, buf, C.byref(need), _stream()))
        return buf.raw[: need.value]

    def load(self, image: bytes):
        """Replaces the state by a checkpoint image (dsmc_load)."""
        L.check(self.lib.dsmc_load(self.ctx, image, len(image), _stream()))

    def state(self, n: int | None = None) -> dict:
        """Views of the current (cell-sorted) particle buffer."""
        ctr = self.counters()
        b = ctr["cur"]
        n = ctr["n"] if n is None else n
        Lo = self.layout
        out = {k: self._view(getattr(Lo, k)[b], n, torch.float32)
               for k in ("x", "y", "vx", "vy", "vz", "er")}
        out["id"] = self._view(Lo.id[b], n, torch.int32)
        return out

    def buffer(self, b: int, n: int) -> dict:
        Lo = self.layout
        out = {k: self._view(getattr(Lo, k)[b], n, torch.float32)
               for k in ("x", "y", "vx", "vy", "vz", "er")}
        out["id"] = self._view(Lo.id[b], n, torch.int32)
        return out

    def array(self, name: str) -> torch.Tensor:
        Lo = self.layout
        cap, nc = self.capacity, self.ncell
        spec = {"cell": (cap, torch.int32), "rank": (cap, torch.int32),
                "perm_raw": (cap, torch.int32), "perm": (cap, torch.int32),
                "start": (nc + 1, torch.int32), "count": (nc, torch.int32),
                "sgmax": (nc, torch.float32), "acc": (nc * 17, torch.float64),
                "sums": (nc * 17, torch.float64), "cell_inst": (nc, torch.int32)}
        n, dt = spec[name]
        return self._view(getattr(Lo, name), n, dt)

    # -- the method -----------------------------------------------------------
    def uniform_fields(self) -> torch.Tensor:
        f = np.zeros((6, self.ncell))
        for i, w in enumerate(self.workloads):
            s = slice(self.cell0[i], self.cell0[i + 1])
            ini = w["init"]
            f[0, s] = ini["rho"]
            f[1, s], f[2, s], f[3, s] = ini["u"]
            f[4, s] = ini["Tt"]
            f[5, s] = ini["Tr"]
        return torch.tensor(f, dtype=torch.float64, device=self.device)

    def init(self, fields: torch.Tensor | None = None, ppc: int | None = None):
        if fields is None:
            fields = self.uniform_fields()
        if ppc is None:
            ppcs = {w.get("ppc", 0) for w in self.workloads}
            ppc = ppcs.pop() if len(ppcs) == 1 else 0
            if ppc == 0 and len(self.workloads) > 1:
                raise ValueError("instances differ in ppc: pass counts through fields (ppc=0)")
        self._fields_keep = fields.contiguous()
        L.check(self.lib.dsmc_init(self.ctx, _ptr(self._fields_keep), int(ppc), _stream()))

    def init_batch(self):
        """Batched start: exactly ppc_i particles per cell of instance i, via the
        Iround count rule with rho chosen so that rho V / N_eff = ppc_i."""
        f = self.uniform_fields()
        for i, w in enumerate(self.workloads):
            s = slice(self.cell0[i], self.cell0[i + 1])
            vol = (w["lx"] / w["nx"]) * ((w["ly"] / w["ny"]) if w["dim"] == 2 else 1.0)
            f[0, s] = w["ppc"] * w["weight"] / vol
        self.init(f, ppc=0)

    def inject(self, arrays: dict, start, step: int = 0, next_id: int | None = None,
               sgmax=None):
        """Write a cell-sorted state into the current buffer and adopt it."""
        n = len(arrays["x"])
        b = self.counters()["cur"]
        views = self.buffer(b, n)
        for k in ("x", "y", "vx", "vy", "vz", "er"):
            views[k].copy_(torch.as_tensor(np.asarray(arrays[k], dtype=np.float32)))
        views["id"].copy_(torch.as_tensor(np.asarray(arrays["id"]).astype(np.uint32)
                                          .view(np.int32)))
        self.array("start").copy_(torch.as_tensor(np.asarray(start, dtype=np.int32)))
        if sgmax is not None:
            self.array("sgmax").copy_(torch.as_tensor(np.asarray(sgmax, dtype=np.float32)))
        torch.cuda.current_stream().synchronize()
        nid = n if next_id is None else next_id
        L.check(self.lib.dsmc_inject(self.ctx, n, int(step), int(nid), _stream()))

    def step(self, nsteps: int = 1, graph: bool = False):
        """nsteps DSMC steps; graph=True launches them as one captured HIP graph."""
        fn = self.lib.dsmc_step_graph if graph else self.lib.dsmc_step
        L.check(fn(self.ctx, int(nsteps), _stream()))

    def tuning(self, group_particles=None, group_cells=None, seq_max=None,
               big_stage_kib=None) -> dict:
        """Current launch configuration; arguments given replace its fields."""
        cur = L.DigTuning()
        L.check(self.lib.dsmc_tuning(self.ctx, None, C.byref(cur)))
        if group_particles is None and group_cells is None and seq_max is None and \
                big_stage_kib is None:
            return cur.as_dict()
        new = L.DigTuning(group_particles or cur.group_particles, group_cells or cur.group_cells,
                          cur.seq_max if seq_max is None else seq_max,
                          big_stage_kib or cur.big_stage_kib, 0.0)
        L.check(self.lib.dsmc_tuning(self.ctx, C.byref(new), None))
        return new.as_dict()

    def autotune(self, steps_per_trial: int = 10, cache_path: str | None = None) -> dict:
        """Coordinate search over the launch configuration (advances the state)."""
        out = L.DigTuning()
        path = cache_path.encode() if cache_path else None
        L.check(self.lib.dsmc_autotune(self.ctx, int(steps_per_trial), path, C.byref(out),
                                       _stream()))
        return out.as_dict()

    def stage(self, mask: int):
        L.check(self.lib.dsmc_stage(self.ctx, int(mask), _stream()))

    def sample(self, mode: str = "average", out: torch.Tensor | None = None) -> torch.Tensor:
        m = {"instant": L.SAMPLE_INSTANT, "average": L.SAMPLE_AVERAGE, "reset": L.SAMPLE_RESET}[mode]
        if m == L.SAMPLE_RESET:
            L.check(self.lib.dsmc_sample(self.ctx, m, None, _stream()))
            return None
        if out is None:
            out = torch.empty((20, self.ncell), dtype=torch.float64, device=self.device)
        L.check(self.lib.dsmc_sample(self.ctx, m, _ptr(out), _stream()))
        return out

    def reset_average(self):
        self.sample("reset")

    def adjust(self, target: torch.Tensor, dig_iter: int):
        t = target.to(device=self.device, dtype=torch.float64).contiguous()
        L.check(self.lib.dig_adjust(self.ctx, _ptr(t), int(dig_iter), _stream()))

    def closure(self, fields: torch.Tensor, A, kn_ref: float, with_nsf: bool = False,
                n_min: float = 0.0):
        """closure_assemble: (hot, mask, kn_gll, nsf or None); cells with a mean
        particle count below n_min are treated as in equilibrium."""
        nc = self.ncell
        f = fields.contiguous()
        hot = torch.empty((12, nc), dtype=torch.float64, device=self.device)
        mask = torch.empty(nc, dtype=torch.uint8, device=self.device)
        kn = torch.empty(nc, dtype=torch.float64, device=self.device)
        nsf = torch.empty((12, nc), dtype=torch.float64, device=self.device) if with_nsf else None
        a = (C.c_double * 4)(*[float(v) for v in A])
        L.check(self.lib.closure_assemble(self.ctx, _ptr(f), a, float(kn_ref), float(n_min),
                                          _ptr(hot),
                                          _ptr(mask), _ptr(kn),
                                          _ptr(nsf) if nsf is not None else None, _stream()))
        return hot, mask, kn, nsf

    def fill_empty(self, fields: torch.Tensor, fallback: torch.Tensor):
        """fields_fill_empty: cells of the time average [20, C] (in place)
        without a usable sample take the fallback state [>=6, C]."""
        assert fields.is_contiguous() and fields.dtype == torch.float64
        fb = fallback[0:6].contiguous()
        L.check(self.lib.fields_fill_empty(self.ctx, _ptr(fields), _ptr(fb), _stream()))
        return fields

    def features(self, fields: torch.Tensor, kngll: torch.Tensor, scaling: dict,
                 hot: torch.Tensor | None = None):
        """Standardised network inputs [C, 9] (and targets [C, 7] from hot)."""
        nc = self.ncell
        x = torch.empty((nc, 9), dtype=torch.float32, device=self.device)
        t = torch.empty((nc, 7), dtype=torch.float32, device=self.device) if hot is not None \
            else None
        sc = L.DigMlpScaling.of(scaling)
        L.check(self.lib.closure_features(
            self.ctx, _ptr(fields.contiguous()), _ptr(kngll.contiguous()),
            _ptr(hot.contiguous()) if hot is not None else None, C.byref(sc), _ptr(x),
            _ptr(t) if t is not None else None, _stream()))
        return x, t

    def blend(self, fields, kngll, mask, y, scaling: dict, hot: torch.Tensor, kn_lo: float,
              kn_hi: float, judge_sigma: float, judge_rel: float, judge_steps: float, A=None):
        """Three-band closure in place on hot; returns the per-cell source code.
        judge_steps: independent samples per particle in the averaged fields."""
        src = torch.empty(self.ncell, dtype=torch.uint8, device=self.device)
        sc = L.DigMlpScaling.of(scaling)
        om = self.workloads[0]["omega"]
        A = A if A is not None else (2.0 / 3.0, 0.0, 0.0, 5.0 / (7.0 - 2.0 * om))
        a = (C.c_double * 4)(*[float(v) for v in A])
        L.check(self.lib.closure_blend(
            self.ctx, _ptr(fields.contiguous()), _ptr(kngll.contiguous()), _ptr(mask.contiguous()),
            _ptr(y.contiguous()), C.byref(sc), a, float(kn_lo), float(kn_hi), float(judge_sigma),
            float(judge_rel), float(judge_steps), _ptr(hot), _ptr(src), _stream()))
        return src

    def profile(self, mode: str, kinds=None, every: int = 1):
        """'on' (reset and enable), 'off', or 'read' -> {kernel: (ms_total, launches)}.
        kinds (with 'on'): the kernel kinds to time, default all; every: time
        one launch of each in every `every`."""
        m = {"off": 0, "on": 1, "read": 2}[mode]
        if m == 1:
            mask = (1 << len(L.KERNELS)) - 1 if kinds is None else \
                sum(1 << L.KERNELS.index(k) for k in kinds)
            L.check(self.lib.dsmc_profile_kinds(self.ctx, mask, int(every)))
        ms = (C.c_double * len(L.KERNELS))()
        nl = (C.c_int64 * len(L.KERNELS))()
        L.check(self.lib.dsmc_profile(self.ctx, m, ms, nl, _stream()))
        if m == 2:
            return {k: (ms[i], nl[i]) for i, k in enumerate(L.KERNELS)}
        return None

    def constants(self, inst: int = 0) -> dict:
        out = (C.c_double * 5)()
        L.check(self.lib.dig_constants(self.ctx, inst, out))
        return dict(csigma=out[0], pinelastic=out[1], mu0=out[2], volume=out[3],
                    sgmax_default=out[4])


def synth_solve(w: dict, m_half: torch.Tensor, hot: torch.Tensor | None = None,
                mask: torch.Tensor | None = None, A=None, cfl: float | None = None,
                wall_mode: str = "dsmc", max_iter: int = 2000, tol: float = 1e-5,
                check_every: int = 128, scheme: str = "explicit"):
    """Synthetic-equation solve on the GPU; returns (m_next [6, C], iterations,
    last relative change).  scheme "explicit" (cfl default 0.5) or "lusgs"
    (implicit, cfl default 1e6).  The change is checked every check_every
    iterations (each check synchronises the host)."""
    if cfl is None:
        cfl = 0.5 if scheme == "explicit" else 1e6
    lib = L.load()
    cfg = L.make_config(w)
    nc = w["nx"] * w.get("ny", 1)
    dev = m_half.device
    ws = torch.empty(int(lib.dig_synth_workspace_bytes(C.byref(cfg))), dtype=torch.uint8,
                     device=dev)
    opts = L.DigSynthOpts()
    om = w["omega"]
    A = A if A is not None else (2.0 / 3.0, 0.0, 0.0, 5.0 / (7.0 - 2.0 * om))
    for k in range(4):
        opts.A[k] = float(A[k])
    opts.cfl = float(cfl)
    opts.wall_mode = {"wall": 0, "dsmc": 1}[wall_mode]
    opts.check_every = int(check_every)
    opts.scheme = L.SYNTH_SCHEMES[scheme]
    m = m_half.contiguous()
    out = torch.empty((6, nc), dtype=torch.float64, device=dev)
    h = hot.contiguous() if hot is not None else None
    mk = mask.contiguous() if mask is not None else None
    it = C.c_int32(0)
    ch = C.c_double(0.0)
    L.check(lib.synth_solve(C.byref(cfg), C.byref(opts), _ptr(m), _ptr(h) if h is not None else None,
                            _ptr(mk) if mk is not None else None, _ptr(out), _ptr(ws), ws.numel(),
                            int(max_iter), float(tol), C.byref(it), C.byref(ch), _stream()))
    return out, it.value, ch.value
