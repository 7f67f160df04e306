"""FP64 CPU oracle for the DSMC + DIG hot path (arXiv:2501.10965).

TEST INFRASTRUCTURE ONLY.  The tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers; the product path never
imports this package.  The C source (``dsmc_oracle.c``) is a plain, single
threaded, double precision transcription of the method: Philox streams,
initialisation, free flight with diffuse walls, stable counting sort, NTC/VHS
collisions with Borgnakke-Larsen exchange, moment sampling, DIG particle
modification and closure assembly.  ``synth.py`` and ``mlp.py`` hold the
synthetic-equation and learned-closure oracles (numpy, FP64).

The HIP library shares no code with this package; both are driven from the
same workload descriptions in ``dig_workloads``.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_DIR, "liboracle.so")
_SRC = [os.path.join(_DIR, "dsmc_oracle.c")]

BC = {"periodic": 0, "diffuse": 1, "specular": 2, "freestream": 3}
GEOM = {"box": 0, "annulus": 1, "graded": 2}
TAG = {"init": 1, "init_n": 2, "wall": 3, "ncand": 4, "coll": 5, "dig_n": 6,
       "dig_del": 7, "dig_src": 8, "dig_empty": 9, "inflow": 10, "er": 11, "bl": 12}


def build(force: bool = True) -> str:
    """Compile the C oracle with plain IEEE double arithmetic (no contraction)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-o", _SO] + _SRC + ["-lm"]
        subprocess.run(cmd, check=True)
    return _SO


class Config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("geometry", C.c_int32),
                ("r_in", C.c_double), ("r_out", C.c_double), ("q", C.c_double),
                ("kn", C.c_double), ("omega", C.c_double), ("alpha", C.c_double),
                ("dr", C.c_int32), ("zrot", C.c_double),
                ("dt", C.c_double), ("weight", C.c_double),
                ("bc_type", C.c_int32 * 4), ("bc_T", C.c_double * 4),
                ("bc_U", (C.c_double * 3) * 4), ("bc_rho", C.c_double * 4),
                ("seed", C.c_uint64), ("instance", C.c_uint32),
                ("xf", C.POINTER(C.c_double)), ("yf", C.POINTER(C.c_double))]


class Stats(C.Structure):
    _fields_ = [("candidates", C.c_int64), ("accepted", C.c_int64),
                ("inelastic", C.c_int64), ("saturated", C.c_int64)]


_lib = None

_d = C.POINTER(C.c_double)
_f = C.POINTER(C.c_float)
_u32 = C.POINTER(C.c_uint32)
_i32 = C.POINTER(C.c_int32)
_i64 = C.POINTER(C.c_int64)
_u8 = C.POINTER(C.c_uint8)


def _configure(L):
    """Sets the argument and result types of the oracle's C entry points."""
    cp = C.POINTER(Config)
    L.orc_philox.argtypes = [_u32, _u32, _u32]
    L.orc_draw.argtypes = [cp, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, _u32]
    L.orc_u01.argtypes = [C.c_uint32]
    L.orc_u01.restype = C.c_double
    L.orc_pick.argtypes = [C.c_uint32, C.c_uint32]
    L.orc_pick.restype = C.c_uint32
    for fn in ("orc_mu0", "orc_csigma", "orc_pinelastic", "orc_cell_volume"):
        getattr(L, fn).argtypes = [cp]
        getattr(L, fn).restype = C.c_double
    L.orc_cell_volume_at.argtypes = [cp, C.c_int32]
    L.orc_cell_volume_at.restype = C.c_double
    L.orc_annulus_face.argtypes = [cp, C.c_int32]
    L.orc_annulus_face.restype = C.c_double
    L.orc_inject.argtypes = [cp, C.c_int64, C.c_int64, _d, _d, _d, _d, _d, _d, _u32,
                             C.c_uint32, C.c_uint64]
    L.orc_inject.restype = C.c_int64
    L.orc_init.argtypes = [cp, _d, C.c_int32, C.c_int64, _d, _d, _d, _d, _d, _d, _u32,
                           _i64]
    L.orc_init.restype = C.c_int64
    L.orc_move.argtypes = [cp, C.c_int64, _d, _d, _d, _d, _d, _d, _u32, C.c_uint32]
    L.orc_move.restype = C.c_int64
    L.orc_cell_index.argtypes = [cp, C.c_int64, _d, _d, _i32]
    L.orc_sort.argtypes = [C.c_int64, _i32, C.c_int32, _i64, _i64]
    L.orc_collide.argtypes = [cp, C.c_int32, _i64, _d, _d, _d, _d, _f, C.c_uint32,
                              C.POINTER(Stats), _d, _d]
    L.orc_sample_sums.argtypes = [C.c_int32, _i64, _d, _d, _d, _d, _d]
    L.orc_sums_to_fields.argtypes = [cp, C.c_int32, _d, C.c_double, _d]
    L.orc_adjust.argtypes = [cp, C.c_int32, _i64, _d, _d, _d, _d, _d, _d, _u32, _d,
                             C.c_uint32, C.c_uint64, C.c_int64, _d, _d, _d, _d, _d,
                             _d, _u32, _i64, _i64, C.POINTER(C.c_uint64)]
    L.orc_adjust.restype = C.c_int
    L.orc_closure.argtypes = [cp, _d, _d, C.c_double, C.c_double, _d, _u8, _d, _d]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = _configure(C.CDLL(_SO))
    return _lib


def build_variant(edits, out_dir: str) -> str:
    """Compiles a copy of the C oracle with textual edits applied.

    edits: sequence of (old, new) strings; each `old` must occur exactly once
    in the source.  Used only by tests that plant a plausible mistake in the
    oracle to show that a pin catches it.  Returns the path of the library."""
    text = open(_SRC[0], encoding="utf-8").read()
    for old, new in edits:
        if text.count(old) != 1:
            raise ValueError(f"edit target occurs {text.count(old)} times: {old!r}")
        text = text.replace(old, new)
    os.makedirs(out_dir, exist_ok=True)
    tag = abs(hash(tuple(edits))) % (1 << 40)
    src = os.path.join(out_dir, f"variant_{tag:x}.c")
    so = os.path.join(out_dir, f"libvariant_{tag:x}.so")
    with open(src, "w", encoding="utf-8") as f:
        f.write(text)
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                    "-shared", "-fPIC", "-I", _DIR, "-o", so, src, "-lm"], check=True)
    return so


@contextlib.contextmanager
def variant(edits, out_dir: str):
    """Within the block, every oracle call uses a copy compiled with `edits`."""
    global _lib
    saved = lib()
    _lib = _configure(C.CDLL(build_variant(edits, out_dir)))
    try:
        yield _lib
    finally:
        _lib = saved


def _p(a: np.ndarray, t):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(t)


def make_config(w: dict) -> Config:
    """Oracle configuration from a workload description (see dig_workloads)."""
    c = Config()
    c.dim = w["dim"]
    c.nx = w["nx"]
    c.ny = w.get("ny", 1)
    c.lx = w.get("lx", 1.0)
    c.ly = w.get("ly", 1.0)
    c.geometry = GEOM[w.get("geometry", "box")]
    c.r_in = w.get("r_in", 0.0)
    c.r_out = w.get("r_out", 0.0)
    c.q = w.get("q", 1.0)
    c.kn = w["kn"]
    c.omega = w["omega"]
    c.alpha = w.get("alpha", 1.0)
    c.dr = w.get("dr", 2)
    c.zrot = w["zrot"]
    c.dt = w["dt"]
    c.weight = w["weight"]
    for f, bc in enumerate(w["bc"]):
        c.bc_type[f] = BC[bc[0]]
        c.bc_T[f] = bc[1]
        for k in range(3):
            c.bc_U[f][k] = bc[2][k]
        c.bc_rho[f] = bc[3] if len(bc) > 3 else 0.0
    c.seed = w["seed"]
    c.instance = w.get("instance", 0)
    if c.geometry == GEOM["graded"]:
        # the face tables live as long as the configuration
        c._xf = np.ascontiguousarray(w["xfaces"], dtype=np.float64)
        c._yf = np.ascontiguousarray(w["yfaces"] if c.dim == 2 else [0.0, 1.0],
                                     dtype=np.float64)
        assert len(c._xf) == c.nx + 1 and len(c._yf) == (c.ny + 1 if c.dim == 2 else 2)
        c.xf = c._xf.ctypes.data_as(C.POINTER(C.c_double))
        c.yf = c._yf.ctypes.data_as(C.POINTER(C.c_double))
    return c


# --------------------------------------------------------------------------
def philox(ctr, key):
    a = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_p(a, _u32), _p(k, _u32), _p(out, _u32))
    return out


def csigma(w):
    return lib().orc_csigma(C.byref(make_config(w)))


def pinelastic(w):
    return lib().orc_pinelastic(C.byref(make_config(w)))


def mu0(w):
    return lib().orc_mu0(C.byref(make_config(w)))


def cell_volume(w, cell=None):
    if cell is None:
        return lib().orc_cell_volume(C.byref(make_config(w)))
    return lib().orc_cell_volume_at(C.byref(make_config(w)), int(cell))


def annulus_face(w, j):
    return lib().orc_annulus_face(C.byref(make_config(w)), int(j))


class State:
    """Particle state of one instance in FP64 (positions in grid units)."""

    def __init__(self, w: dict, cap: int):
        self.w = w
        self.cfg = make_config(w)
        self.ncell = w["nx"] * w.get("ny", 1)
        self.cap = int(cap)
        z = lambda: np.zeros(self.cap, dtype=np.float64)
        self.x, self.y, self.vx, self.vy, self.vz, self.er = z(), z(), z(), z(), z(), z()
        self.id = np.zeros(self.cap, dtype=np.uint32)
        self.n = 0
        self.start = np.zeros(self.ncell + 1, dtype=np.int64)
        self.sgmax = np.zeros(self.ncell, dtype=np.float32)
        self.acc = np.zeros((self.ncell, 17), dtype=np.float64)
        self.nsamp = 0
        self.step_no = 0
        self.next_id = 0

    # -- state injection --------------------------------------------------
    def load(self, x, y, vx, vy, vz, er, id_, start=None, sgmax=None, step=None,
             next_id=None):
        n = len(x)
        assert n <= self.cap
        for dst, src in ((self.x, x), (self.y, y), (self.vx, vx), (self.vy, vy),
                         (self.vz, vz), (self.er, er)):
            dst[:n] = np.asarray(src, dtype=np.float64)
        self.id[:n] = np.asarray(id_, dtype=np.uint32)
        self.n = n
        if start is not None:
            self.start[:] = np.asarray(start, dtype=np.int64)
        if sgmax is not None:
            self.sgmax[:] = np.asarray(sgmax, dtype=np.float32)
        if step is not None:
            self.step_no = int(step)
        if next_id is not None:
            self.next_id = int(next_id)

    def arrays(self):
        n = self.n
        return dict(x=self.x[:n].copy(), y=self.y[:n].copy(), vx=self.vx[:n].copy(),
                    vy=self.vy[:n].copy(), vz=self.vz[:n].copy(), er=self.er[:n].copy(),
                    id=self.id[:n].copy())

    # -- steps -------------------------------------------------------------
    def init(self, fields: np.ndarray, ppc: int, sgmax0: float):
        f = np.ascontiguousarray(fields, dtype=np.float64)
        n = lib().orc_init(C.byref(self.cfg), _p(f, _d), int(ppc), self.cap, _p(self.x, _d),
                           _p(self.y, _d), _p(self.vx, _d), _p(self.vy, _d), _p(self.vz, _d),
                           _p(self.er, _d), _p(self.id, _u32), _p(self.start, _i64))
        if n < 0:
            raise RuntimeError("oracle init: capacity exceeded")
        self.n = int(n)
        self.next_id = self.n
        self.sgmax[:] = np.float32(sgmax0)

    def move(self):
        return lib().orc_move(C.byref(self.cfg), self.n, _p(self.x, _d), _p(self.y, _d),
                              _p(self.vx, _d), _p(self.vy, _d), _p(self.vz, _d),
                              _p(self.er, _d), _p(self.id, _u32), self.step_no)

    def cells(self):
        cell = np.zeros(max(self.n, 1), dtype=np.int32)
        lib().orc_cell_index(C.byref(self.cfg), self.n, _p(self.x, _d), _p(self.y, _d),
                             _p(cell, _i32))
        return cell[: self.n]

    def sort(self):
        """Stable counting sort by cell; returns the permutation applied."""
        cell = np.ascontiguousarray(self.cells())
        perm = np.zeros(max(self.n, 1), dtype=np.int64)
        lib().orc_sort(self.n, _p(cell, _i32), self.ncell, _p(perm, _i64),
                       _p(self.start, _i64))
        n_new = int(self.start[-1])  # particles outside an open boundary are dropped
        perm = perm[:n_new]
        for a in (self.x, self.y, self.vx, self.vy, self.vz, self.er, self.id):
            a[:n_new] = a[: self.n][perm]
        self.n = n_new
        return perm

    def inject(self):
        """Freestream inflow of this step appended after the current particles."""
        k = lib().orc_inject(C.byref(self.cfg), self.n, self.cap, _p(self.x, _d),
                             _p(self.y, _d), _p(self.vx, _d), _p(self.vy, _d), _p(self.vz, _d),
                             _p(self.er, _d), _p(self.id, _u32), self.step_no, self.next_id)
        if k < 0:
            raise RuntimeError("oracle inflow: capacity exceeded")
        self.n += int(k)
        self.next_id += int(k)
        return int(k)

    def collide(self, with_obs=False):
        st = Stats()
        obs = np.zeros(self.ncell, dtype=np.float64)
        margin = np.zeros(self.ncell, dtype=np.float64)
        lib().orc_collide(C.byref(self.cfg), self.ncell, _p(self.start, _i64),
                          _p(self.vx, _d), _p(self.vy, _d), _p(self.vz, _d), _p(self.er, _d),
                          _p(self.sgmax, _f), self.step_no, C.byref(st), _p(obs, _d),
                          _p(margin, _d))
        res = dict(candidates=st.candidates, accepted=st.accepted, inelastic=st.inelastic,
                   saturated=st.saturated)
        if with_obs:
            res["obs"] = obs
            res["margin"] = margin
        return res

    def sums(self):
        s = np.zeros((self.ncell, 17), dtype=np.float64)
        lib().orc_sample_sums(self.ncell, _p(self.start, _i64), _p(self.vx, _d),
                              _p(self.vy, _d), _p(self.vz, _d), _p(self.er, _d), _p(s, _d))
        return s

    def step(self, sample=True):
        """One DSMC step: inflow (open boundaries), move, index + stable sort,
        collide, sample."""
        if self.w.get("geometry") == "annulus" and self.w["bc"][1][0] == "freestream":
            self.inject()
        self.move()
        self.sort()
        st = self.collide()
        if sample:
            self.acc += self.sums()
            self.nsamp += 1
        self.step_no += 1
        return st

    def fields(self, sums=None, nsteps=None):
        if sums is None:
            sums, nsteps = self.acc, max(self.nsamp, 1)
        s = np.ascontiguousarray(sums, dtype=np.float64)
        out = np.zeros((20, self.ncell), dtype=np.float64)
        lib().orc_sums_to_fields(C.byref(self.cfg), self.ncell, _p(s, _d), float(nsteps),
                                 _p(out, _d))
        return out

    def reset_average(self):
        self.acc[:] = 0.0
        self.nsamp = 0

    def adjust(self, target: np.ndarray, dig_iter: int):
        t = np.ascontiguousarray(target, dtype=np.float64)
        out = State(self.w, self.cap)
        n_out = C.c_int64(0)
        nid = C.c_uint64(0)
        rc = lib().orc_adjust(C.byref(self.cfg), self.ncell, _p(self.start, _i64),
                              _p(self.x, _d), _p(self.y, _d), _p(self.vx, _d), _p(self.vy, _d),
                              _p(self.vz, _d), _p(self.er, _d), _p(self.id, _u32), _p(t, _d),
                              int(dig_iter), self.next_id, self.cap, _p(out.x, _d),
                              _p(out.y, _d), _p(out.vx, _d), _p(out.vy, _d), _p(out.vz, _d),
                              _p(out.er, _d), _p(out.id, _u32), _p(out.start, _i64),
                              C.byref(n_out), C.byref(nid))
        if rc != 0:
            return rc
        for name in ("x", "y", "vx", "vy", "vz", "er", "id", "start"):
            setattr(self, name, getattr(out, name))
        self.n = int(n_out.value)
        self.next_id = int(nid.value)
        return 0


def closure(w: dict, fields: np.ndarray, A, kn_ref: float, n_min: float = 0.0):
    cfg = make_config(w)
    ncell = w["nx"] * w.get("ny", 1)
    f = np.ascontiguousarray(fields, dtype=np.float64)
    assert f.shape == (20, ncell), f.shape  # rows as produced by the sampling (row 19: N)
    a = np.ascontiguousarray(A, dtype=np.float64)
    hot = np.zeros((12, ncell))
    nsf = np.zeros((12, ncell))
    mask = np.zeros(ncell, dtype=np.uint8)
    kn = np.zeros(ncell)
    lib().orc_closure(C.byref(cfg), _p(f, _d), _p(a, _d), float(kn_ref), float(n_min), _p(hot, _d),
                      _p(mask, _u8), _p(kn, _d), _p(nsf, _d))
    return hot, mask, kn, nsf


def fill_empty(fields: np.ndarray, fallback: np.ndarray, dr: int = 2) -> np.ndarray:
    """Cells of a time average [20, C] without a usable sample (mean count,
    row 19, not positive; rho or Tt not positive; Tr negative; or rows 0..5
    not finite) take rho, u, Tt, Tr from fallback [6, C] (the previous
    macroscopic solution of the DIG loop), zero stresses and heat fluxes,
    the total temperature (3 Tt + d_r Tr) / (3 + d_r) of the fallback, and
    N = 0.  Returns a new array.  (Not in the paper: the thinnest cells of a
    wall-refined grid can stay empty over a whole DIG cycle, and the
    synthetic solve needs a state in every cell.)"""
    f = np.array(fields, dtype=np.float64, copy=True)
    fb = np.asarray(fallback, dtype=np.float64)
    for c in range(f.shape[1]):
        rho, tt, tr, n = f[0, c], f[4, c], f[5, c], f[19, c]
        usable = (n > 0 and rho > 0 and tt > 0 and tr >= 0
                  and all(np.isfinite(f[k, c]) for k in range(6)))
        if usable:
            continue
        f[0:6, c] = fb[0:6, c]
        f[6:18, c] = 0.0
        f[18, c] = (3.0 * fb[4, c] + dr * fb[5, c]) / (3.0 + dr)
        f[19, c] = 0.0
    return f


def sgmax_default(w: dict) -> float:
    """Initial majorant of sigma_T g per cell: the VHS value at a relative speed
    of six times the relative-velocity spread at the workload's reference
    temperature (raised later to the observed maximum)."""
    g = 6.0 * np.sqrt(2.0 * w["tref"])
    return csigma(w) * g ** (2.0 - 2.0 * w["omega"])


def new_state(w: dict, cap_factor: float = 1.3, cap: int | None = None) -> "State":
    """Oracle state of a workload, initialised with its uniform fields."""
    import dig_workloads as _wl  # input recipes only

    nc = w["nx"] * w.get("ny", 1)
    if cap is None:
        est = nc * w["ppc"] if w["ppc"] > 0 else w["n_target"]
        cap = int(est * cap_factor) + 64
    s = State(w, cap)
    s.init(_wl.fields_uniform(w), w["ppc"], sgmax_default(w))
    return s
