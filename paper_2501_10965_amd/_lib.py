"""ctypes declarations of the libdig C ABI (include/dig.h)."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdig.so")

DIG_OK, DIG_ERR_INVALID, DIG_ERR_CAPACITY, DIG_ERR_HIP, DIG_ERR_STATE, DIG_ERR_NUMERIC = range(6)
BC = {"periodic": 0, "diffuse": 1, "specular": 2, "freestream": 3}
GEOM = {"box": 0, "annulus": 1, "graded": 2}
STAGE_MOVE, STAGE_SORT, STAGE_COLLIDE, STAGE_ALL = 1, 2, 4, 7
SAMPLE_INSTANT, SAMPLE_AVERAGE, SAMPLE_RESET = 0, 1, 2
SYNTH_STATIC_BYTES = 32 << 20
SYNTH_SCHEMES = {"explicit": 0, "lusgs": 1}
EBIT_SORT_OVERFLOW, EBIT_GROUPS, EBIT_TARGET, EBIT_CAPACITY, EBIT_INFLOW = 1, 2, 4, 8, 16


class DigBC(C.Structure):
    _fields_ = [("type", C.c_int32), ("T", C.c_double), ("U", C.c_double * 3),
                ("rho", C.c_double)]


class DigConfig(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("geometry", C.c_int32),
                ("r_in", C.c_double), ("r_out", C.c_double), ("q", C.c_double),
                ("kn", C.c_double),
                ("omega", C.c_double), ("alpha", C.c_double), ("dr", C.c_int32),
                ("zrot", C.c_double), ("dt", C.c_double), ("weight", C.c_double),
                ("bc", DigBC * 4), ("seed", C.c_uint64), ("instance_id", C.c_uint32),
                ("sgmax_init", C.c_double), ("tref", C.c_double),
                ("xfaces", C.POINTER(C.c_double)), ("yfaces", C.POINTER(C.c_double))]


class DigLayout(C.Structure):
    _fields_ = [("total_bytes", C.c_size_t), ("capacity", C.c_int64), ("ncell", C.c_int64),
                ("x", C.c_size_t * 2), ("y", C.c_size_t * 2), ("vx", C.c_size_t * 2),
                ("vy", C.c_size_t * 2), ("vz", C.c_size_t * 2), ("er", C.c_size_t * 2),
                ("id", C.c_size_t * 2), ("cell", C.c_size_t), ("rank", C.c_size_t),
                ("perm_raw", C.c_size_t), ("perm", C.c_size_t), ("start", C.c_size_t),
                ("count", C.c_size_t), ("sgmax", C.c_size_t), ("acc", C.c_size_t),
                ("sums", C.c_size_t), ("cell_inst", C.c_size_t), ("cvol", C.c_size_t),
                ("counters", C.c_size_t)]


class DigSynthOpts(C.Structure):
    _fields_ = [("A", C.c_double * 4), ("cfl", C.c_double), ("wall_mode", C.c_int32),
                ("check_every", C.c_int32), ("scheme", C.c_int32), ("reserved", C.c_int32)]


class DigCounters(C.Structure):
    _fields_ = [("n", C.c_int64), ("step", C.c_int64), ("nsamp", C.c_int64),
                ("next_id", C.c_int64), ("candidates", C.c_int64), ("accepted", C.c_int64),
                ("inelastic", C.c_int64), ("saturated", C.c_int64), ("wall_hits", C.c_int64),
                ("removed", C.c_int64), ("injected", C.c_int64),
                ("err", C.c_uint32), ("cur", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DigTuning(C.Structure):
    _fields_ = [("group_particles", C.c_int32), ("group_cells", C.c_int32),
                ("seq_max", C.c_int32), ("big_stage_kib", C.c_int32),
                ("ms_per_step", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DigMlpLayout(C.Structure):
    _fields_ = [("total_bytes", C.c_size_t), ("max_batch", C.c_int32), ("params", C.c_size_t),
                ("grads", C.c_size_t), ("adam_m", C.c_size_t), ("adam_v", C.c_size_t),
                ("loss", C.c_size_t)]


MLP_NPARAM = 39312


class DigMlpScaling(C.Structure):
    _fields_ = [("x_mean", C.c_double * 9), ("x_std", C.c_double * 9),
                ("y_mean", C.c_double * 7), ("y_std", C.c_double * 7)]

    @classmethod
    def of(cls, sc: dict):
        v = cls()
        for k in ("x_mean", "x_std", "y_mean", "y_std"):
            arr = getattr(v, k)
            for i, val in enumerate(sc[k]):
                arr[i] = float(val)
        return v


# every exported entry point of include/dig.h
EXPORTS = ["dig_plan", "dsmc_create", "dsmc_init", "dsmc_inject", "dsmc_step", "dsmc_stage",
           "dsmc_sample", "dig_adjust", "closure_assemble", "dig_synth_workspace_bytes",
           "synth_solve", "dsmc_query", "dig_constants", "dsmc_profile", "dsmc_profile_kinds",
           "dsmc_tuning", "dsmc_autotune", "dsmc_step_graph", "mlp_plan", "mlp_create", "mlp_sync", "mlp_forward",
           "mlp_grad", "mlp_adam", "mlp_train_step", "mlp_destroy", "closure_features",
           "closure_blend", "dsmc_save", "dsmc_load", "synth_solve_static", "fields_fill_empty",
           "dig_last_error",
           "dsmc_destroy"]
KERNELS = ["move", "scan", "place", "order", "collide", "adjust", "sample", "closure"]

_lib = None


class DigError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdig error {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libdig.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libdig.so not built at {path}; run __graft_entry__.build()")
    # PyTorch's HIP runtime must be the process's HIP runtime: load it first so
    # that libdig's libamdhip64.so.7 dependency binds to it.
    import torch  # noqa: F401

    L = C.CDLL(path)
    vp, cp = C.c_void_p, C.POINTER(DigConfig)
    L.dig_plan.argtypes = [cp, C.c_int32, C.c_int64, C.POINTER(DigLayout)]
    L.dsmc_create.argtypes = [cp, C.c_int32, C.c_int64, vp, C.c_size_t, C.c_int32, C.c_int32,
                              vp, C.POINTER(vp)]
    L.dsmc_init.argtypes = [vp, vp, C.c_int32, vp]
    L.dsmc_inject.argtypes = [vp, C.c_int64, C.c_int64, C.c_int64, vp]
    L.dsmc_step.argtypes = [vp, C.c_int32, vp]
    L.dsmc_step_graph.argtypes = [vp, C.c_int32, vp]
    L.mlp_plan.argtypes = [C.c_int32, C.POINTER(DigMlpLayout)]
    L.mlp_create.argtypes = [vp, C.c_size_t, C.c_int32, vp, C.POINTER(vp)]
    L.mlp_sync.argtypes = [vp, vp]
    L.mlp_forward.argtypes = [vp, vp, vp, C.c_int64, vp]
    L.mlp_grad.argtypes = [vp, vp, vp, C.c_int64, vp]
    L.mlp_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int64, vp]
    L.mlp_train_step.argtypes = [vp, vp, vp, C.c_int64, C.c_float, C.c_int64, vp]
    L.mlp_destroy.argtypes = [vp]
    L.closure_features.argtypes = [vp, vp, vp, vp, C.POINTER(DigMlpScaling), vp, vp, vp]
    L.closure_blend.argtypes = [vp, vp, vp, vp, vp, C.POINTER(DigMlpScaling),
                                C.POINTER(C.c_double), C.c_double, C.c_double, C.c_double,
                                C.c_double, C.c_double, vp, vp, vp]
    L.mlp_destroy.restype = None
    L.dsmc_tuning.argtypes = [vp, C.POINTER(DigTuning), C.POINTER(DigTuning)]
    L.dsmc_autotune.argtypes = [vp, C.c_int32, C.c_char_p, C.POINTER(DigTuning), vp]
    L.dsmc_stage.argtypes = [vp, C.c_int32, vp]
    L.dsmc_sample.argtypes = [vp, C.c_int32, vp, vp]
    L.dig_adjust.argtypes = [vp, vp, C.c_uint32, vp]
    L.fields_fill_empty.argtypes = [vp, vp, vp, vp]
    L.closure_assemble.argtypes = [vp, vp, C.POINTER(C.c_double), C.c_double, C.c_double, vp,
                                   vp, vp, vp, vp]
    L.dsmc_query.argtypes = [vp, C.POINTER(DigCounters), vp]
    L.synth_solve_static.argtypes = [cp, C.POINTER(DigSynthOpts), vp, vp, vp, vp, C.c_int32,
                                     C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                     vp]
    L.dsmc_save.argtypes = [vp, vp, C.POINTER(C.c_size_t), vp]
    L.dsmc_load.argtypes = [vp, vp, C.c_size_t, vp]
    L.dig_constants.argtypes = [vp, C.c_int32, C.POINTER(C.c_double)]
    L.dsmc_profile.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64), vp]
    L.dsmc_profile_kinds.argtypes = [vp, C.c_uint32, C.c_int32]
    L.dig_synth_workspace_bytes.argtypes = [cp]
    L.dig_synth_workspace_bytes.restype = C.c_size_t
    L.synth_solve.argtypes = [cp, C.POINTER(DigSynthOpts), vp, vp, vp, vp, vp, C.c_size_t,
                              C.c_int32, C.c_double, C.POINTER(C.c_int32),
                              C.POINTER(C.c_double), vp]
    L.dig_last_error.restype = C.c_char_p
    L.dsmc_destroy.argtypes = [vp]
    L.dsmc_destroy.restype = None
    for name in EXPORTS:
        if name not in ("dig_last_error", "dsmc_destroy", "dig_synth_workspace_bytes",
                        "mlp_destroy"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(code: int):
    if code != DIG_OK:
        raise DigError(code, load().dig_last_error().decode())
    return code


def make_config(w: dict) -> DigConfig:
    """libdig configuration from a workload description."""
    c = DigConfig()
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
        c.bc[f].type = BC[bc[0]]
        c.bc[f].T = bc[1]
        for k in range(3):
            c.bc[f].U[k] = bc[2][k]
        c.bc[f].rho = bc[3] if len(bc) > 3 else 0.0
    c.seed = w["seed"]
    c.instance_id = w.get("instance", 0)
    c.sgmax_init = w.get("sgmax_init", 0.0)
    c.tref = w.get("tref", 1.0)
    if c.geometry == GEOM["graded"]:
        # face tables held by the configuration object for its lifetime
        c._xf = (C.c_double * (c.nx + 1))(*[float(v) for v in w["xfaces"]])
        c.xfaces = C.cast(c._xf, C.POINTER(C.c_double))
        if c.dim == 2:
            c._yf = (C.c_double * (c.ny + 1))(*[float(v) for v in w["yfaces"]])
            c.yfaces = C.cast(c._yf, C.POINTER(C.c_double))
    return c
