"""Seeded synthetic workloads shared by the HIP library's tests/bench and the oracle.

This module only describes inputs (geometry, gas parameters, boundary
conditions, seeds, initial fields and counts); it holds none of the method's
arithmetic.  Every workload is synthetic, with the structure of the paper's
cases: equilibrium Maxwellian starts, tens to thousands of particles per cell,
fully diffuse isothermal walls, nitrogen-like VHS parameters (omega = 0.74,
alpha = 1, two rotational degrees of freedom).

Time steps are stated as a fraction of the mean collision time at unit density
and temperature; ``TAU_C_PER_KN`` is that time per unit Knudsen number for
omega = 0.74 (the oracle test suite checks it against the oracle's collision
rate).
"""
from __future__ import annotations

import copy
import math

import numpy as np

OMEGA_N2 = 0.74
TAU_C_PER_KN = 0.5167738723407999      # (5-2w)(7-2w) sqrt(2/pi) / 30 at w = 0.74
LID_MA03 = 0.35496478698597694         # 0.3 * sqrt(1.4)
U_INF_MA5 = 5.916079783099616          # 5 * sqrt(1.4)


def _bc(kind, T=1.0, U=(0.0, 0.0, 0.0)):
    return (kind, float(T), tuple(float(u) for u in U))


def box(dim, nx, ny=1, lx=1.0, ly=1.0, kn=0.05, zrot=5.0, omega=OMEGA_N2, ppc=50,
        dt_frac=0.2, bc=None, seed=1, instance=0, rho=1.0, u=(0.0, 0.0, 0.0), Tt=1.0,
        Tr=None, tref=None, dt=None, dr=2):
    """A uniform box workload with uniform initial fields.  dr: rotational
    degrees of freedom (2..6)."""
    if bc is None:
        bc = [_bc("periodic")] * 4
    ny = ny if dim == 2 else 1
    vol = (lx / nx) * ((ly / ny) if dim == 2 else 1.0)
    Tr = Tt if Tr is None else Tr
    if dt is None:
        dt = dt_frac * TAU_C_PER_KN * kn
    temps = [Tt, Tr] + [b[1] for b in bc if b[0] == "diffuse"]
    return dict(dim=dim, nx=nx, ny=ny, lx=lx, ly=ly, kn=kn, omega=omega, alpha=1.0, dr=dr,
                zrot=zrot, dt=dt, weight=rho * vol / ppc, bc=bc, seed=seed,
                instance=instance, ppc=ppc,
                init=dict(rho=rho, u=tuple(u), Tt=Tt, Tr=Tr),
                tref=max(temps) if tref is None else tref)


def fields_uniform(w):
    """Initial fields [rho, ux, uy, uz, Tt, Tr] (6 x ncell) of a workload."""
    nc = w["nx"] * w["ny"]
    i = w["init"]
    f = np.empty((6, nc), dtype=np.float64)
    f[0] = i["rho"]
    f[1], f[2], f[3] = i["u"]
    f[4] = i["Tt"]
    f[5] = i["Tr"]
    return f


# ---------------------------------------------------------------------------
# The five configurations.

def fourier_1d(seed=1001, nx=100, ppc=50, kn=0.05, zrot=5.0):
    """1D Fourier heat transfer between diffuse plates at T = 1.0 and 1.5."""
    bc = [_bc("diffuse", 1.0), _bc("diffuse", 1.5), _bc("periodic"), _bc("periodic")]
    w = box(1, nx, kn=kn, zrot=zrot, ppc=ppc, bc=bc, seed=seed, Tt=1.25, Tr=1.25)
    w["steps"] = 2000
    w["name"] = f"fourier1d_{nx}c_{ppc}ppc_kn{kn}"
    return w


def cavity_2d(seed=2001, n=200, ppc=50, kn=0.01, lid=LID_MA03, zrot=5.0):
    """Lid-driven cavity: diffuse walls at T = 1, lid (y = 1) moving in +x."""
    bc = [_bc("diffuse", 1.0), _bc("diffuse", 1.0), _bc("diffuse", 1.0),
          _bc("diffuse", 1.0, (lid, 0.0, 0.0))]
    w = box(2, n, n, kn=kn, zrot=zrot, ppc=ppc, bc=bc, seed=seed)
    w["ns"] = 50
    w["name"] = f"cavity2d_{n}x{n}_{ppc}ppc_kn{kn}"
    return w


BATCH_CELLS = [100, 139, 193, 268, 373, 518, 720, 1000]
BATCH_PPC = [20, 39, 75, 144, 278, 537, 1036, 2000]


def batch_1d(n_inst=64, seed_base=3000, scale=1.0):
    """64 uneven 1D instances: Kn log-spaced 1e-3..1, Z in {3, 5, 10}, even
    instances Fourier (walls 1.0 / 1.5), odd instances Couette (T = 1, walls
    moving -0.5 / +0.5 in y).  ``scale`` < 1 shrinks particle counts for tests."""
    out = []
    for i in range(n_inst):
        nx = BATCH_CELLS[i % 8]
        ppc = max(2, int(round(BATCH_PPC[(i // 8) % 8] * scale)))
        kn = 10.0 ** (-3.0 + 3.0 * ((29 * i) % 64) / 63.0)
        zrot = [3.0, 5.0, 10.0][i % 3]
        if i % 2 == 0:
            bc = [_bc("diffuse", 1.0), _bc("diffuse", 1.5), _bc("periodic"), _bc("periodic")]
            T0 = 1.25
        else:
            bc = [_bc("diffuse", 1.0, (0, -0.5, 0)), _bc("diffuse", 1.0, (0, 0.5, 0)),
                  _bc("periodic"), _bc("periodic")]
            T0 = 1.0
        dx = 1.0 / nx
        dt = min(0.2 * TAU_C_PER_KN * kn, 0.5 * dx / math.sqrt(8.0 * 1.5 / math.pi))
        w = box(1, nx, kn=kn, zrot=zrot, ppc=ppc, bc=bc, seed=seed_base + i, instance=i,
                Tt=T0, Tr=T0, dt=dt)
        w["name"] = f"batch{i}"
        out.append(w)
    return out


def scaled(w, **kw):
    v = copy.deepcopy(w)
    v.update(kw)
    return v


def random_sorted_state(w, seed, n_per_cell_mean=None, rng_kind="poisson"):
    """A cell-sorted random particle state for injection into both sides:
    per-cell counts (Poisson), positions uniform in the cell (grid units),
    Maxwellian velocities around the initial flow, exponential rotational
    energies.  Returns (x, y, vx, vy, vz, er, id, start) in float32/uint32."""
    rng = np.random.default_rng(seed)
    nc = w["nx"] * w["ny"]
    if n_per_cell_mean is not None:
        lam = n_per_cell_mean
    elif w.get("geometry") == "graded":
        fx = np.diff(np.asarray(w["xfaces"]))
        fy = np.diff(np.asarray(w["yfaces"])) if w["dim"] == 2 else np.ones(1)
        lam = w["init"]["rho"] * np.outer(fy, fx).ravel() / w["weight"]
    else:
        lam = w["ppc"]
    counts = rng.poisson(lam, size=nc) if rng_kind == "poisson" else \
        np.full(nc, int(lam)) if np.isscalar(lam) else np.rint(lam).astype(np.int64)
    start = np.zeros(nc + 1, dtype=np.int64)
    start[1:] = np.cumsum(counts)
    n = int(start[-1])
    cell = np.repeat(np.arange(nc), counts)
    ix = cell % w["nx"]
    iy = cell // w["nx"]
    if w.get("geometry") == "graded":
        # physical units, uniform in the cell, strictly inside its FP32 faces
        fx = np.asarray(w["xfaces"])
        x = fx[ix] + rng.random(n) * (fx[ix + 1] - fx[ix])
        x = np.clip(x.astype(np.float32), np.nextafter(fx[ix].astype(np.float32), np.float32(2)),
                    np.nextafter(fx[ix + 1].astype(np.float32), np.float32(0)))
        if w["dim"] == 2:
            fy = np.asarray(w["yfaces"])
            y = fy[iy] + rng.random(n) * (fy[iy + 1] - fy[iy])
            y = np.clip(y.astype(np.float32),
                        np.nextafter(fy[iy].astype(np.float32), np.float32(2)),
                        np.nextafter(fy[iy + 1].astype(np.float32), np.float32(0)))
        else:
            y = np.zeros(n, dtype=np.float32)
    else:
        x = (ix + rng.random(n)).astype(np.float32)
        y = ((iy + rng.random(n)) if w["dim"] == 2 else np.zeros(n)).astype(np.float32)
        # keep positions strictly inside their cell after rounding to float32
        x = np.minimum(x, np.nextafter((ix + 1).astype(np.float32), np.float32(0)))
        if w["dim"] == 2:
            y = np.minimum(y, np.nextafter((iy + 1).astype(np.float32), np.float32(0)))
    i = w["init"]
    s = math.sqrt(i["Tt"])
    vx = (i["u"][0] + s * rng.standard_normal(n)).astype(np.float32)
    vy = (i["u"][1] + s * rng.standard_normal(n)).astype(np.float32)
    vz = (i["u"][2] + s * rng.standard_normal(n)).astype(np.float32)
    er = (i["Tr"] * rng.exponential(size=n)).astype(np.float32)
    ids = rng.permutation(n).astype(np.uint32)
    return dict(x=x, y=y, vx=vx, vy=vy, vz=vz, er=er, id=ids, start=start)


def wall_refined_faces(n, length=1.0, first=0.001):
    """Face coordinates of n cells on [0, length] refined toward both ends:
    the width of cell k is first * q^min(k, n - 1 - k), with the ratio q found
    by bisection so that the widths add up to `length` (q = 1 when first
    = length / n).  Returns n + 1 float64 values from 0 to length."""
    k = np.minimum(np.arange(n), n - 1 - np.arange(n)).astype(np.float64)

    def total(q):
        return float(np.sum(first * q ** k))

    if abs(total(1.0) - length) < 1e-14 * length:
        q = 1.0
    else:
        lo, hi = 1.0, 2.0
        while total(hi) < length:
            hi *= 2.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if total(mid) < length:
                lo = mid
            else:
                hi = mid
        q = 0.5 * (lo + hi)
    widths = first * q ** k
    faces = np.concatenate([[0.0], np.cumsum(widths)])
    faces *= length / faces[-1]
    faces[-1] = length
    return faces


def graded_box(dim, xfaces, yfaces=None, kn=0.05, zrot=5.0, omega=OMEGA_N2, ppc=50,
               dt_frac=0.2, bc=None, seed=1, instance=0, rho=1.0, u=(0.0, 0.0, 0.0), Tt=1.0,
               Tr=None, tref=None, dt=None):
    """A box with cells of different widths between the face tables xfaces
    (nx + 1 values from 0 to lx) and yfaces (dim 2).  One particle weight for
    all cells, set so that the mean count per cell is `ppc` at density rho;
    counts then follow the cell volumes (Iround(rho V / N_eff))."""
    xfaces = np.asarray(xfaces, dtype=np.float64)
    nx = len(xfaces) - 1
    if dim == 2:
        yfaces = np.asarray(yfaces, dtype=np.float64)
        ny = len(yfaces) - 1
    else:
        yfaces, ny = np.array([0.0, 1.0]), 1
    lx, ly = float(xfaces[-1]), float(yfaces[-1])
    w = box(dim, nx, ny, lx=lx, ly=ly, kn=kn, zrot=zrot, omega=omega, ppc=ppc,
            dt_frac=dt_frac, bc=bc, seed=seed, instance=instance, rho=rho, u=u, Tt=Tt, Tr=Tr,
            tref=tref, dt=dt)
    w.update(geometry="graded", xfaces=xfaces.tolist(), yfaces=yfaces.tolist(), ppc=0,
             weight=rho * lx * (ly if dim == 2 else 1.0) / (ppc * nx * ny),
             n_target=int(ppc * nx * ny))
    return w


def cavity_graded(seed=2101, n=100, first=0.001, ppc=50, kn=0.01, lid=LID_MA03, zrot=5.0,
                  dt_frac=0.2):
    """Lid-driven cavity on n x n cells refined toward all four walls (first
    cell width `first`), diffuse walls at T = 1, lid (y = 1) moving in +x."""
    f = wall_refined_faces(n, 1.0, first)
    bc = [_bc("diffuse", 1.0), _bc("diffuse", 1.0), _bc("diffuse", 1.0),
          _bc("diffuse", 1.0, (lid, 0.0, 0.0))]
    w = graded_box(2, f, f, kn=kn, zrot=zrot, ppc=ppc, bc=bc, seed=seed, dt_frac=dt_frac)
    w["ns"] = 50
    w["name"] = f"cavity_graded_{n}x{n}_first{first}_kn{kn}"
    return w


def mlp_init(seed=7):
    """Initial weights of the closure network: Glorot-uniform over the real
    fan-in/fan-out (9 inputs, 7 outputs), zero padding and zero biases; values
    representable in FP32.  Returned as float64 arrays keyed W0..W3, b0..b3."""
    rng = np.random.default_rng(seed)
    dims = [(32, 128, 9, 128), (128, 128, 128, 128), (128, 128, 128, 128), (128, 16, 128, 7)]
    p = {}
    for l, (fin, fout, rin, rout) in enumerate(dims):
        s = math.sqrt(6.0 / (rin + rout))
        W = np.zeros((fout, fin))
        W[:rout, :rin] = rng.uniform(-s, s, size=(rout, rin))
        p[f"W{l}"] = W.astype(np.float32).astype(np.float64)
        p[f"b{l}"] = np.zeros(fout)
    return p


def radial_ratio(r_in, r_out, nr, first):
    """Geometric radial stretch ratio q with first cell width `first`:
    (r_out - r_in)(q - 1)/(q^nr - 1) = first (bisection)."""
    span = r_out - r_in
    if abs(span / nr - first) < 1e-15:
        return 1.0
    lo, hi = 1.0 + 1e-12, 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        w1 = span * (mid - 1.0) / (mid ** nr - 1.0)
        if w1 > first:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def cylinder(seed=5001, nth=500, nr=400, r_in=0.5, r_out=5.5, first=0.002, kn=0.01,
             mach=5.0, n_target=50_000_000, dt_frac=0.1, zrot=5.0, Tw=1.0, outer="freestream"):
    """Flow of a diatomic gas past a cylinder of radius r_in: annulus
    r_in < r < r_out, nth angular x nr radial cells with geometric radial
    stretching from a first cell of width `first`; isothermal diffuse cylinder
    wall; freestream (rho = 1, T = 1, U = Mach sqrt(1.4) along +x) at the outer
    circle.  One particle weight for all cells, set by n_target particles at
    rho = 1.  Initial gas at rest, rho = 1, T = 1."""
    q = radial_ratio(r_in, r_out, nr, first)
    U = mach * math.sqrt(1.4)
    area = math.pi * (r_out * r_out - r_in * r_in)
    if outer == "freestream":
        ob = ("freestream", 1.0, (U, 0.0, 0.0), 1.0)
    else:
        ob = _bc(outer, 1.0)
    bc = [_bc("diffuse", Tw), ob, _bc("periodic"), _bc("periodic")]
    T0 = 1.0 + 0.2 * mach * mach
    return dict(dim=2, geometry="annulus", nx=nth, ny=nr, r_in=r_in, r_out=r_out, q=q,
                lx=1.0, ly=1.0, kn=kn, omega=OMEGA_N2, alpha=1.0, dr=2, zrot=zrot,
                dt=dt_frac * TAU_C_PER_KN * kn, weight=area / n_target, bc=bc, seed=seed,
                instance=0, ppc=0, n_target=int(n_target),
                init=dict(rho=1.0, u=(0.0, 0.0, 0.0), Tt=1.0, Tr=1.0), tref=max(T0, Tw),
                name=f"cylinder_{nth}x{nr}_kn{kn}_ma{mach}")


def random_annulus_state(w, seed, density=1.0, drift=(0.0, 0.0, 0.0), T=1.0):
    """A random particle state of an annulus workload, listed cell by cell:
    Poisson counts of mean density x area / weight, positions uniform over each
    polar cell (r^2 uniform between its face radii, angle uniform), Maxwellian
    velocities about `drift`, exponential rotational energies.  Float32
    arrays plus the cell starts."""
    rng = np.random.default_rng(seed)
    nth, nr = w["nx"], w["ny"]
    q, ri, ro = w["q"], w["r_in"], w["r_out"]
    j = np.arange(nr + 1, dtype=np.float64)
    faces = ri + (ro - ri) * (j / nr if q == 1.0 else (q ** j - 1.0) / (q ** nr - 1.0))
    dth = 2.0 * math.pi / nth
    area = 0.5 * dth * (faces[1:] ** 2 - faces[:-1] ** 2)  # per radial ring
    lam = np.repeat(density * area / w["weight"], nth)     # cell c = i + nth j
    counts = rng.poisson(lam)
    start = np.zeros(len(counts) + 1, dtype=np.int64)
    start[1:] = np.cumsum(counts)
    n = int(start[-1])
    cell = np.repeat(np.arange(len(counts)), counts)
    ic, jc = cell % nth, cell // nth
    r = np.sqrt(faces[jc] ** 2 + rng.random(n) * (faces[jc + 1] ** 2 - faces[jc] ** 2))
    th = dth * (ic + rng.random(n))
    out = dict(x=(r * np.cos(th)).astype(np.float32), y=(r * np.sin(th)).astype(np.float32),
               vx=(drift[0] + math.sqrt(T) * rng.standard_normal(n)).astype(np.float32),
               vy=(drift[1] + math.sqrt(T) * rng.standard_normal(n)).astype(np.float32),
               vz=(drift[2] + math.sqrt(T) * rng.standard_normal(n)).astype(np.float32),
               er=(T * rng.exponential(size=n)).astype(np.float32),
               id=np.arange(n, dtype=np.uint32), start=start)
    return out
