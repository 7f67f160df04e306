"""FP64 oracle of the synthetic-equation solve (DIG step 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The synthetic equations are the steady conservation laws of mass, momentum and
total energy plus the rotational-energy relaxation equation (equation
macroscopic_equation, Section 2.3), closed by sigma = sigma_NSF + HoT_sigma,
q_t = q_t,NSF + HoT_qt, q_r = q_r,NSF + HoT_qr (equations full_constitutive,
ns_constitutive, kappa_A), with HoT set to zero where the adaptive mask is on
(Section 3.1).  The paper leaves the numerical scheme to other work; the
scheme below is this project's reading, written out plainly:

* unknowns per cell W = [rho, rho ux, rho uy, rho uz, rho E, rho e_r] with
  E = (3 Tt + d_r Tr)/2 + |u|^2/2 and e_r = d_r Tr / 2; pressure p = rho Tt;
* finite volumes on the grid of the workload (uniform, or graded: cells of
  different widths between per-axis face tables); inviscid face flux by HLLC (Toro) with
  Davis wave-speed estimates u_n -/+ c, c = sqrt(gamma Tt),
  gamma = (5 + d_r)/(3 + d_r); tangential velocity and rotational energy are
  carried by the contact wave, so a stationary contact gives no mass flux;
* viscous and heat fluxes at a face from the NSF relations with the face
  normal derivative (right - left)/d, d the distance between the two cell
  centres (h on a uniform grid), and the tangential derivative averaged
  from the two cells' central differences; mu = mu0 Tt^omega evaluated at the
  mean of the two cells' Tt, kappa from A; HoT at a face = mean of the two
  cells' (masked) HoT;
* walls: Dirichlet face state with zero normal velocity; tangential velocity
  and temperatures either the wall's own (mode "wall") or those of the
  wall-adjacent cell of the DSMC field M^{n+1/2} (mode "dsmc": slip and jump
  taken from DSMC); face density = adjacent cell density; derivatives at the
  wall face use the half cell (interior - wall)/(h/2);
* cell-centred derivatives: the difference of the two neighbours over the
  distance between their centres, one-sided at walls (exact for linear
  fields on any grid); the divergence of a cell divides the face-flux
  difference by its own width;
* rotational relaxation source (d_r rho / 2)(T - Tr)/(Z tau), tau = mu/p;
* explicit pseudo-time marching with one step for all cells (so that the
  total mass is conserved exactly): the minimum over cells of
  cfl / ( sum_axes (|u_a| + c)/h_a + 2 nu sum_axes 1/h_a^2 ) and 0.5 Z tau,
  nu = max(4 mu / (3 rho), gamma kappa_total / (rho c_v));
* stop after max_iter steps or when the largest change of (rho, u/sqrt(Tt),
  Tt, Tr), relative to rho, 1, Tt, Tr, falls below tol.
"""
from __future__ import annotations

import numpy as np


def _grid_params(w):
    nx, ny = w["nx"], (w.get("ny", 1) if w["dim"] == 2 else 1)
    hx = w["lx"] / nx
    hy = (w["ly"] / ny) if w["dim"] == 2 else 1.0
    return nx, ny, hx, hy


def _axis_geometry(w, axis, n, h):
    """(widths [n], gaps [n + 1]) of one axis: the cell widths, and for
    every face the distance between the centres on either side of it (a
    wall face: half the width of its cell; a periodic seam: the wrapped
    distance).  Uniform grids: h everywhere, h/2 at walls."""
    periodic = w["bc"][2 * axis][0] == "periodic"
    if w.get("geometry") == "graded" and (axis == 0 or w["dim"] == 2):
        f = np.asarray(w["xfaces"] if axis == 0 else w["yfaces"], dtype=np.float64)
        width = f[1:] - f[:-1]
        c = 0.5 * (f[1:] + f[:-1])
        gap = np.empty(n + 1)
        gap[1:-1] = c[1:] - c[:-1]
        if periodic:
            gap[0] = gap[-1] = c[0] + (f[-1] - c[-1])
        else:
            gap[0] = c[0] - f[0]
            gap[-1] = f[-1] - c[-1]
        return width, gap
    width = np.full(n, h)
    gap = np.full(n + 1, h)
    if not periodic:
        gap[0] = gap[-1] = 0.5 * h
    return width, gap


def _conductivities(mu, A, dr):
    att, atr, art, arr = A
    det = att * arr - atr * art
    kt = 0.5 * mu * (arr * 5.0 - atr * dr) / det
    kr = 0.5 * mu * (-art * 5.0 + att * dr) / det
    return kt, kr


def _prepare(w, m_half, hot, mask, A, wall_mode):
    """Grid, gas constants, masked higher-order terms, wall face states and the
    conservative start state W of a solve."""
    nx, ny, hx, hy = _grid_params(w)
    dr = w.get("dr", 2)
    om = w["omega"]
    if A is None:
        A = (2.0 / 3.0, 0.0, 0.0, 5.0 / (7.0 - 2.0 * om))
    two = w["dim"] == 2
    m = np.asarray(m_half, dtype=np.float64)
    rho0 = m[0].reshape(ny, nx)
    u0 = m[1:4].reshape(3, ny, nx)
    tt0 = m[4].reshape(ny, nx)
    tr0 = m[5].reshape(ny, nx)
    H = np.zeros((12, ny, nx))
    if hot is not None:
        H = np.asarray(hot, dtype=np.float64).reshape(12, ny, nx).copy()
        if mask is not None:
            H[:, np.asarray(mask).reshape(ny, nx) != 0] = 0.0
    # conservative state
    W = np.zeros((6, ny, nx))
    W[0] = rho0
    W[1:4] = rho0 * u0
    W[4] = rho0 * (0.5 * (3 * tt0 + dr * tr0) + 0.5 * (u0 ** 2).sum(axis=0))
    W[5] = rho0 * 0.5 * dr * tr0
    # wall face states: faces 0 (x-), 1 (x+), 2 (y-), 3 (y+)
    bct = [b[0] for b in w["bc"]]
    walls = {}
    for f in range(4 if two else 2):
        if bct[f] == "periodic":
            continue
        if f == 0:
            idx = (slice(None), 0)
        elif f == 1:
            idx = (slice(None), nx - 1)
        elif f == 2:
            idx = (0, slice(None))
        else:
            idx = (ny - 1, slice(None))
        if wall_mode == "wall":
            T = np.full(rho0[idx].shape, w["bc"][f][1])
            ut = [np.full(rho0[idx].shape, w["bc"][f][2][k]) for k in range(3)]
            walls[f] = dict(u=ut, tt=T, tr=T.copy())
        else:
            walls[f] = dict(u=[u0[k][idx].copy() for k in range(3)], tt=tt0[idx].copy(),
                            tr=tr0[idx].copy())
        axis = f // 2
        walls[f]["u"][axis] = np.zeros_like(walls[f]["u"][axis])
    wx, gx = _axis_geometry(w, 0, nx, hx)
    if two:
        wy, gy = _axis_geometry(w, 1, ny, hy)
    else:
        wy, gy = np.ones(1), np.ones(2)
    # widths broadcast over cell arrays [..., ny, nx], gaps over face arrays;
    # vol: cell volumes (areas in 2D, lengths in 1D)
    vol = np.outer(wy, wx) if two else wx[None, :]
    return dict(nx=nx, ny=ny, hx=hx, hy=hy, width={0: wx, 1: wy[:, None]}, vol=vol,
                gap={0: gx, 1: gy[:, None]}, dr=dr, om=om, A=A, two=two, H=H, W=W,
                bct=bct, walls=walls, mu0=w["kn"] * np.sqrt(2.0 / np.pi), Z=w["zrot"],
                gam=(5.0 + dr) / (3.0 + dr), cv=(3.0 + dr) / 2.0)


def _prims(W, dr):
    rho = W[0]
    u = W[1:4] / rho
    tr = 2.0 * W[5] / (dr * rho)
    tt = (W[4] / rho - 0.5 * (u ** 2).sum(axis=0) - 0.5 * dr * tr) * 2.0 / 3.0
    return rho, u, tt, tr


def _dcen(P, f, axis):
    """Cell-centred derivative along `axis`: central inside, one-sided at
    walls, wrapped across periodic faces (used for tangential face terms)."""
    out = np.zeros_like(f)
    if axis == 1 and not P["two"]:
        return out
    n = f.shape[1] if axis == 0 else f.shape[0]
    g = P["gap"][axis].ravel()          # [n + 1]: centre distances across faces
    span = g[:-1] + g[1:]               # [n]: distance between the two neighbours
    per = P["bct"][2 * axis] == "periodic"
    if axis == 0:
        if per:
            out[:] = (np.roll(f, -1, 1) - np.roll(f, 1, 1)) / span
        elif n > 1:
            out[:, 1:-1] = (f[:, 2:] - f[:, :-2]) / span[1:-1]
            out[:, 0] = (f[:, 1] - f[:, 0]) / g[1]
            out[:, -1] = (f[:, -1] - f[:, -2]) / g[n - 1]
    else:
        if per:
            out[:] = (np.roll(f, -1, 0) - np.roll(f, 1, 0)) / span[:, None]
        elif n > 1:
            out[1:-1] = (f[2:] - f[:-2]) / span[1:-1, None]
            out[0] = (f[1] - f[0]) / g[1]
            out[-1] = (f[-1] - f[-2]) / g[n - 1]
    return out


def _axis_fluxes(P, W, axis):
    """Total face fluxes normal to `axis` of state W (see _face_fluxes)."""
    rho, u, tt, tr = _prims(W, P["dr"])
    mu = P["mu0"] * tt ** P["om"]
    du = [[_dcen(P, u[i], a) for a in range(2)] for i in range(3)]
    return _face_fluxes(axis, W, rho, u, tt, tr, mu, du, P["H"], P["walls"], P["bct"],
                        P["gap"][axis], P["two"], P["dr"], P["gam"], P["mu0"], P["om"],
                        P["A"], P["nx"], P["ny"])


def _residual(P, W):
    """R = -(sum of face-flux differences)/h + rotational relaxation source,
    and the explicit stability bound inv_dt of every cell.  Also returns the
    primitive state and the relaxation time."""
    rho, u, tt, tr = _prims(W, P["dr"])
    dr, gam, two = P["dr"], P["gam"], P["two"]
    mu = P["mu0"] * tt ** P["om"]
    kt_c, kr_c = _conductivities(mu, P["A"], dr)
    du = [[_dcen(P, u[i], a) for a in range(2)] for i in range(3)]
    R = np.zeros_like(W)
    inv_dt = np.zeros((P["ny"], P["nx"]))
    c = np.sqrt(gam * tt)
    ktot = kt_c + kr_c
    nu = np.maximum(4.0 * mu / (3.0 * rho), gam * ktot / (rho * P["cv"]))
    for axis in range(2 if two else 1):
        h = P["width"][axis]
        inv_dt += (np.abs(u[axis]) + c) / h + 2.0 * nu / h ** 2
        F = _face_fluxes(axis, W, rho, u, tt, tr, mu, du, P["H"], P["walls"], P["bct"],
                         P["gap"][axis], two, dr, gam, P["mu0"], P["om"], P["A"], P["nx"],
                         P["ny"])
        # F has shape (6, ny, nx+1) for axis 0 or (6, ny+1, nx) for axis 1
        if axis == 0:
            R -= (F[:, :, 1:] - F[:, :, :-1]) / h
        else:
            R -= (F[:, 1:, :] - F[:, :-1, :]) / h
    tau = mu / (rho * tt)
    T = (3.0 * tt + dr * tr) / (3.0 + dr)
    R[5] += 0.5 * dr * rho * (T - tr) / (P["Z"] * tau)
    return R, inv_dt, (rho, u, tt, tr), tau


def _relative_change(old, new):
    rho, u, tt, tr = old
    rn, un, ttn, trn = new
    ch = np.max(np.abs(rn - rho) / rho)
    ch = max(ch, np.max(np.abs(un - u) / np.sqrt(tt)))
    ch = max(ch, np.max(np.abs(ttn - tt) / tt))
    ch = max(ch, np.max(np.abs(trn - tr) / np.maximum(tr, 1e-300)))
    return ch


def _output(P, W):
    rho, u, tt, tr = _prims(W, P["dr"])
    C = P["nx"] * P["ny"]
    out = np.zeros((6, C))
    out[0] = rho.ravel()
    out[1:4] = u.reshape(3, C)
    out[4] = tt.ravel()
    out[5] = tr.ravel()
    return out


def solve(w, m_half, hot=None, mask=None, A=None, max_iter=2000, tol=1e-5, cfl=0.5,
          wall_mode="dsmc"):
    """Explicit pseudo-time marching.  Returns (m_next [6, C], iterations,
    last relative change)."""
    P = _prepare(w, m_half, hot, mask, A, wall_mode)
    W = P["W"]
    it = 0
    change = np.inf
    for it in range(1, max_iter + 1):
        R, inv_dt, prim, tau = _residual(P, W)
        dtau = min(np.min(cfl / inv_dt), np.min(0.5 * P["Z"] * tau))
        Wn = W + dtau * R
        ch = _relative_change(prim, _prims(Wn, P["dr"]))
        W = Wn
        change = ch
        if ch < tol:
            break
    return _output(P, W), it, change


def _euler_flux(W, axis, dr):
    """Inviscid flux of the conservative state W along `axis` (cell values)."""
    rho, u, tt, tr = _prims(W, dr)
    p = rho * tt
    un = u[axis]
    F = np.empty_like(W)
    F[0] = W[0] * un
    for k in range(3):
        F[1 + k] = W[1 + k] * un + (p if k == axis else 0.0)
    F[4] = (W[4] + p) * un
    F[5] = W[5] * un
    return F


def _neighbour(a, axis, side, periodic):
    """Values of the neighbour on `side` (+1 or -1) along `axis` of every cell
    (cell arrays [..., ny, nx]); zero where that neighbour is a wall."""
    ax = -1 if axis == 0 else -2
    out = np.roll(a, -side, axis=ax)
    if not periodic:
        idx = [slice(None)] * a.ndim
        idx[ax] = -1 if side > 0 else 0
        out[tuple(idx)] = 0.0
    return out


def solve_lusgs(w, m_half, hot=None, mask=None, A=None, max_iter=500, tol=1e-5, cfl=1e6,
                wall_mode="dsmc"):
    """Implicit pseudo-time solve of the same discrete steady equations as
    `solve` (same residual R), by LU-SGS: one symmetric Gauss-Seidel sweep
    pair per iteration on the approximately factored implicit operator, in
    matrix-free form (Yoon and Jameson).

    Per cell i, with r_a = |u_a| + c + 2 nu / h_a the spectral radius along
    axis a (nu as in `solve`) and j running over the neighbours across
    interior or periodic faces (n_ij the unit normal from i to j):

      D_i dW_i + sum_j (dF_j . n_ij - r_j dW_j) / (2 h) = R_i,
      D_i = (1 + 1/cfl) sum_a r_a / h_a   (+ 1/(Z tau) on the rotational row),

    where dF_j = F(W_j + dW_j) - F(W_j) is the change of the inviscid flux of
    the neighbour.  The cells are ordered in two colours, (i + j) even first
    (a red-black ordering; every neighbour of a cell has the other colour):
    the lower sweep gives dW* = R / D on the first colour, then
    dW* = (R - sum_j (dF*_j . n_ij - r_j dW*_j) / (2h)) / D on the second;
    the upper sweep keeps dW = dW* on the second colour and sets
    dW = dW* - sum_j (dF_j . n_ij - r_j dW_j) / (2h D) on the first.
    Here h is the width of the receiving cell i along the axis.  After the
    update, every conservative variable is scaled by the ratio of the initial
    to the current total mass, sum of rho V (the implicit operator is not
    conservative; the box is closed or periodic, so the steady state keeps
    the initial mass).  Stops as `solve` does.  Periodic axes need an even
    cell count (two colours).  Returns (m_next [6, C], iterations, change)."""
    P = _prepare(w, m_half, hot, mask, A, wall_mode)
    W = P["W"]
    nx, ny, two, dr = P["nx"], P["ny"], P["two"], P["dr"]
    axes = (0, 1) if two else (0,)
    per = {a: P["bct"][2 * a] == "periodic" for a in axes}
    for a in axes:
        if per[a] and (nx if a == 0 else ny) % 2:
            raise ValueError("periodic axes need an even cell count")
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    first = ((ii + jj) % 2 == 0)          # first colour
    vol = P["vol"]
    mass0 = (W[0] * vol).sum()
    it = 0
    change = np.inf
    for it in range(1, max_iter + 1):
        R, inv_dt, prim, tau = _residual(P, W)
        rho, u, tt, tr = prim
        mu = P["mu0"] * tt ** P["om"]
        kt_c, kr_c = _conductivities(mu, P["A"], dr)
        c = np.sqrt(P["gam"] * tt)
        nu = np.maximum(4.0 * mu / (3.0 * rho), P["gam"] * (kt_c + kr_c) / (rho * P["cv"]))
        h = P["width"]
        r = {a: np.abs(u[a]) + c + 2.0 * nu / h[a] for a in axes}
        D = np.zeros_like(W)
        for a in axes:
            D += (1.0 + 1.0 / cfl) * r[a] / h[a]
        D[5] += 1.0 / (P["Z"] * tau)
        F = {a: _euler_flux(W, a, dr) for a in axes}

        def offdiag(dW):
            """sum_j (dF_j . n_ij - r_j dW_j) / (2 h) of every cell from the
            neighbours' increments dW (zero where not yet known)."""
            out = np.zeros_like(W)
            for a in axes:
                dF = _euler_flux(W + dW, a, dr) - F[a]
                for side in (1, -1):
                    t = side * dF - r[a] * dW
                    out += _neighbour(t, a, side, per[a]) / (2.0 * h[a])
            return out

        dW = np.zeros_like(W)
        # lower sweep: first colour, then second
        dW[:, first] = R[:, first] / D[:, first]
        rhs = R - offdiag(np.where(first, dW, 0.0))
        dW[:, ~first] = rhs[:, ~first] / D[:, ~first]
        # upper sweep: second colour unchanged, then first
        corr = offdiag(np.where(first, 0.0, dW))
        dW[:, first] = dW[:, first] - corr[:, first] / D[:, first]
        Wn = W + dW
        Wn = Wn * (mass0 / (Wn[0] * vol).sum())
        ch = _relative_change(prim, _prims(Wn, dr))
        W = Wn
        change = ch
        if ch < tol:
            break
    return _output(P, W), it, change


def face_fluxes(w, fields, axis, hot=None, A=None, wall_mode="wall"):
    """Total flux (inviscid HLLC + NSF viscous and heat + masked higher-order
    terms) through every face normal to `axis` for the primitive fields
    [rho, ux, uy, uz, Tt, Tr] (first six rows of `fields`), the arithmetic of
    one pseudo-time step.  Shape (6, ny, nx+1) for axis 0, (6, ny+1, nx) for
    axis 1; rows mass, momentum x y z, total energy, rotational energy."""
    P = _prepare(w, fields, hot, None, A, wall_mode)
    return _axis_fluxes(P, P["W"], axis)


def _face_fluxes(axis, W, rho, u, tt, tr, mu, du, H, walls, bct, gap, two, dr, gam, mu0, om, A,
                 nx, ny):
    """Total (inviscid + viscous + heat) flux through the faces normal to axis;
    gap: the centre distance across every face (half a cell at a wall)."""
    # left/right states on every face; boundary faces filled below
    if axis == 0:
        nf = (ny, nx + 1)
        L = lambda a: np.concatenate([a[..., -1:], a], axis=-1)   # left neighbour of face i
        Rr = lambda a: np.concatenate([a, a[..., :1]], axis=-1)   # right neighbour of face i
    else:
        nf = (ny + 1, nx)
        L = lambda a: np.concatenate([a[..., -1:, :], a], axis=-2)
        Rr = lambda a: np.concatenate([a, a[..., :1, :]], axis=-2)
    rl, rr = L(rho), Rr(rho)
    ul, ur = L(u), Rr(u)
    tl, tR = L(tt), Rr(tt)
    trl, trr = L(tr), Rr(tr)
    Wl, Wr = L(W), Rr(W)
    Hl, Hr = L(H), Rr(H)
    dul = [[L(du[i][a]) for a in range(2)] for i in range(3)]
    dur = [[Rr(du[i][a]) for a in range(2)] for i in range(3)]
    periodic = bct[2 * axis] == "periodic"
    # ---------------- inviscid (HLLC) on interior / periodic faces
    def euler(Wc, rc, uc, tc):
        p = rc * tc
        un = uc[axis]
        F = np.empty_like(Wc)
        F[0] = Wc[0] * un
        for k in range(3):
            F[1 + k] = Wc[1 + k] * un + (p if k == axis else 0.0)
        F[4] = (Wc[4] + p) * un
        F[5] = Wc[5] * un
        return F

    def star(Wc, rc, uc, pc, SK, Ss):
        f = rc * (SK - uc[axis]) / (SK - Ss)
        U = np.empty_like(Wc)
        U[0] = f
        for k in range(3):
            U[1 + k] = f * (Ss if k == axis else uc[k])
        U[4] = f * (Wc[4] / rc + (Ss - uc[axis]) * (Ss + pc / (rc * (SK - uc[axis]))))
        U[5] = f * Wc[5] / rc
        return U

    Fl, Fr = euler(Wl, rl, ul, tl), euler(Wr, rr, ur, tR)
    pl, pr = rl * tl, rr * tR
    cl, cr = np.sqrt(gam * tl), np.sqrt(gam * tR)
    SL = np.minimum(ul[axis] - cl, ur[axis] - cr)
    SR = np.maximum(ul[axis] + cl, ur[axis] + cr)
    Ss = (pr - pl + rl * ul[axis] * (SL - ul[axis]) - rr * ur[axis] * (SR - ur[axis])) / \
        (rl * (SL - ul[axis]) - rr * (SR - ur[axis]))
    FsL = Fl + SL * (star(Wl, rl, ul, pl, SL, Ss) - Wl)
    FsR = Fr + SR * (star(Wr, rr, ur, pr, SR, Ss) - Wr)
    F = np.where(SL >= 0, Fl, np.where(Ss >= 0, FsL, np.where(SR > 0, FsR, Fr)))
    # ---------------- viscous / heat on interior / periodic faces
    tf = 0.5 * (tl + tR)
    uf = 0.5 * (ul + ur)
    dn = [(ur[i] - ul[i]) / gap for i in range(3)]               # d u_i / d x_axis
    dt_ = [0.5 * (dul[i][1 - axis] + dur[i][1 - axis]) for i in range(3)] if two else \
        [np.zeros(nf)] * 3                                        # d u_i / d x_other
    dTt = (tR - tl) / gap
    dTr = (trr - trl) / gap
    Hf = 0.5 * (Hl + Hr)
    V = _visc(axis, tf, uf, dn, dt_, dTt, dTr, Hf, mu0, om, A, dr, two)
    F = F + V
    # ---------------- boundary faces: walls
    if not periodic:
        for side, f in ((0, 2 * axis), (1, 2 * axis + 1)):
            wl = walls[f]
            if axis == 0:
                fi = 0 if side == 0 else nx
                ci = 0 if side == 0 else nx - 1
                cell = lambda a: a[..., :, ci]
                sl = (slice(None), slice(None), fi)
                half = gap[fi]
            else:
                fi = 0 if side == 0 else ny
                ci = 0 if side == 0 else ny - 1
                cell = lambda a: a[..., ci, :]
                sl = (slice(None), fi, slice(None))
                half = gap[fi, 0]
            sgn = 1.0 if side == 0 else -1.0      # (interior - wall) / (h/2) * sgn = d/dx
            rc, uc, tc, trc = cell(rho), cell(u), cell(tt), cell(tr)
            Fw = np.zeros((6,) + rc.shape)
            Fw[1 + axis] = rc * tc                 # pressure on the wall
            uw = np.array(wl["u"])
            tfw = 0.5 * (tc + wl["tt"])
            dnw = [sgn * (uc[i] - uw[i]) / half for i in range(3)]
            dtw = [cell(du[i][1 - axis]) for i in range(3)] if two else \
                [np.zeros(rc.shape)] * 3
            dTtw = sgn * (tc - wl["tt"]) / half
            dTrw = sgn * (trc - wl["tr"]) / half
            Hw = cell(H)
            Vw = _visc(axis, tfw, uw, dnw, dtw, dTtw, dTrw, Hw, mu0, om, A, dr, two)
            Fw = Fw + Vw
            Fw[0] = 0.0
            F[sl] = Fw
    return F


def _visc(axis, tf, uf, dn, dt_, dTt, dTr, Hf, mu0, om, A, dr, two):
    """NSF + HoT stress and heat flux through a face normal to `axis`."""
    mu = mu0 * tf ** om
    kt, kr = _conductivities(mu, A, dr)
    # velocity-gradient tensor entries g[i][j] = d u_i / d x_j
    g = [[None] * 3 for _ in range(3)]
    other = 1 - axis
    for i in range(3):
        g[i][axis] = dn[i]
        g[i][other] = dt_[i]
        g[i][2] = np.zeros_like(dn[i])
    div = g[0][0] + g[1][1]
    # sigma_{axis, j}
    hidx = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3, (0, 2): 4, (2, 0): 4,
            (1, 2): 5, (2, 1): 5}
    sig = []
    for j in range(3):
        s = -mu * (g[axis][j] + g[j][axis] - (2.0 / 3.0 * div if j == axis else 0.0))
        sig.append(s + Hf[hidx[(axis, j)]])
    qt = -kt * dTt + Hf[6 + axis]
    qr = -kr * dTr + Hf[9 + axis]
    V = np.zeros((6,) + np.shape(dn[0]))
    for j in range(3):
        V[1 + j] = sig[j]
    V[4] = sig[0] * uf[0] + sig[1] * uf[1] + sig[2] * uf[2] + qt + qr
    V[5] = qr
    return V
