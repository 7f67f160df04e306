"""FP64 oracle of the learned-closure plumbing: the network's inputs and
targets computed from time-averaged fields, and the three-band blend of
network and DSMC-extracted higher-order terms (Section 3.1, with the learned
band between Kn_lo and Kn_hi).

TEST INFRASTRUCTURE ONLY: only the test suite may import this module.

Field layout [20][C]: rho, ux, uy, uz, Tt, Tr, sigma (xx, yy, zz, xy, xz, yz),
q_t (x, y, z), q_r (x, y, z), T, N.  HoT layout [12][C]: sigma (xx, yy, zz,
xy, xz, yz), q_t (x, y, z), q_r (x, y, z).
"""
from __future__ import annotations

import math

import numpy as np

HOT_OF_TARGET = [0, 3, 1, 6, 7, 9, 10]  # sigma_xx, sigma_xy, sigma_yy, qt_x, qt_y, qr_x, qr_y


def _centres(w, axis):
    """Cell-centre coordinates along `axis` (uniform or graded grid) and the
    axis length."""
    n = w["nx"] if axis == 0 else w["ny"]
    L = w["lx"] if axis == 0 else w["ly"]
    if w.get("geometry") == "graded":
        f = np.asarray(w["xfaces"] if axis == 0 else w["yfaces"], dtype=np.float64)
        return 0.5 * (f[1:] + f[:-1]), L
    return (np.arange(n) + 0.5) * (L / n), L


def gradient(w, f, axis):
    """d f / d x_axis: the difference of the two neighbours over the distance
    between their centres inside, one-sided at wall faces, wrapped at periodic
    faces (the wrapped distance); zero along y in 1D.  On a uniform grid the
    distances are 2h and h."""
    nx = w["nx"]
    ny = w.get("ny", 1) if w["dim"] == 2 else 1
    if axis == 1 and w["dim"] == 1:
        return np.zeros_like(f)
    g = f.reshape(ny, nx)
    graded = w.get("geometry") == "graded"
    h = (w["lx"] / nx) if axis == 0 else (w["ly"] / ny)
    xc, L = _centres(w, axis)
    n = nx if axis == 0 else ny

    def gap(a, b):  # centre distance from cell a to cell b = a + 1 (mod n)
        if not graded:
            return h
        return xc[b] - xc[a] + (L if b < a else 0.0)
    out = np.zeros_like(g)
    if n < 2:
        return out.reshape(-1)
    ax = 1 if axis == 0 else 0
    periodic = w["bc"][2 * axis][0] == "periodic"
    for i in range(n):
        sl = [slice(None), slice(None)]

        def at(k):
            s2 = list(sl)
            s2[ax] = k
            return g[tuple(s2)]

        if 0 < i < n - 1:
            d = (at(i + 1) - at(i - 1)) / (gap(i - 1, i) + gap(i, i + 1))
        elif periodic:
            ip, im = (i + 1) % n, (i - 1) % n
            d = (at(ip) - at(im)) / (gap(im, i) + gap(i, ip))
        elif i == 0:
            d = (at(1) - at(0)) / gap(0, 1)
        else:
            d = (at(n - 1) - at(n - 2)) / gap(n - 2, n - 1)
        s3 = list(sl)
        s3[ax] = i
        out[tuple(s3)] = d
    return out.reshape(-1)


def features(w, F, kn, scaling, hot=None):
    """Standardised inputs [C, 9] and (with hot) targets [C, 7]."""
    C = F.shape[1]
    rho, tt = F[0], F[4]
    ok = (rho > 0) & (tt > 0) & np.isfinite(kn)
    mu0 = w["kn"] * math.sqrt(2.0 / math.pi)
    with np.errstate(divide="ignore", invalid="ignore"):
        mu = mu0 * np.power(np.where(ok, tt, 1.0), w["omega"])
        lam = mu / (rho * tt) * np.sqrt(math.pi * tt / 2.0)
        su, st = lam / np.sqrt(tt), lam / tt
        f = np.zeros((C, 9))
        f[:, 0] = su * gradient(w, F[1], 0)
        f[:, 1] = su * gradient(w, F[1], 1)
        f[:, 2] = su * gradient(w, F[2], 0)
        f[:, 3] = su * gradient(w, F[2], 1)
        f[:, 4] = st * gradient(w, F[4], 0)
        f[:, 5] = st * gradient(w, F[4], 1)
        f[:, 6] = st * gradient(w, F[5], 0)
        f[:, 7] = st * gradient(w, F[5], 1)
        f[:, 8] = kn
        y = np.zeros((C, 7))
        if hot is not None:
            p = rho * tt
            pq = p * np.sqrt(tt)
            for j, hk in enumerate(HOT_OF_TARGET):
                y[:, j] = hot[hk] / (p if j < 3 else pq)
    f = (f - np.asarray(scaling["x_mean"])) / np.asarray(scaling["x_std"])
    y = (y - np.asarray(scaling["y_mean"])) / np.asarray(scaling["y_std"])
    f[~ok] = 0.0
    y[~ok] = 0.0
    return f, (y if hot is not None else None)


# Per-particle standard deviations of the scaled DSMC-extracted terms of an
# equilibrium cell (Maxwellian velocities, exponential rotational energy),
# the peculiar velocity c taken about the cell's sample mean: sigma_xx/p and
# sigma_yy/p from (2/3) c_x^2 - (c_y^2 + c_z^2)/3 (variance 4/3 T^2),
# sigma_xy/p from c_x c_y (variance T^2); q_t/(p sqrt(T)) from
# c_x |c|^2 / 2, which to first order is v_x |v|^2 / 2 - (5/2) T v_x
# (variance 35/4 - 25/2 + 25/4 = 5/2, in T^3); q_r/(p sqrt(T)) from c_x er,
# to first order v_x er - T v_x (variance 2 - 2 + 1 = 1, in T^3).
DIRECT_SD = [math.sqrt(4.0 / 3.0), 1.0, math.sqrt(4.0 / 3.0), math.sqrt(2.5),
             math.sqrt(2.5), 1.0, 1.0]


def judge_se(w, F, A, judge_steps):
    """Standard error [C, 7] of the DSMC-extracted higher-order terms of the
    time-averaged field F (target order, scaled by p or p sqrt(Tt)) from the
    sampling noise of M = N x judge_steps independent particle samples per
    cell (N the mean particle count, row 19): the direct moment sum
    (DIRECT_SD / sqrt(M)) and the NSF terms subtracted from it, whose central
    differences over 2h carry the noise of the mean velocity (variance Tt/M),
    Tt (2 Tt^2 / (3 M)) and Tr (Tr^2 / M) of the two neighbours.  On a graded
    grid h is the cell's own width along each axis (the neighbours' distance
    is about twice that)."""
    C = F.shape[1]
    rho, tt, tr, N = F[0], F[4], F[5], F[19]
    two = w["dim"] == 2
    nx, ny = w["nx"], (w["ny"] if two else 1)
    if w.get("geometry") == "graded":
        wx = np.diff(np.asarray(w["xfaces"], dtype=np.float64))
        wy = np.diff(np.asarray(w["yfaces"], dtype=np.float64)) if two else np.ones(1)
    else:
        wx = np.full(nx, w["lx"] / nx)
        wy = np.full(ny, w["ly"] / ny) if two else np.ones(1)
    ihx2_c = np.tile(1.0 / (2.0 * wx * wx), ny)
    ihy2_c = np.repeat(1.0 / (2.0 * wy * wy), nx) if two else np.zeros(C)
    mu0 = w["kn"] * math.sqrt(2.0 / math.pi)
    att, atr, art, arr = A
    det = att * arr - atr * art
    dr = w.get("dr", 2)
    se = np.full((C, 7), np.inf)
    for c in range(C):
        if not (rho[c] > 0 and tt[c] > 0 and N[c] > 0):
            continue
        M = N[c] * judge_steps
        ihx2, ihy2 = ihx2_c[c], ihy2_c[c]
        mu = mu0 * tt[c] ** w["omega"]
        kt = 0.5 * mu * (arr * 5.0 - atr * dr) / det
        kr = 0.5 * mu * (-art * 5.0 + att * dr) / det
        p = rho[c] * tt[c]
        pq = p * math.sqrt(tt[c])
        vu, vt, vr = tt[c] / M, 2.0 * tt[c] ** 2 / (3.0 * M), tr[c] ** 2 / M
        nsf = [mu * mu * vu * (16.0 / 9.0 * ihx2 + 4.0 / 9.0 * ihy2) / (p * p),
               mu * mu * vu * (ihx2 + ihy2) / (p * p),
               mu * mu * vu * (16.0 / 9.0 * ihy2 + 4.0 / 9.0 * ihx2) / (p * p),
               kt * kt * vt * ihx2 / (pq * pq), kt * kt * vt * ihy2 / (pq * pq),
               kr * kr * vr * ihx2 / (pq * pq), kr * kr * vr * ihy2 / (pq * pq)]
        for j in range(7):
            se[c, j] = math.sqrt(DIRECT_SD[j] ** 2 / M + nsf[j])
    return se


def blend(w, F, kn, mask, ypred, scaling, A, hot, kn_lo, kn_hi, judge_sigma, judge_rel,
          judge_steps):
    """Returns (new hot [12, C], source code [C]): 0 NSF, 1 DSMC, 2 network,
    3 network rejected by the judge.  Inside the band a prediction is rejected
    when, in some component, |network - DSMC| (scaled) exceeds judge_sigma
    standard errors of the DSMC term (judge_se) plus judge_rel |DSMC|."""
    hot = hot.copy()
    C = F.shape[1]
    se = judge_se(w, F, A, judge_steps)
    src = np.where(mask != 0, 0, 1).astype(np.uint8)
    for c in range(C):
        rho, tt = F[0, c], F[4, c]
        if mask[c] or not (rho > 0 and tt > 0) or not (kn_lo <= kn[c] < kn_hi):
            continue
        p = rho * tt
        pq = p * math.sqrt(tt)
        pr = np.empty(7)
        ok = True
        for j, hk in enumerate(HOT_OF_TARGET):
            s = p if j < 3 else pq
            pr[j] = (ypred[c, j] * scaling["y_std"][j] + scaling["y_mean"][j]) * s
            ds = hot[hk, c]
            if abs(pr[j] - ds) / s > judge_sigma * se[c, j] + judge_rel * abs(ds) / s:
                ok = False
        if not ok:
            src[c] = 3
            continue
        new = np.zeros(12)
        new[0], new[3], new[1] = pr[0], pr[1], pr[2]
        new[2] = -(pr[0] + pr[2])
        new[6], new[7], new[9], new[10] = pr[3], pr[4], pr[5], pr[6]
        hot[:, c] = new
        src[c] = 2
    return hot, src
