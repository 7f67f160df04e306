"""Oracle pin: Fourier heat conduction in the small-Kn limit (1D plates).

With kappa proportional to mu ~ T^omega, steady Fourier conduction makes the
energy flux uniform and T^(1+omega) linear in x, with slope
-(1 + omega) q / kappa0.  In the monatomic limit (no inelastic collisions) the
first Chapman-Enskog approximation gives kappa_t = (15/4) mu.  The polyatomic
conductivity of the Borgnakke-Larsen model is a property of the model that the
paper says cannot be tuned to a chosen A (Section 2.2); it is reported, not
pinned.
"""
import numpy as np

import dig_workloads as wl
import oracle


def _run(zrot, seed, ppc=100, steps=7000, dt_frac=0.1):
    w = wl.fourier_1d(seed=seed, ppc=ppc, zrot=zrot)
    w["dt"] = dt_frac * wl.TAU_C_PER_KN * w["kn"]
    s = oracle.new_state(w)
    for k in range(steps):
        if k == steps // 5:
            s.reset_average()
        s.step()
    return w, s.fields()


def _kappa(w, f, T, q, lo=0.25, hi=0.75):
    nx = w["nx"]
    xc = (np.arange(nx) + 0.5) / nx
    b = slice(int(lo * nx), int(hi * nx))
    om = w["omega"]
    slope, icpt = np.polyfit(xc[b], T[b] ** (1 + om), 1)
    kappa0 = -q[b].mean() * (1 + om) / slope
    resid = T[b] ** (1 + om) - (slope * xc[b] + icpt)
    return kappa0 / oracle.mu0(w), resid, q[b]


def test_fourier_monatomic_limit_conductivity():
    w, f = _run(zrot=1e30, seed=1101)
    k, resid, q = _kappa(w, f, f[4], f[12])
    assert abs(k / 3.75 - 1.0) < 0.06, k
    # linear T^(1+w) in the bulk: residual at the noise level of the profile
    assert np.abs(resid).max() < 0.03
    # uniform energy flux: four bulk blocks agree
    blocks = np.array([b.mean() for b in np.array_split(q, 4)])
    assert np.abs(blocks / q.mean() - 1.0).max() < 0.1


def test_fourier_polyatomic_energy_flux_uniform():
    w, f = _run(zrot=5.0, seed=1102, steps=5000)
    qt = f[12] + f[15]
    k, resid, q = _kappa(w, f, f[18], qt)
    blocks = np.array([b.mean() for b in np.array_split(q, 4)])
    assert np.abs(blocks / q.mean() - 1.0).max() < 0.1
    # heat flows from the hot plate (x = 1) to the cold one
    assert q.mean() < 0
    # total conductivity of the BL model: between the translational-only and
    # the modified-Eucken estimate (15/4 + (7 - 2 w)/5 = 4.854)
    assert 3.75 < k < 5.1, k
