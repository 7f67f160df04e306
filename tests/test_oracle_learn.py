"""Pins of the learned-closure plumbing oracle: linear fields give exact
gradients, so the network inputs have closed forms; targets scale HoT by p and
p sqrt(Tt); the blend follows its three bands and the judge."""
import math

import numpy as np

import dig_workloads as wl
from oracle import learn

UNIT = {"x_mean": np.zeros(9), "x_std": np.ones(9), "y_mean": np.zeros(7), "y_std": np.ones(7)}


def _linear_fields(w, a=0.3, b=-0.2, c=0.1, d=0.05, gt=(0.2, -0.1), gr=(0.05, 0.15)):
    nx, ny = w["nx"], w["ny"]
    xs = (np.arange(nx) + 0.5) * w["lx"] / nx
    ys = (np.arange(ny) + 0.5) * w["ly"] / ny
    X, Y = np.meshgrid(xs, ys)
    F = np.zeros((20, nx * ny))
    F[0] = 1.0
    F[1] = (a * X + b * Y).reshape(-1)
    F[2] = (c * X + d * Y).reshape(-1)
    F[4] = (1.0 + gt[0] * X + gt[1] * Y).reshape(-1)
    F[5] = (1.0 + gr[0] * X + gr[1] * Y).reshape(-1)
    return F


def test_features_of_linear_fields_closed_form():
    w = wl.cavity_2d(n=12, kn=0.05)
    F = _linear_fields(w)
    kn = np.full(144, 0.07)
    hot = np.random.default_rng(1).standard_normal((12, 144)) * 0.01
    f, y = learn.features(w, F, kn, UNIT, hot)
    tt = F[4]
    mu = 0.05 * math.sqrt(2 / math.pi) * tt ** w["omega"]
    lam = mu / tt * np.sqrt(math.pi * tt / 2)
    np.testing.assert_allclose(f[:, 0], lam / np.sqrt(tt) * 0.3, rtol=1e-10)
    np.testing.assert_allclose(f[:, 1], lam / np.sqrt(tt) * -0.2, rtol=1e-10)
    np.testing.assert_allclose(f[:, 2], lam / np.sqrt(tt) * 0.1, rtol=1e-10)
    np.testing.assert_allclose(f[:, 3], lam / np.sqrt(tt) * 0.05, rtol=1e-10)
    np.testing.assert_allclose(f[:, 4], lam / tt * 0.2, rtol=1e-10)
    np.testing.assert_allclose(f[:, 5], lam / tt * -0.1, rtol=1e-10)
    np.testing.assert_allclose(f[:, 6], lam / tt * 0.05, rtol=1e-10)
    np.testing.assert_allclose(f[:, 7], lam / tt * 0.15, rtol=1e-10)
    np.testing.assert_array_equal(f[:, 8], kn)
    p = tt
    np.testing.assert_allclose(y[:, 0], hot[0] / p, rtol=1e-14)
    np.testing.assert_allclose(y[:, 1], hot[3] / p, rtol=1e-14)
    np.testing.assert_allclose(y[:, 2], hot[1] / p, rtol=1e-14)
    np.testing.assert_allclose(y[:, 6], hot[10] / (p * np.sqrt(tt)), rtol=1e-14)
    # standardisation
    sc = {"x_mean": np.arange(9.0), "x_std": np.full(9, 2.0), "y_mean": np.ones(7),
          "y_std": np.full(7, 4.0)}
    f2, y2 = learn.features(w, F, kn, sc, hot)
    np.testing.assert_allclose(f2, (f - np.arange(9.0)) / 2.0, rtol=1e-14)
    np.testing.assert_allclose(y2, (y - 1.0) / 4.0, rtol=1e-14)


def test_periodic_gradient_wraps_and_1d_has_no_y():
    w = wl.fourier_1d(nx=8)
    w["bc"] = [("periodic", 1, (0, 0, 0))] * 4
    f = np.sin(2 * np.pi * (np.arange(8) + 0.5) / 8)
    g = learn.gradient(w, f, 0)
    h = 1 / 8
    assert abs(g[0] - (f[1] - f[7]) / (2 * h)) < 1e-14
    assert np.all(learn.gradient(w, f, 1) == 0)


def test_blend_bands_and_judge():
    C = 6
    F = np.zeros((20, C))
    F[0] = 1.0
    F[4] = 1.0
    kn = np.array([0.005, 0.03, 0.07, 0.07, 0.2, np.inf])
    mask = (kn < 0.01).astype(np.uint8)
    hot = np.zeros((12, C))
    hot[0] = 0.01
    hot[3] = -0.02
    ypred = np.zeros((C, 7))
    ypred[:, 0] = 0.012
    ypred[:, 1] = -0.018
    ypred[3, 1] = 0.5  # far from DSMC: rejected
    new, src = learn.blend(F, kn, mask, ypred, UNIT, hot, 0.05, 0.1, 0.05, 0.1)
    np.testing.assert_array_equal(src, [0, 1, 2, 3, 1, 1])
    assert new[0, 2] == 0.012 and new[3, 2] == -0.018 and new[1, 2] == 0.0
    assert new[2, 2] == -0.012
    np.testing.assert_array_equal(new[:, 3], hot[:, 3])
    np.testing.assert_array_equal(new[:, [0, 1, 4, 5]], hot[:, [0, 1, 4, 5]])
