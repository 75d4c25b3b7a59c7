"""Pins of the warm start's input features and guess smoother in the
oracle: the cube means against scipy's uniform filter, a delta and a
constant (closed forms); the feature channels' definitions; the damped
sweep's factor on eigenmodes (closed form, smooth and checkerboard ends)
and the exact discrete solution as its fixed point."""

import math

import numpy as np
import pytest
import scipy.fft as sf
from scipy import ndimage

import oracle
import synth
from oracle import cnn


@pytest.mark.parametrize("h", [1, 2, 5])
def test_box_mean_equals_scipy_uniform_filter(h):
    a = synth.rng(3).standard_normal((7, 9, 12))
    want = ndimage.uniform_filter(a, size=2 * h + 1, mode="constant", cval=0.0)
    np.testing.assert_allclose(cnn.box_mean(a, h), want, rtol=1e-12, atol=1e-14)


def test_box_mean_of_a_delta_and_of_ones():
    h = 2
    a = np.zeros((6, 7, 9))
    a[3, 2, 4] = 1.0
    got = cnn.box_mean(a, h)
    vol = (2 * h + 1) ** 3
    k, j, i = np.meshgrid(np.arange(6), np.arange(7), np.arange(9), indexing="ij")
    inside = (np.abs(k - 3) <= h) & (np.abs(j - 2) <= h) & (np.abs(i - 4) <= h)
    assert np.array_equal(got, np.where(inside, 1.0 / vol, 0.0))

    def counts(n):
        return np.array([min(t + h, n - 1) - max(t - h, 0) + 1 for t in range(n)], float)
    want = (counts(6)[:, None, None] * counts(7)[None, :, None] * counts(9)[None, None, :]) / vol
    np.testing.assert_allclose(cnn.box_mean(np.ones((6, 7, 9)), h), want, rtol=1e-15)


def test_feature_channels():
    nx, ny, nz = 14, 11, 9
    u = synth.dirichlet_uniform(nx, ny, nz, 2)
    f = synth.gaussian_sources(nx, ny, nz, 3, 4)
    F, s = cnn.features(u, f)
    assert F.shape == (8, nz, ny, nx)
    g = cnn.boundary_lift(u)
    fi = f[1:-1, 1:-1, 1:-1]
    assert s == max(np.abs(fi).max(), np.abs(g).max())
    np.testing.assert_array_equal(F[0], fi / s)
    np.testing.assert_array_equal(F[1], g / s)
    for c, h in zip((2, 3, 4, 5, 7), cnn.BOX_HALF):
        np.testing.assert_allclose(F[c], ndimage.uniform_filter(fi / s, 2 * h + 1,
                                                                mode="constant"), atol=1e-14)
    phi, _ = cnn.slowest_modes(nx, ny, nz)
    np.testing.assert_array_equal(F[6], phi)
    assert F[6].max() <= 1.0 and F[6].min() > 0.0


def _mode(nx, ny, nz, a, b, c):
    sx = np.sin(np.pi * a * np.arange(1, nx + 1) / (nx + 1))
    sy = np.sin(np.pi * b * np.arange(1, ny + 1) / (ny + 1))
    sz = np.sin(np.pi * c * np.arange(1, nz + 1) / (nz + 1))
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


@pytest.mark.parametrize("mode", [(1, 1, 1), (2, 1, 3), (10, 8, 6), (5, 4, 3)])
def test_damped_sweep_factor_on_eigenmodes(mode):
    nx, ny, nz = 10, 8, 6
    e = _mode(nx, ny, nz, *mode)
    x = synth.zeros(nx, ny, nz)
    x[1:-1, 1:-1, 1:-1] = e
    mu = (math.cos(math.pi * mode[0] / (nx + 1)) + math.cos(math.pi * mode[1] / (ny + 1))
          + math.cos(math.pi * mode[2] / (nz + 1))) / 3
    w = 2.0 / 3.0
    for m in (1, 3):
        got = cnn.smooth_guess(x, None, m)[1:-1, 1:-1, 1:-1]
        np.testing.assert_allclose(got, (1 - w * (1 - mu)) ** m * e, atol=1e-14)
    assert np.array_equal(cnn.smooth_guess(x, None, 0), x)


def test_exact_solution_is_a_fixed_point_of_the_smoother():
    nx, ny, nz = 12, 10, 8
    f = synth.gaussian_sources(nx, ny, nz, 3, 9)

    def eigs(n):
        return 2.0 * np.cos(np.pi * np.arange(1, n + 1) / (n + 1)) - 2.0
    lam = eigs(nz)[:, None, None] + eigs(ny)[None, :, None] + eigs(nx)[None, None, :]
    x = synth.zeros(nx, ny, nz)
    x[1:-1, 1:-1, 1:-1] = sf.idstn(sf.dstn(f[1:-1, 1:-1, 1:-1], type=1) / lam, type=1)
    assert oracle.residual_norm(x, f) < 1e-12 * np.linalg.norm(f)
    np.testing.assert_allclose(cnn.smooth_guess(x, f, 4), x, atol=1e-12 * np.abs(x).max())
