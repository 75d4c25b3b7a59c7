"""Pins of the red-black Gauss-Seidel oracle against facts independent of
its code: the dense-matrix red-black iteration, exact fixed points, the
classical rate rho(GS) = rho(Jacobi)^2 of a consistently ordered matrix, and
numpy.linalg.solve."""

import math

import numpy as np
import pytest

import oracle
import synth
from test_oracle_jacobi import dense_system, linear_field


def _vec(u, idx):
    return np.array([u[k + 1, j + 1, i + 1] for (i, j, k) in idx])


@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 3, 3), (4, 3, 2), (5, 1, 2), (1, 1, 1)])
def test_sweep_equals_dense_red_black_gauss_seidel(dims):
    nx, ny, nz = dims
    u = synth.dirichlet_uniform(nx, ny, nz, 71)
    u[1:-1, 1:-1, 1:-1] = synth.rng(72).standard_normal((nz, ny, nx))
    f = synth.gaussian_sources(nx, ny, nz, 2, 73)
    A, b, idx = dense_system(u, f)
    red = np.array([(i + j + k) % 2 == 0 for (i, j, k) in idx])
    x = _vec(u, idx)
    v = u
    for _ in range(6):
        # x_R <- D_R^-1 (b_R - A_RB x_B), then x_B <- D_B^-1 (b_B - A_BR x_R)
        for colour in (red, ~red):
            xn = x.copy()
            xn[colour] = (b[colour] - (A[colour][:, ~colour] @ x[~colour])) / np.diag(A)[colour]
            x = xn
        v = oracle.rbgs_sweep(v, f)
        assert np.allclose(_vec(v, idx), x, rtol=1e-13, atol=1e-13)


def test_half_sweep_changes_one_colour_by_the_jacobi_update():
    nx, ny, nz = 7, 5, 4
    u = synth.dirichlet_uniform(nx, ny, nz, 74)
    u[1:-1, 1:-1, 1:-1] = synth.rng(75).standard_normal((nz, ny, nx))
    f = synth.gaussian_sources(nx, ny, nz, 2, 76)
    jac = oracle.jacobi_sweep(u, f)
    for red in (True, False):
        h = oracle.rbgs_half(u, f, red)
        m = oracle.red_mask(u) if red else ~oracle.red_mask(u)
        assert np.array_equal(h[1:-1, 1:-1, 1:-1][m], jac[1:-1, 1:-1, 1:-1][m])
        assert np.array_equal(h[1:-1, 1:-1, 1:-1][~m], u[1:-1, 1:-1, 1:-1][~m])
        hh = h.copy()
        hh[1:-1, 1:-1, 1:-1] = 0.0
        uu = u.copy()
        uu[1:-1, 1:-1, 1:-1] = 0.0
        assert np.array_equal(hh, uu)  # halo untouched


@pytest.mark.parametrize("coef", [(3, 1, -2, 5), (0, 2, 0, 0)])
def test_integer_linear_fields_are_exact_fixed_points(coef):
    u = linear_field(9, 6, 5, coef)
    assert np.array_equal(oracle.rbgs_sweep(u, None), u)


def test_asymptotic_rate_is_the_square_of_the_jacobi_rate():
    """Red-black ordering is consistent, so rho(GS) = rho(J)^2 (Young)."""
    nx, ny, nz = 10, 8, 6
    rho_j = (math.cos(math.pi / (nx + 1)) + math.cos(math.pi / (ny + 1))
             + math.cos(math.pi / (nz + 1))) / 3.0
    u = synth.zeros(nx, ny, nz)
    u[1:-1, 1:-1, 1:-1] = synth.rng(77).random((nz, ny, nx))
    _, hist = oracle.rbgs_sweeps(u, None, 400)
    rate = (hist[-1] / hist[-101]) ** (1.0 / 100)
    assert rate == pytest.approx(rho_j ** 2, rel=2e-3)


def test_solve_converges_to_the_dense_solution_in_about_half_the_jacobi_sweeps():
    nx, ny, nz = 6, 5, 4
    u = synth.dirichlet_uniform(nx, ny, nz, 78)
    f = synth.gaussian_sources(nx, ny, nz, 3, 79)
    A, b, idx = dense_system(u, f)
    xs = np.linalg.solve(A, b)
    K, uk, hist, res0, ok = oracle.rbgs_solve(u, f, 1e-12, 100000)
    assert ok and hist[K] / res0 <= 1e-12 < hist[K - 1] / res0
    assert np.allclose(_vec(uk, idx), xs, rtol=0, atol=1e-10 * np.max(np.abs(xs)))
    kj, *_ = oracle.jacobi_solve(u, f, 1e-12, 100000)
    assert 0.4 < K / kj < 0.6
