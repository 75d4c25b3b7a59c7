"""Pins of the oracle's start selection for the learned warm start: the two
slowest Jacobi modes are eigenvectors of the 7-point operator with the
eigenvalues the closed form gives, the projection length has its closed
form on them and vanishes on every other eigenvector, and the three rules
decide as the definitions require on guesses built from the exact discrete
solution (discrete sine transform, which diagonalises the operator)."""

import math

import numpy as np
import pytest
import scipy.fft as sf

import oracle
import synth
from oracle import cnn

SHAPES = [(7, 5, 4), (6, 6, 6), (9, 4, 3)]


def _field(interior):
    nz, ny, nx = interior.shape
    u = synth.zeros(nx, ny, nz)
    u[1:-1, 1:-1, 1:-1] = interior
    return u


def _axis_eigs(n):
    return 2.0 * np.cos(np.pi * np.arange(1, n + 1) / (n + 1)) - 2.0


def _mode(nx, ny, nz, a, b, c):
    """Eigenvector (a, b, c) of the operator (1-based wave numbers)."""
    sx = np.sin(np.pi * a * np.arange(1, nx + 1) / (nx + 1))
    sy = np.sin(np.pi * b * np.arange(1, ny + 1) / (ny + 1))
    sz = np.sin(np.pi * c * np.arange(1, nz + 1) / (nz + 1))
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def _exact(f_int):
    nz, ny, nx = f_int.shape
    lam = (_axis_eigs(nz)[:, None, None] + _axis_eigs(ny)[None, :, None]
           + _axis_eigs(nx)[None, None, :])
    return sf.idstn(sf.dstn(f_int, type=1) / lam, type=1)


@pytest.mark.parametrize("shape", SHAPES)
def test_slowest_modes_are_eigenvectors_with_rates_plus_and_minus_rho(shape):
    nx, ny, nz = shape
    phi, psi = cnn.slowest_modes(nx, ny, nz)
    cs = sum(math.cos(math.pi / (n + 1)) for n in shape)
    rho = cs / 3.0
    # L(phi) = (2 sum cos - 6) phi, L(psi) = (-2 sum cos - 6) psi; residual = -L
    np.testing.assert_allclose(oracle.residual(_field(phi)), -(2 * cs - 6) * phi, atol=1e-13)
    np.testing.assert_allclose(oracle.residual(_field(psi)), -(-2 * cs - 6) * psi, atol=1e-13)
    # one Jacobi sweep multiplies them by +rho and -rho
    np.testing.assert_allclose(oracle.interior(oracle.jacobi_sweep(_field(phi))), rho * phi,
                               atol=1e-13)
    np.testing.assert_allclose(oracle.interior(oracle.jacobi_sweep(_field(psi))), -rho * psi,
                               atol=1e-13)


@pytest.mark.parametrize("shape", SHAPES)
def test_slow_mode_norm_closed_form_and_orthogonality(shape):
    nx, ny, nz = shape
    phi, psi = cnn.slowest_modes(nx, ny, nz)
    nn = (nx + 1) * (ny + 1) * (nz + 1) / 8.0  # ||phi||^2 = prod (n + 1) / 2
    assert cnn.slow_mode_norm(3.0 * phi) == pytest.approx(3.0 * nn, rel=1e-12)
    assert cnn.slow_mode_norm(-2.0 * psi) == pytest.approx(2.0 * nn, rel=1e-12)
    assert cnn.slow_mode_norm(3.0 * phi - 4.0 * psi) == pytest.approx(5.0 * nn, rel=1e-12)
    # every other eigenvector is orthogonal to both
    for a, b, c in [(2, 1, 1), (1, 2, 1), (1, 1, 2), (nx, ny, nz - 1), (2, 3, 1)]:
        if a <= nx and b <= ny and c <= nz and (a, b, c) not in ((1, 1, 1), (nx, ny, nz)):
            assert cnn.slow_mode_norm(_mode(nx, ny, nz, a, b, c)) < 1e-12 * nn


def test_dst_gives_the_exact_discrete_solution():
    f = synth.gaussian_sources(9, 7, 6, 3, 5)
    x = _exact(f[1:-1, 1:-1, 1:-1])
    assert oracle.residual_norm(_field(x), f) < 1e-12 * np.linalg.norm(f)


def test_start_choice_rules():
    nx, ny, nz = 12, 10, 8
    u = synth.zeros(nx, ny, nz)
    f = synth.gaussian_sources(nx, ny, nz, 3, 7)
    x = _exact(f[1:-1, 1:-1, 1:-1])
    # the exact solution: every rule takes it
    for rule in cnn.RULES:
        use, meas = cnn.start_choice(u, f, x, rule)
        assert use, rule
        assert meas[0] < 1e-10 * meas[1] and meas[2] < 1e-10 * meas[3]
    # the zero guess ties with u0: only "force" takes it
    for rule in cnn.RULES:
        use, meas = cnn.start_choice(u, f, np.zeros_like(x), rule)
        assert meas[0] == meas[1] and meas[2] == meas[3]
        assert use == (rule == "force")
    # exact + a large high-frequency eigenvector: the residual grows past
    # ||r(u0)||, the slowest components stay those of the exact solution
    hf = _mode(nx, ny, nz, 6, 5, 4)
    g = x + 4.0 * np.abs(x).max() * hf
    use_r, meas = cnn.start_choice(u, f, g, "residual")
    use_s, _ = cnn.start_choice(u, f, g, "slow_modes")
    assert meas[0] > meas[1] and not use_r
    assert meas[2] < 1e-9 * meas[3] and use_s
    # exact + twice the zero guess's slowest error component: the slow-mode
    # rule rejects it
    phi, _ = cnn.slowest_modes(nx, ny, nz)
    lam1 = 2 * sum(math.cos(math.pi / (n + 1)) for n in (nx, ny, nz)) - 6
    p0 = float(np.sum(f[1:-1, 1:-1, 1:-1] * phi))
    c = 2.0 * p0 / (lam1 * np.sum(phi * phi))
    use_s, meas = cnn.start_choice(u, f, x + c * phi, "slow_modes")
    # the guess's residual is -lam1 c phi: its projection is 2 |<f, phi>|
    assert meas[2] == pytest.approx(2.0 * abs(p0), rel=1e-9)
    assert meas[2] > meas[3] and not use_s
    with pytest.raises(ValueError):
        cnn.start_choice(u, f, x, "nope")
