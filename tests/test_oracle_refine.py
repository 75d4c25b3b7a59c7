"""Pins of the oracle's FP32-storage + FP64 iterative refinement and of its
power-of-two scaling, against facts independent of the oracle's stencil code:
an explicitly assembled dense system, numpy.linalg.solve, and the FP32
precision plateau that refinement exists to get past."""

import math

import numpy as np
import pytest

import oracle
import synth
from test_oracle_jacobi import dense_system


@pytest.mark.parametrize("norm,ncells", [(1.0, 1), (3.0, 4), (1e-300, 7), (5e300, 2),
                                         (0.7, 1000), (2.0 ** 40, 2.0 ** 20)])
def test_pow2_scale_brackets_the_rms_residual(norm, ncells):
    s = oracle.pow2_scale(norm, int(ncells))
    m = norm / math.sqrt(ncells)
    mant, _ = math.frexp(s)
    assert mant == 0.5  # a power of two
    assert s <= m < 2 * s


@pytest.mark.parametrize("norm", [0.0, float("inf"), float("nan")])
def test_pow2_scale_of_a_degenerate_norm_is_one(norm):
    assert oracle.pow2_scale(norm, 10) == 1.0


def _interior_vector(x, idx):
    return np.array([x[k + 1, j + 1, i + 1] for (i, j, k) in idx])


def _problem(dims, seed):
    nx, ny, nz = dims
    u = synth.dirichlet_uniform(nx, ny, nz, seed)
    f = synth.gaussian_sources(nx, ny, nz, 3, seed + 1)
    return u, f


@pytest.mark.parametrize("dims", [(6, 5, 4), (9, 3, 7)])
def test_refined_answer_meets_the_tolerance_of_the_dense_system(dims):
    u, f = _problem(dims, 40)
    A, b, idx = dense_system(u, f)
    out = oracle.refined_solve(u, f, 1e-11, 1e-4, 20, 100000, 256)
    assert out["converged"]
    x = _interior_vector(out["x"], idx)
    # residual of the dense system b - A x, relative to the zero interior's (= b)
    assert np.linalg.norm(b - A @ x) <= 1e-11 * np.linalg.norm(b) * (1 + 1e-6)
    xs = np.linalg.solve(A, b)
    cond = np.linalg.cond(A)
    assert np.linalg.norm(x - xs) <= 2 * cond * 1e-11 * np.linalg.norm(xs)
    # the halo is the input's
    h = out["x"].copy()
    h[1:-1, 1:-1, 1:-1] = 0.0
    assert np.array_equal(h, oracle.zero_interior(u))


def test_refinement_gets_past_the_fp32_plateau():
    """FP32 storage alone stalls near FP32 precision; each refinement step
    resumes from an FP64 residual, so the outer residual keeps falling."""
    dims = (8, 6, 5)
    u, f = _problem(dims, 50)
    res0 = oracle.residual_norm(oracle.zero_interior(u), f)
    # plain FP32 Jacobi on the whole problem (FP32 halo and right-hand side)
    e = u.astype(np.float32)
    for _ in range(4000):
        e = oracle.sweep_f32(e, f.astype(np.float32))
    plateau = oracle.residual_norm(e.astype(np.float64), f) / res0
    assert plateau > 1e-9  # FP32 cannot represent a much better answer
    out = oracle.refined_solve(u, f, 1e-13, 1e-5, 20, 100000, 256)
    assert out["converged"] and out["hist"][-1] <= 1e-13
    assert out["hist"][-1] < 1e-3 * plateau
    # every outer step reduces the residual
    assert all(b < a for a, b in zip(out["hist"], out["hist"][1:]))


def test_each_outer_step_gains_at_least_the_inner_reduction():
    """With a coarse inner target (eta = 0.5) every outer step still cuts the
    outer residual by about that factor (the inner solve is exact up to FP32
    rounding), and the refinement converges."""
    u, f = _problem((7, 7, 7), 60)
    coarse = oracle.refined_solve(u, f, 1e-8, 0.5, 60, 100000, 256)
    assert coarse["converged"] and coarse["hist"][-1] <= 1e-8
    h = coarse["hist"]
    assert all(b <= 0.5 * a * (1 + 1e-3) for a, b in zip(h, h[1:]))
