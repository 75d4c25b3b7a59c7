"""Pins of the oracle's 7-point sweep, residual and solve against facts the
paper and the mathematics fix (not against a retyping of the oracle)."""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")


class Counted:
    """Float wrapper counting every +, -, * applied to it (flop counter)."""

    n = 0
    __slots__ = ("v",)

    def __init__(self, v):
        self.v = float(v)

    @staticmethod
    def _val(o):
        return o.v if isinstance(o, Counted) else float(o)

    def _op(self, o, fn):
        Counted.n += 1
        return Counted(fn(self.v, Counted._val(o)))

    def __add__(self, o):
        return self._op(o, lambda a, b: a + b)

    def __radd__(self, o):
        return self._op(o, lambda a, b: b + a)

    def __sub__(self, o):
        return self._op(o, lambda a, b: a - b)

    def __rsub__(self, o):
        return self._op(o, lambda a, b: b - a)

    def __mul__(self, o):
        return self._op(o, lambda a, b: a * b)

    def __rmul__(self, o):
        return self._op(o, lambda a, b: b * a)


def counted_grid(a):
    out = np.empty(a.shape, dtype=object)
    for idx, v in np.ndenumerate(a):
        out[idx] = Counted(v)
    return out


def linear_field(nx, ny, nz, coef):
    a, b, c, d = coef
    k, j, i = np.meshgrid(np.arange(-1, nz + 1), np.arange(-1, ny + 1),
                          np.arange(-1, nx + 1), indexing="ij")
    return (a + b * i + c * j + d * k).astype(np.float64)


# ---------------------------------------------------------------- flop count

def test_update_costs_six_flops_per_cell_like_the_paper():
    facts = json.load(open(GOLDEN))
    nx, ny, nz = 3, 4, 2
    u = counted_grid(synth.dirichlet_uniform(nx, ny, nz, 5))
    Counted.n = 0
    oracle.jacobi_sweep(u, None, c6=oracle.C6_F64)
    assert Counted.n == facts["laplace_flops_per_cell"]["value"] * nx * ny * nz
    f = counted_grid(synth.gaussian_sources(nx, ny, nz, 2, 3))
    Counted.n = 0
    oracle.jacobi_sweep(u, f, c6=oracle.C6_F64)
    assert Counted.n == 7 * nx * ny * nz  # one more for the right-hand side


# ------------------------------------------------------------- fixed points

@pytest.mark.parametrize("dims", [(5, 4, 3), (16, 16, 16), (33, 7, 12)])
@pytest.mark.parametrize("coef", [(0, 1, 0, 0), (3, -2, 5, 7), (-1000, 17, -3, 250)])
def test_integer_linear_fields_are_exact_fixed_points(dims, coef):
    u = linear_field(*dims, coef)
    for f in (None, np.zeros_like(u)):
        v = oracle.jacobi_sweep(u, f)
        assert np.array_equal(v, u)
        assert oracle.residual_norm(u, f) == 0.0


def test_constant_field_is_a_fixed_point_for_every_sweep_count():
    u = np.full((10, 9, 8), 0.375)
    v, hist = oracle.jacobi_sweeps(u, None, 7)
    assert np.array_equal(v, u)
    assert hist == [0.0] * 8


def test_halo_is_never_written():
    u = synth.dirichlet_uniform(6, 5, 4, 11)
    u[1:-1, 1:-1, 1:-1] = synth.rng(12).random((4, 5, 6))
    v = oracle.jacobi_sweep(u, synth.gaussian_sources(6, 5, 4, 3, 1))
    mask = np.ones(u.shape, bool)
    mask[1:-1, 1:-1, 1:-1] = False
    assert np.array_equal(v[mask], u[mask])


# ------------------------------------------------------------ quadratic

@pytest.mark.parametrize("q", [(1, 2, 3, 0, 0, 0), (2, -1, 4, 3, -2, 5), (-3, 1, 1, 1, 1, 1)])
def test_laplacian_of_a_quadratic_is_exact(q):
    a, b, c, dxy, dyz, dxz = q
    nx, ny, nz = 7, 6, 5
    k, j, i = np.meshgrid(np.arange(-1, nz + 1), np.arange(-1, ny + 1),
                          np.arange(-1, nx + 1), indexing="ij")
    u = (a * i * i + b * j * j + c * k * k + dxy * i * j + dyz * j * k
         + dxz * i * k + 5 * i - 2 * j + 9).astype(np.float64)
    lap = 2 * (a + b + c)  # the cross and linear terms are harmonic
    f = np.full_like(u, float(lap))
    r = oracle.residual(u, f)
    assert np.all(r == 0.0)
    # r = 0 - lap everywhere: the norm of a constant residual is |c| sqrt(N)
    n = nx * ny * nz
    got = oracle.residual_norm(u, None)
    assert got == pytest.approx(abs(lap) * math.sqrt(n), rel=2e-16)


def test_residual_norm_is_exact_sum_on_small_grid():
    u = synth.dirichlet_uniform(4, 3, 5, 2)
    u[1:-1, 1:-1, 1:-1] = synth.rng(3).standard_normal((5, 3, 4))
    f = synth.gaussian_sources(4, 3, 5, 2, 9)
    exact = oracle.residual(u.astype(object) * Fraction(1), f.astype(object) * Fraction(1))
    s = sum(Fraction(x) ** 2 for x in exact.ravel())
    want = math.sqrt(float(s))
    assert oracle.residual_norm(u, f) == pytest.approx(want, rel=1e-15)


# ------------------------------------------------------------ eigenmode

@pytest.mark.parametrize("dims", [(8, 8, 8), (12, 7, 9)])
def test_eigenmode_decays_by_the_jacobi_spectral_radius(dims):
    nx, ny, nz = dims
    u0 = synth.eigenmode(nx, ny, nz)
    rho = (math.cos(math.pi / (nx + 1)) + math.cos(math.pi / (ny + 1))
           + math.cos(math.pi / (nz + 1))) / 3.0
    u = u0
    for k in range(1, 41):
        u = oracle.jacobi_sweep(u, None)
        err = np.max(np.abs(u - rho ** k * u0))
        assert err <= 8 * k * 2.0 ** -53


# ------------------------------------------------- dense-matrix Jacobi (tiny)

def dense_system(u, f):
    """Assemble A x = b for the interior unknowns of the 7-point Poisson
    problem by walking every cell's six neighbours (no stencil code)."""
    nz, ny, nx = (s - 2 for s in u.shape)
    idx = {}
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                idx[(i, j, k)] = len(idx)
    n = len(idx)
    A = np.zeros((n, n))
    b = np.zeros(n)
    for (i, j, k), p in idx.items():
        A[p, p] = -6.0
        b[p] = f[k + 1, j + 1, i + 1] if f is not None else 0.0
        for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            q = (i + d[0], j + d[1], k + d[2])
            if q in idx:
                A[p, idx[q]] = 1.0
            else:  # Dirichlet neighbour moves to the right-hand side
                b[p] -= u[q[2] + 1, q[1] + 1, q[0] + 1]
    return A, b, idx


@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 3, 3), (4, 3, 2), (1, 1, 1), (5, 1, 2)])
def test_sweeps_equal_dense_matrix_jacobi(dims):
    nx, ny, nz = dims
    u = synth.dirichlet_uniform(nx, ny, nz, 21)
    u[1:-1, 1:-1, 1:-1] = synth.rng(22).standard_normal((nz, ny, nx))
    f = synth.gaussian_sources(nx, ny, nz, 3, 23)
    A, b, idx = dense_system(u, f)
    D = np.diag(np.diag(A))
    R = A - D
    x = np.array([u[k + 1, j + 1, i + 1] for (i, j, k) in idx])
    v = u
    for _ in range(25):
        x = np.linalg.solve(D, b - R @ x)
        v = oracle.jacobi_sweep(v, f)
        got = np.array([v[k + 1, j + 1, i + 1] for (i, j, k) in idx])
        assert np.allclose(got, x, rtol=1e-13, atol=1e-13)
        # the residual of the oracle is the dense b - A x
        rd = b - A @ got
        assert oracle.residual_norm(v, f) == pytest.approx(np.linalg.norm(rd), rel=1e-11, abs=1e-13)


def test_solve_converges_to_dense_solution():
    nx, ny, nz = 4, 3, 3
    u = synth.dirichlet_uniform(nx, ny, nz, 31)
    f = synth.gaussian_sources(nx, ny, nz, 4, 32)
    A, b, idx = dense_system(u, f)
    xs = np.linalg.solve(A, b)
    K, uk, hist, res0, ok = oracle.jacobi_solve(u, f, 1e-12, 10000)
    assert ok
    got = np.array([uk[k + 1, j + 1, i + 1] for (i, j, k) in idx])
    assert np.allclose(got, xs, rtol=0, atol=1e-10 * np.max(np.abs(xs)) + 1e-12)
    # K is the first index that meets the tolerance
    assert hist[K] / res0 <= 1e-12 < hist[K - 1] / res0


# ------------------------------------------------------ iteration count

@pytest.mark.parametrize("tol", [1e-3, 1e-6])
def test_iteration_count_of_an_eigenmode_problem(tol):
    """Exact solution phi (an eigenvector of the Jacobi operator with
    eigenvalue rho) and zero start: r_k = rho^k r_0, so K = ceil(ln tol / ln rho)."""
    nx, ny, nz = 10, 8, 6
    phi = synth.eigenmode(nx, ny, nz)
    rho = (math.cos(math.pi / (nx + 1)) + math.cos(math.pi / (ny + 1))
           + math.cos(math.pi / (nz + 1))) / 3.0
    f = np.zeros_like(phi)
    f[1:-1, 1:-1, 1:-1] = -6.0 * (1.0 - rho) * phi[1:-1, 1:-1, 1:-1]
    K, _, hist, res0, ok = oracle.jacobi_solve(np.zeros_like(phi), f, tol, 100000)
    assert ok
    want = math.ceil(math.log(tol) / math.log(rho))
    assert abs(K - want) <= 1
    for k in (1, K // 2, K):
        assert hist[k] / res0 == pytest.approx(rho ** k, rel=1e-9)


def test_zero_reference_residual_gives_zero_sweeps():
    u = synth.eigenmode(5, 5, 5)  # zero halo, f = 0: u^0 = 0 is exact
    K, uk, hist, res0, ok = oracle.jacobi_solve(u, None, 1e-8, 10)
    assert (K, res0, ok) == (0, 0.0, True)
    assert np.array_equal(uk, u)


def test_not_converged_stops_at_max_sweeps():
    u = synth.dirichlet_uniform(6, 6, 6, 1)
    K, _, hist, res0, ok = oracle.jacobi_solve(u, None, 1e-14, 5)
    assert not ok and K == 5 and len(hist) == 6


def test_f32_sweep_matches_exact_rounding_of_each_step():
    """Each FP32 step is the correctly rounded result of its exact inputs."""
    e = np.zeros((5, 6, 7), np.float32)
    e[1:-1, 1:-1, 1:-1] = synth.rng(4).standard_normal((3, 4, 5)).astype(np.float32)
    rh = np.zeros_like(e)
    rh[1:-1, 1:-1, 1:-1] = synth.rng(5).standard_normal((3, 4, 5)).astype(np.float32)
    got = oracle.sweep_f32(e, rh)
    c6 = Fraction(1, 6)
    c6_32 = np.float32(float(c6))  # nearest float32 to 1/6
    assert oracle.C6_F32 == c6_32
    for (k, j, i) in [(1, 1, 1), (2, 3, 4), (3, 4, 5)]:
        # sums and products of two float32 values are exact in float64, so
        # Fraction -> float64 -> float32 rounds once
        s = e[k, j, i + 1]
        for t in (e[k, j, i - 1], e[k, j + 1, i], e[k, j - 1, i], e[k + 1, j, i], e[k - 1, j, i]):
            s = np.float32(float(Fraction(float(s)) + Fraction(float(t))))
        d = np.float32(float(Fraction(float(s)) - Fraction(float(rh[k, j, i]))))
        want = np.float32(float(Fraction(float(d)) * Fraction(float(c6_32))))
        assert got[k, j, i] == want
