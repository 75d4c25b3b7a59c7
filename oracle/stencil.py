"""Oracle for the stencil sweeps, the residual norm, convergence control,
FP32-storage refinement and the advection source term.

TEST INFRASTRUCTURE ONLY -- see the package docstring. Parity status of each
function is stated in its docstring; the pins live in ``tests/test_oracle_*``.

Notation: a field ``u`` is a halo-padded array indexed [k, j, i] (z, y, x);
"interior" is [1:-1, 1:-1, 1:-1]. The paper's stencil.apply (Section 2.2,
Listing 2) reads a bounded input with a one-cell halo at constant offsets
and produces a new field on the interior, so every update here is
out-of-place and never writes the halo.
"""

from __future__ import annotations

import math

import numpy as np

# fl(1/6): the listings multiply by a constant rather than divide
# (Section 2.2, Listing 2 multiplies the neighbour sum by 0.25).
C6_F64 = 1.0 / 6.0
C6_F32 = np.float32(1.0) / np.float32(6.0)

INTERIOR = (slice(1, -1), slice(1, -1), slice(1, -1))


def interior(a):
    return a[INTERIOR]


def shifted(a, di: int, dj: int, dk: int):
    """View of ``a`` at offset (di, dj, dk) from every interior cell."""
    nz, ny, nx = (s - 2 for s in a.shape)
    return a[1 + dk:nz + 1 + dk, 1 + dj:ny + 1 + dj, 1 + di:nx + 1 + di]


def zero_interior(u):
    z = u.copy()
    z[INTERIOR] = 0
    return z


def neighbour_sum(u):
    """Six-neighbour sum S of the 7-point stencil (Section 4.1, Gauss-Seidel
    benchmark: the orthogonal neighbours in three dimensions).

    Accumulation order (a reading; the paper's listings are sketches): per
    dimension the +1 neighbour then the -1 neighbour, dimensions x, y, z:
    S = (((((u[i+1] + u[i-1]) + u[j+1]) + u[j-1]) + u[k+1]) + u[k-1]).
    """
    return (((((shifted(u, 1, 0, 0) + shifted(u, -1, 0, 0))
               + shifted(u, 0, 1, 0)) + shifted(u, 0, -1, 0))
             + shifted(u, 0, 0, 1)) + shifted(u, 0, 0, -1))


def _c6_for(u):
    if u.dtype == np.float32:
        return C6_F32
    return C6_F64


def jacobi_sweep(u, f=None, c6=None):
    """One 7-point Jacobi update (Section 4.1: the average of the six
    neighbours, six flops per cell; with a right-hand side one more).

    u'(p) = (S(p) - f(p)) * C6 on the interior, C6 = fl(1/6); with no f,
    u'(p) = S(p) * C6 (identical bits to f = 0). The halo is copied, never
    updated: it holds the Dirichlet values. Works in the dtype of ``u``
    (float64, or float32 for the FP32-storage inner sweeps).

    Reading: the benchmark is named Gauss-Seidel but stencil.apply produces a
    new field (Section 2.2), i.e. a Jacobi update; the right-hand side
    generalises Laplace to Poisson, L(u) = S - 6u = f with h = 1.
    """
    if c6 is None:
        c6 = _c6_for(u)
    out = u.copy()
    s = neighbour_sum(u)
    if f is None:
        out[INTERIOR] = s * c6
    else:
        out[INTERIOR] = (s - interior(f)) * c6
    return out


def sweep_f32(e, rhat):
    """FP32-storage, FP32-arithmetic sweep of the inner correction solve
    L(e) = rhat: e' = (S32(e) - rhat) * fl32(1/6), same order as
    ``jacobi_sweep``."""
    assert e.dtype == np.float32 and rhat.dtype == np.float32
    return jacobi_sweep(e, rhat, C6_F32)


def residual(u, f=None):
    """r = f - (S - u*6) on the interior, in the dtype of ``u``.

    Reading: the paper has no convergence test; the residual is the true
    residual of the discrete system L(u) = f (not the update size), evaluated
    in exactly this order. With no f, r = -(S - 6u).
    """
    lap = neighbour_sum(u) - interior(u) * 6
    if f is None:
        return -lap
    return interior(f) - lap


def residual_norm(u, f=None) -> float:
    """||f - L(u)||_2 over the interior, accumulated in FP64."""
    r = residual(u, f)
    r = np.asarray(r, dtype=np.float64)
    return math.sqrt(float(np.sum(r * r)))


def residual_norm_f32_storage(e, rhat) -> float:
    """FP64 residual norm of an FP32-stored iterate: the FP32 values are
    widened exactly to FP64 and the residual is formed in FP64."""
    return residual_norm(np.asarray(e, np.float64), np.asarray(rhat, np.float64))


def jacobi_sweeps(u0, f, n: int):
    """Exactly ``n`` sweeps from u0. Returns (u_n, hist) where hist[k] is
    ||r(u_k)|| for k = 0..n (n + 1 values)."""
    u = u0.copy()
    hist = [residual_norm(u, f)]
    for _ in range(n):
        u = jacobi_sweep(u, f)
        hist.append(residual_norm(u, f))
    return u, hist


def jacobi_solve(u0, f, tol: float, max_sweeps: int):
    """FP64 Jacobi to a relative residual.

    K = the smallest k >= 0 with ||r(u_k)|| / ||r(u^0)|| <= tol, where u^0 is
    u0 with its interior zeroed (same halo, same f), so every starting guess
    aims at one absolute target. If ||r(u^0)|| = 0 then K = 0. Returns
    (K, u_K, hist, res0, converged); hist[k] = ||r(u_k)||. If no k <=
    max_sweeps qualifies, returns K = max_sweeps, converged = False.
    """
    res0 = residual_norm(zero_interior(u0), f)
    u = u0.copy()
    hist = []
    k = 0
    while True:
        rk = residual_norm(u, f)
        hist.append(rk)
        if res0 == 0.0 or rk / res0 <= tol:
            return k, u, hist, res0, True
        if k == max_sweeps:
            return k, u, hist, res0, False
        u = jacobi_sweep(u, f)
        k += 1


def pow2_scale(norm: float, ncells: int) -> float:
    """Power-of-two scale s with s <= norm/sqrt(N) < 2s (s = 1 if norm = 0).

    Scaling by a power of two is exact, so the FP32 right-hand side
    fl32(r / s) and the update x + s*e depend on the residual norm only
    through its binary exponent.
    """
    m = norm / math.sqrt(float(ncells))
    if m == 0.0 or not math.isfinite(m):
        return 1.0
    _, e = math.frexp(m)
    return math.ldexp(1.0, e - 1)


def refined_solve(x0, f, tol: float, eta: float, max_outer: int, max_inner: int,
                  stall: int, inner_counts=None):
    """FP32-storage Jacobi with FP64 iterative refinement.

    Outer step: r = f - L(x) in FP64; stop when ||r|| / ||r(u^0)|| <= tol.
    Otherwise s = pow2_scale(||r||, N), rhat = fl32(r / s), and the inner FP32
    Jacobi solves L(e) = rhat from e = 0 with a zero halo. Inner sweep j
    first measures the FP64 residual rho_j = ||rhat - L(e_j)|| of its input;
    the inner stops at the first j with rho_j <= eta_o * rho_0, or j =
    max_inner, or (stagnation) j >= stall and rho_j >= rho_{j - stall}.
    The inner target eta_o = max(eta, tol / (2 rel_o)) asks for no more than
    the reduction that brings the outer residual to half the tolerance.
    Then x += s * e on the interior, in FP64.

    ``inner_counts`` replays given inner sweep counts instead of testing
    the stopping rule (used to compare fields bit for bit).

    Returns dict(x, converged, outer, inner=[...], hist=[rel per outer],
    res0, sweeps, rho=[[rho_0, rho_1, ...] per outer], eta=[eta_o per outer]).
    """
    nz, ny, nx = (s - 2 for s in x0.shape)
    ncells = nx * ny * nz
    res0 = residual_norm(zero_interior(x0), f)
    x = np.array(x0, dtype=np.float64, copy=True)
    inner_done = []
    rhos, etas = [], []
    rels = []
    converged = False
    outer = 0
    while True:
        r = residual(x, f)
        nr = math.sqrt(float(np.sum(r * r)))
        rel = nr / res0 if res0 != 0.0 else 0.0
        rels.append(rel)
        if res0 == 0.0 or rel <= tol:
            converged = True
            break
        if outer == max_outer:
            break
        s = pow2_scale(nr, ncells)
        eta_o = max(eta, 0.5 * tol / rel)
        rhat = np.zeros(x.shape, np.float32)
        rhat[INTERIOR] = (r / s).astype(np.float32)
        e = np.zeros(x.shape, np.float32)
        rho = [residual_norm_f32_storage(e, rhat)]
        j = 0
        while True:
            if inner_counts is not None:
                if j == inner_counts[outer]:
                    break
            else:
                if rho[j] <= eta_o * rho[0] or j == max_inner:
                    break
                if j >= stall and rho[j] >= rho[j - stall]:
                    break
            e = sweep_f32(e, rhat)
            j += 1
            rho.append(residual_norm_f32_storage(e, rhat))
        inner_done.append(j)
        rhos.append(rho)
        etas.append(eta_o)
        x[INTERIOR] = interior(x) + s * interior(e).astype(np.float64)
        outer += 1
    return dict(x=x, converged=converged, outer=outer, inner=inner_done,
                hist=rels, res0=res0, sweeps=int(sum(inner_done)), rho=rhos, eta=etas)


def stencil_apply(taps, inp, rhs=None, rhs_coef=0.0, scale=1.0):
    """General constant-offset stencil (Section 2.2, Listing 2 and the
    semantics of stencil.apply stated there): for every interior cell p,

        out(p) = scale * ((...((w0*in[p+o0]) + w1*in[p+o1]) + ...) + c*rhs[p])

    accumulated in tap order; the rhs term is present only when ``rhs`` is
    given. ``taps`` is a sequence of (dx, dy, dz, w) with |d| <= 1.
    Returns the interior values (the halo of the output is not written).
    """
    acc = None
    for dx, dy, dz, w in taps:
        term = w * shifted(inp, dx, dy, dz)
        acc = term if acc is None else acc + term
    if rhs is not None:
        term = rhs_coef * interior(rhs)
        acc = term if acc is None else acc + term
    return scale * acc


def advect_source(u, v, w, tzc1, tzc2, tcx, tcy):
    """Fused three-field advection source term (Section 4.1: the
    Piacsek-Williams scheme, three stencils over three fields fused into one
    region, 63 flops per cell).

    PARITY UNPINNED against the paper: it prints no formula. This is the
    project's definition on a staggered C-grid (u at i+1/2, v at j+1/2,
    w at k+1/2), pinned by the 63-flop count, exact-rational error bounds,
    homogeneity and second-order convergence to the continuous operator.

    For phi in (u, v, w):
      s_phi = (tcx*(Px- - Px+) + tcy*(Py- - Py+)) + (tzc1[k]*Pz- - tzc2[k]*Pz+)
    where each P is phi at the neighbour on that side times the sum of the
    two samples of the advecting velocity straddling that face.
    ``tzc1``/``tzc2`` have one value per interior level k.
    Returns (su, sv, sw) interior arrays.
    """
    def sh(a, di, dj, dk):
        return shifted(a, di, dj, dk)

    nz = u.shape[0] - 2
    t1 = np.asarray(tzc1).reshape(nz, 1, 1)
    t2 = np.asarray(tzc2).reshape(nz, 1, 1)

    def combine(pxm, pxp, pym, pyp, pzm, pzp):
        return (tcx * (pxm - pxp) + tcy * (pym - pyp)) + (t1 * pzm - t2 * pzp)

    su = combine(
        sh(u, -1, 0, 0) * (sh(u, -1, 0, 0) + sh(u, 0, 0, 0)),
        sh(u, 1, 0, 0) * (sh(u, 0, 0, 0) + sh(u, 1, 0, 0)),
        sh(u, 0, -1, 0) * (sh(v, 0, -1, 0) + sh(v, 1, -1, 0)),
        sh(u, 0, 1, 0) * (sh(v, 0, 0, 0) + sh(v, 1, 0, 0)),
        sh(u, 0, 0, -1) * (sh(w, 0, 0, -1) + sh(w, 1, 0, -1)),
        sh(u, 0, 0, 1) * (sh(w, 0, 0, 0) + sh(w, 1, 0, 0)),
    )
    sv = combine(
        sh(v, -1, 0, 0) * (sh(u, -1, 0, 0) + sh(u, -1, 1, 0)),
        sh(v, 1, 0, 0) * (sh(u, 0, 0, 0) + sh(u, 0, 1, 0)),
        sh(v, 0, -1, 0) * (sh(v, 0, -1, 0) + sh(v, 0, 0, 0)),
        sh(v, 0, 1, 0) * (sh(v, 0, 0, 0) + sh(v, 0, 1, 0)),
        sh(v, 0, 0, -1) * (sh(w, 0, 0, -1) + sh(w, 0, 1, -1)),
        sh(v, 0, 0, 1) * (sh(w, 0, 0, 0) + sh(w, 0, 1, 0)),
    )
    sw = combine(
        sh(w, -1, 0, 0) * (sh(u, -1, 0, 0) + sh(u, -1, 0, 1)),
        sh(w, 1, 0, 0) * (sh(u, 0, 0, 0) + sh(u, 0, 0, 1)),
        sh(w, 0, -1, 0) * (sh(v, 0, -1, 0) + sh(v, 0, -1, 1)),
        sh(w, 0, 1, 0) * (sh(v, 0, 0, 0) + sh(v, 0, 0, 1)),
        sh(w, 0, 0, -1) * (sh(w, 0, 0, -1) + sh(w, 0, 0, 0)),
        sh(w, 0, 0, 1) * (sh(w, 0, 0, 0) + sh(w, 0, 0, 1)),
    )
    return su, sv, sw
