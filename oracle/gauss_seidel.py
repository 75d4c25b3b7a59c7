"""Red-black Gauss-Seidel for the 7-point Poisson problem.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading (Section 4.1 and Listing 1): the evaluation's Laplace benchmark is
called Gauss-Seidel and its loop updates the field in place, which in
lexicographic order is a sequential recurrence. This reading takes the
data-parallel ordering of Gauss-Seidel: colour every interior cell by the
parity of i + j + k (red: even, black: odd); a sweep first updates every red
cell from its six neighbours (all black, not yet changed), then every black
cell from its six neighbours (all red, just updated). Each update is the
Jacobi expression in the Jacobi operation order, (S - f) * fl(1/6), so a
cell of one colour changes exactly as a Jacobi update of the current field
would change it. The residual and the relative-residual stopping rule are
the Jacobi solve's (relative to the zero interior's residual), tested after
every sweep.
"""

from __future__ import annotations

import numpy as np

from .stencil import INTERIOR, jacobi_sweep, residual_norm, zero_interior


def red_mask(u):
    """Boolean (nz, ny, nx) array: True where i + j + k is even (interior
    index coordinates)."""
    nz, ny, nx = (s - 2 for s in u.shape)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (i + j + k) % 2 == 0


def rbgs_half(u, f, red: bool):
    """Update the cells of one colour from the current field; the other
    colour and the halo are copied."""
    upd = jacobi_sweep(u, f)
    out = u.copy()
    m = red_mask(u) if red else ~red_mask(u)
    out[INTERIOR][m] = upd[INTERIOR][m]
    return out


def rbgs_sweep(u, f=None):
    """One red-black sweep: red half, then black half."""
    return rbgs_half(rbgs_half(u, f, True), f, False)


def rbgs_sweeps(u0, f, n: int):
    """Exactly ``n`` sweeps. Returns (u_n, hist), hist[k] = ||r(u_k)||,
    k = 0..n."""
    u = u0.copy()
    hist = [residual_norm(u, f)]
    for _ in range(n):
        u = rbgs_sweep(u, f)
        hist.append(residual_norm(u, f))
    return u, hist


def rbgs_solve(u0, f, tol: float, max_sweeps: int):
    """Red-black Gauss-Seidel to a relative residual: K = the smallest
    k >= 0 with ||r(u_k)|| / ||r(u^0)|| <= tol, u^0 = u0 with its interior
    zeroed (the Jacobi solve's rule). Returns (K, u_K, hist, res0, ok)."""
    res0 = residual_norm(zero_interior(u0), f)
    u = np.array(u0, copy=True)
    hist = []
    k = 0
    while True:
        r = residual_norm(u, f)
        hist.append(r)
        if res0 == 0.0 or r / res0 <= tol:
            return k, u, hist, res0, True
        if k == max_sweeps:
            return k, u, hist, res0, False
        u = rbgs_sweep(u, f)
        k += 1
