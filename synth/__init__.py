"""Seeded synthetic inputs for the stencil hot path.

This module only draws random numbers and lays them out on halo-padded
grids. It holds none of the method's arithmetic (no stencil, residual,
advection or network step), so both the HIP path and the CPU oracle may be
fed from it.

Grid layout (shared by every producer here): a field over an interior of
``nx * ny * nz`` cells plus a one-cell halo is a C-contiguous float64 array of
shape ``(nz + 2, ny + 2, nx + 2)``; x is the fastest axis and index ``[1, 1, 1]``
is interior cell ``(0, 0, 0)``. This is the column-major Fortran order of the
paper's listings (first index contiguous), written with numpy's reversed axes.

Every generator takes an explicit seed and uses numpy's PCG64, so the same
seed gives the same array on any machine with the same numpy/BLAS build.
Separable pieces are combined with a matrix product; the result is the
definition of the input, not an approximation of another formula.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng",
    "zeros",
    "dirichlet_uniform",
    "gaussian_sources",
    "gaussian_params",
    "sinusoid_field",
    "velocity_fields",
    "tzc_arrays",
    "eigenmode",
    "batch_sizes",
    "padded",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def zeros(nx: int, ny: int, nz: int, dtype=np.float64) -> np.ndarray:
    return np.zeros((nz + 2, ny + 2, nx + 2), dtype=dtype)


def padded(a: np.ndarray, pad_x: int = 0, pad_y: int = 0) -> np.ndarray:
    """Return a strided view of ``a`` whose rows and planes carry extra pitch.

    The view has the same logical shape as ``a`` but the underlying buffer
    has ``pad_x`` unused elements after each x-row and ``pad_y`` unused rows
    after each plane (filled with NaN so a read of the padding shows up).
    """
    nz2, ny2, nx2 = a.shape
    buf = np.full((nz2, ny2 + pad_y, nx2 + pad_x), np.nan, dtype=a.dtype)
    view = buf[:, :ny2, :nx2]
    view[...] = a
    return view


def dirichlet_uniform(nx: int, ny: int, nz: int, seed: int) -> np.ndarray:
    """Halo cells ~ U[0, 1) from ``seed``; interior set to zero."""
    a = rng(seed).random((nz + 2, ny + 2, nx + 2))
    a[1:-1, 1:-1, 1:-1] = 0.0
    return a


def gaussian_params(nx: int, ny: int, nz: int, count: int, seed: int):
    """Draw ``count`` anisotropic Gaussian sources.

    Per source, in this order: centre (cx, cy, cz) ~ U[0, n_a - 1] in
    interior index coordinates; relative widths (wx, wy, wz) ~ U[0.02, 0.1]
    giving sigma_a = w_a * n_a; amplitude A ~ N(0, 1).
    """
    g = rng(seed)
    out = []
    dims = (nx, ny, nz)
    for _ in range(count):
        c = [g.uniform(0.0, n - 1) for n in dims]
        w = [g.uniform(0.02, 0.1) for _ in dims]
        amp = g.standard_normal()
        sig = [wa * n for wa, n in zip(w, dims)]
        out.append((c, sig, amp))
    return out


def gaussian_sources(nx: int, ny: int, nz: int, count: int, seed: int,
                     dtype=np.float64) -> np.ndarray:
    """Right-hand side: sum of ``count`` Gaussian sources on the interior.

    Source s contributes A_s * gx_s(i) * gy_s(j) * gz_s(k), with
    g_a(t) = exp(-(t - c_a)^2 / (2 sigma_a^2)). The halo of the result is 0.
    """
    f = zeros(nx, ny, nz)
    params = gaussian_params(nx, ny, nz, count, seed)
    if not params:
        return f.astype(dtype)
    xs, ys, zs = np.arange(nx), np.arange(ny), np.arange(nz)
    # rows: A_s * (gy_s outer gx_s) flattened; columns: gz_s
    plane = np.empty((len(params), ny * nx))
    zcol = np.empty((nz, len(params)))
    for s, (c, sig, amp) in enumerate(params):
        gx = np.exp(-((xs - c[0]) ** 2) / (2.0 * sig[0] ** 2))
        gy = np.exp(-((ys - c[1]) ** 2) / (2.0 * sig[1] ** 2))
        gz = np.exp(-((zs - c[2]) ** 2) / (2.0 * sig[2] ** 2))
        plane[s] = amp * np.outer(gy, gx).ravel()
        zcol[:, s] = gz
    f[1:-1, 1:-1, 1:-1] = (zcol @ plane).reshape(nz, ny, nx)
    return f.astype(dtype)


def random_source_count(seed: int, lo: int = 1, hi: int = 8) -> int:
    """Number of Gaussian sources for a training/evaluation instance."""
    return int(rng(seed).integers(lo, hi + 1))


def sinusoid_field(nx: int, ny: int, nz: int, seed: int, stagger=(0.0, 0.0, 0.0),
                   modes: int = 16, amp_max: float = 10.0) -> np.ndarray:
    """Smooth periodic field = sum of ``modes`` seeded sinusoids, |phi| <= amp_max.

    Mode m: a_m * sin(2*pi*(kx x/nx + ky y/ny + kz z/nz) + theta_m) with
    integer wave numbers k in [0, 4]^3 (not all zero), theta ~ U[0, 2*pi),
    a ~ U[0, amp_max / modes]. The field is sampled at positions
    (i + sx, j + sy, k + sz) for halo-inclusive indices i in [-1, nx] etc.,
    so a staggered variable passes its offset in ``stagger``.

    sin(P + Q) = sin P cos Q + cos P sin Q with P the (x, y) phase and Q the
    z phase turns the sum into one (nz+2, 2m) x (2m, (ny+2)(nx+2)) product.
    """
    g = rng(seed)
    x = np.arange(-1, nx + 1) + stagger[0]
    y = np.arange(-1, ny + 1) + stagger[1]
    z = np.arange(-1, nz + 1) + stagger[2]
    basis = np.empty((2 * modes, (ny + 2) * (nx + 2)))
    coef = np.empty((nz + 2, 2 * modes))
    for m in range(modes):
        while True:
            k = g.integers(0, 5, size=3)
            if k.any():
                break
        theta = g.uniform(0.0, 2.0 * math.pi)
        a = g.uniform(0.0, amp_max / modes)
        p = 2.0 * math.pi * (k[0] * x[None, :] / nx + k[1] * y[:, None] / ny) + theta
        q = 2.0 * math.pi * k[2] * z / nz
        basis[2 * m] = np.sin(p).ravel()
        basis[2 * m + 1] = np.cos(p).ravel()
        coef[:, 2 * m] = a * np.cos(q)
        coef[:, 2 * m + 1] = a * np.sin(q)
    return (coef @ basis).reshape(nz + 2, ny + 2, nx + 2)


def velocity_fields(nx: int, ny: int, nz: int, seed: int):
    """u, v, w on a staggered C-grid (u at i+1/2, v at j+1/2, w at k+1/2)."""
    u = sinusoid_field(nx, ny, nz, seed * 3 + 0, stagger=(0.5, 0.0, 0.0))
    v = sinusoid_field(nx, ny, nz, seed * 3 + 1, stagger=(0.0, 0.5, 0.0))
    w = sinusoid_field(nx, ny, nz, seed * 3 + 2, stagger=(0.0, 0.0, 0.5))
    return u, v, w


def tzc_arrays(nz: int, seed: int):
    """Per-level vertical coefficients tzc1, tzc2 ~ U[0.5, 2], length nz."""
    g = rng(seed)
    return g.uniform(0.5, 2.0, nz), g.uniform(0.5, 2.0, nz)


def eigenmode(nx: int, ny: int, nz: int) -> np.ndarray:
    """prod_a sin(pi (idx_a + 1) / (n_a + 1)) on the interior, zero halo."""
    sx = np.sin(np.pi * (np.arange(nx) + 1) / (nx + 1))
    sy = np.sin(np.pi * (np.arange(ny) + 1) / (ny + 1))
    sz = np.sin(np.pi * (np.arange(nz) + 1) / (nz + 1))
    u = zeros(nx, ny, nz)
    u[1:-1, 1:-1, 1:-1] = sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    return u


def batch_sizes(count: int, seed: int, lo: int = 32, hi: int = 256):
    """``count`` (nx, ny, nz) triples, each axis round(exp(U[ln lo, ln hi]))."""
    g = rng(seed)
    out = []
    for _ in range(count):
        dims = tuple(int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))
                     for _ in range(3))
        out.append(dims)
    return out
