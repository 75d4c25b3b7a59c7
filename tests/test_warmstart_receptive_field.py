"""Why a four-layer 3x3x3 network fed only the right-hand side (and the
boundary lift) cannot make a good initial guess at 128^3 -- the reason the
network's input also carries cube means of the right-hand side at larger
scales and the cell's position.

Such a network's output at a cell depends only on the 9x9x9 patch of its
input around that cell. Where that patch of the right-hand side is
(numerically) zero -- far from every source -- it outputs one and the same
value, while the exact solution there varies (the potential of a source
decays like 1/r). The best constant over those cells therefore bounds the
error of every such network from below. The exact discrete solution comes
from the discrete sine transform, which diagonalises the 7-point operator
with a zero Dirichlet boundary."""

import numpy as np
import scipy.fft as sf
from scipy import ndimage

import oracle
import synth

N = 128


def _dst_solve(f):
    """Exact solution of S(u) - 6u = f (zero Dirichlet boundary) on the interior."""
    k = np.arange(1, N + 1)
    lam = 2.0 * np.cos(np.pi * k / (N + 1)) - 2.0
    L = lam[:, None, None] + lam[None, :, None] + lam[None, None, :]
    return sf.idstn(sf.dstn(f, type=1) / L, type=1)


def test_dst_solution_is_the_discrete_solution():
    f = synth.gaussian_sources(N, N, N, 3, 20000)
    u = synth.zeros(N, N, N)
    u[1:-1, 1:-1, 1:-1] = _dst_solve(f[1:-1, 1:-1, 1:-1])
    assert oracle.residual_norm(u, f) <= 1e-10 * np.linalg.norm(f)


def test_error_floor_of_any_9_cubed_receptive_field():
    floors = []
    for seed in (20000, 20001, 20002):
        f = synth.gaussian_sources(N, N, N, synth.random_source_count(seed), seed)[1:-1, 1:-1, 1:-1]
        u = _dst_solve(f)
        far = ndimage.maximum_filter(np.abs(f), size=9) <= 1e-3 * np.abs(f).max()
        uf = u[far]
        floors.append(np.linalg.norm(uf - uf.mean()) / np.linalg.norm(u))
    # most of the volume is far from every source, and there the solution is
    # far from constant: at least ~30% relative L2 error for any such network
    assert min(floors) > 0.25, floors
    print("relative-error floors:", [round(x, 3) for x in floors])
