"""Fields with more than 2^31 elements (int64 addressing throughout): a
1030 x 1030 x 2048 FP64 grid (2.18e9 elements with the halo, 17.4 GB a
field). Sampled cells of one sweep, of two fused sweeps and of one
red-black Gauss-Seidel sweep are recomputed by the oracle on the cells'
neighbourhoods; the residual norm of a constant right-hand side has a
closed form."""

import math

import numpy as np
import pytest
import torch

import oracle
from gpuhelp import note

pytestmark = pytest.mark.gpu

import paper_2310_01882_amd as ms  # noqa: E402

NX, NY, NZ = 1030, 1030, 2048


@pytest.fixture(scope="module")
def big():
    note(f"case: max-size grid {NX}x{NY}x{NZ} ({(NX + 2) * (NY + 2) * (NZ + 2) / 1e9:.2f}e9 "
         "elements a field)")
    g = torch.Generator(device="cuda").manual_seed(5)
    u = ms.alloc_field(NX, NY, NZ)
    u.copy_(torch.rand(u.shape, dtype=torch.float64, device="cuda", generator=g))
    f = ms.alloc_field(NX, NY, NZ)
    f.copy_(torch.rand(f.shape, dtype=torch.float64, device="cuda", generator=g) - 0.5)
    assert u.numel() > 2 ** 31
    yield u, f
    del u, f
    torch.cuda.empty_cache()


def _samples(seed, count, margin):
    """Cells near the far end of the field (offsets above 2^31), at least
    `margin` cells from the boundary, plus corner cells when margin is 0."""
    rg = np.random.Generator(np.random.PCG64(seed))
    pts = [(NX - 1, NY - 1, NZ - 1), (0, 0, 0), (NX // 2, NY - 1, NZ - 2)] if margin == 0 else []
    while len(pts) < count:
        pts.append((int(rg.integers(margin, NX - margin)), int(rg.integers(margin, NY - margin)),
                    int(rg.integers(NZ - 64, NZ - margin))))
    return pts


def _block(t, i, j, k, lo, hi):
    """The halo-padded neighbourhood of interior cells [i-lo, i+hi] x
    [j-lo', ...] (lo, hi: per-axis (x, y, z) extents) as a grid of its own;
    returns it and the centre's index. Cells beyond the field's own halo are
    zero (they only ever sit in the block's halo)."""
    shape = tuple(lo[a] + hi[a] + 3 for a in (2, 1, 0))
    blk = np.zeros(shape)
    c = (k, j, i)
    src, dst = [], []
    for ax, n in zip((2, 1, 0), (NZ, NY, NX)):
        start = c[2 - ax] - lo[ax]  # halo-inclusive index of the block's first plane
        s0, s1 = max(start, 0), min(start + shape[2 - ax], n + 2)
        src.append(slice(s0, s1))
        dst.append(slice(s0 - start, s1 - start))
    blk[tuple(dst)] = t[tuple(src)].cpu().numpy()
    return blk, (lo[2] + 1, lo[1] + 1, lo[0] + 1)


def test_sweeps_at_max_size_match_the_oracle_on_samples(big):
    u, f = big
    a, tmp = ms.alloc_field(NX, NY, NZ), ms.alloc_field(NX, NY, NZ)
    a.copy_(u)  # u itself is kept for the samples
    tmp.copy_(u)
    one = ms.jacobi_sweeps(a, tmp, 1, f=f)
    torch.cuda.synchronize()
    for (i, j, k) in _samples(1, 40, 0):
        (bu, c), (bf, _) = (_block(t, i, j, k, (1, 1, 1), (1, 1, 1)) for t in (u, f))
        want = oracle.jacobi_sweep(bu, bf)[c]
        assert one[k + 1, j + 1, i + 1].item() == want, (i, j, k)
    del one, a, tmp
    torch.cuda.empty_cache()


def test_two_sweeps_per_pass_and_red_black_at_max_size(big):
    u, f = big
    a, b = ms.alloc_field(NX, NY, NZ), ms.alloc_field(NX, NY, NZ)
    a.copy_(u)
    b.copy_(u)
    two = ms.jacobi_sweeps(a, b, 2, f=f, temporal_block=2)
    torch.cuda.synchronize()
    for (i, j, k) in _samples(2, 20, 3):
        (bu, c), (bf, _) = (_block(t, i, j, k, (2, 2, 2), (2, 2, 2)) for t in (u, f))
        want = oracle.jacobi_sweep(oracle.jacobi_sweep(bu, bf), bf)[c]
        assert two[k + 1, j + 1, i + 1].item() == want, (i, j, k)
    a.copy_(u)
    b.copy_(u)
    gs = ms.rbgs_sweeps(a, b, 1, f=f)
    torch.cuda.synchronize()
    for (i, j, k) in _samples(3, 20, 3):
        # the block's first interior cell must have an even i + j + k so
        # that its colouring is the field's: one more x layer when odd
        lo = (2 + (i + j + k) % 2, 2, 2)
        (bu, c), (bf, _) = (_block(t, i, j, k, lo, (2, 2, 2)) for t in (u, f))
        want = oracle.rbgs_sweep(bu, bf)[c]
        assert gs[k + 1, j + 1, i + 1].item() == want, (i, j, k)
    del a, b, two, gs
    torch.cuda.empty_cache()


def test_residual_norm_closed_form_at_max_size():
    """u = 0 (halo too), f = c: r = f everywhere, ||r|| = c sqrt(N)."""
    c = 0.375
    u = ms.alloc_field(NX, NY, NZ)
    f = ms.alloc_field(NX, NY, NZ, fill=c)
    r = ms.residual_norm(u, f)
    assert r == pytest.approx(c * math.sqrt(NX * NY * NZ), rel=1e-12)
    del u, f
    torch.cuda.empty_cache()
