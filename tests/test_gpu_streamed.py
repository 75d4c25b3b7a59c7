"""Jacobi sweeps on a field held in host memory, streamed through the device
in z slabs: every value bit-identical to the oracle's sweeps, for slab sizes
and sweeps per pass that do and do not divide the field, FP64 and FP32."""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpuhelp import note

pytestmark = pytest.mark.gpu

import paper_2310_01882_amd as ms  # noqa: E402


def _host(a, pin=True):
    t = torch.from_numpy(np.array(a))  # a copy of its own
    return t.pin_memory() if pin else t


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("dims,T,S,n", [((20, 9, 13), 3, 4, 7), ((33, 7, 10), 4, 7, 8),
                                        ((16, 16, 16), 1, 5, 3), ((9, 5, 6), 8, 2, 10),
                                        ((70, 12, 21), 5, 64, 11), ((8, 8, 1), 2, 1, 3)])
def test_streamed_sweeps_are_bit_exact(dims, T, S, n, dtype):
    note(f"case: streamed {dims} T={T} S={S} n={n} {np.dtype(dtype).name}")
    u = synth.dirichlet_uniform(*dims, sum(dims))
    u[1:-1, 1:-1, 1:-1] = synth.rng(7).standard_normal(dims[::-1])
    f = synth.gaussian_sources(*dims, 3, 8)
    u, f = u.astype(dtype), f.astype(dtype)
    hu, ht, hf = _host(u), _host(u), _host(f)
    out = ms.jacobi_sweeps_streamed(hu, ht, n, f=hf, sweeps_per_pass=T, slab_planes=S)
    want = u
    for _ in range(n):
        want = oracle.jacobi_sweep(want, f) if dtype == np.float64 else oracle.sweep_f32(want, f)
    assert np.array_equal(out.numpy(), want)


def test_streamed_equals_device_sweeps_at_size_and_without_f():
    note("case: streamed 256^2 x 128 vs jacobi_sweeps")
    nx, ny, nz = 256, 256, 128
    u = synth.dirichlet_uniform(nx, ny, nz, 3)
    hu, ht = _host(u), _host(u)
    out = ms.jacobi_sweeps_streamed(hu, ht, 20, sweeps_per_pass=8, slab_planes=48)
    du, dt = torch.from_numpy(u).cuda(), torch.from_numpy(u).cuda()
    ref = ms.jacobi_sweeps(du, dt, 20)
    torch.cuda.synchronize()
    assert torch.equal(out, ref.cpu())
    # pageable host memory works too (copies do not overlap)
    hu2, ht2 = _host(u, pin=False), _host(u, pin=False)
    out2 = ms.jacobi_sweeps_streamed(hu2, ht2, 20, sweeps_per_pass=8, slab_planes=48)
    assert torch.equal(out2, ref.cpu())
