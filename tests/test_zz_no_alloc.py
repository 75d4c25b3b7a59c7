"""The sweep entry point that allocates nothing (jacobi_sweeps_noalloc),
called through the C ABI and compared with jacobi_sweeps_tb on the same
inputs: fields and residual norms bit-identical, on two calls in a row, the
second on a smaller grid (the fixed scratch array keeps the first call's
partials, which the second must not see)."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from gpuhelp import host, note

pytestmark = pytest.mark.gpu

import paper_2310_01882_amd as ms  # noqa: E402


def _problem(nx, ny, nz, seed, dtype):
    u = synth.dirichlet_uniform(nx, ny, nz, seed)
    u[1:-1, 1:-1, 1:-1] = synth.rng(seed + 1).standard_normal((nz, ny, nx))
    f = synth.gaussian_sources(nx, ny, nz, 3, seed + 2)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    return u.astype(npdt), f.astype(npdt)


def _run(entry, u_h, f_h, n, tb, dtype):
    du, dt, df = (ms.field_from(a, dtype) for a in (u_h, u_h, f_h))
    res = torch.full((n + 1,), float("nan"), dtype=torch.float64, device="cuda")
    g = ms.grid_of(du)
    code = ms.MS_F64 if dtype == torch.float64 else ms.MS_F32
    s = ms._stream()
    if entry == "noalloc":
        rc = ms.lib.jacobi_sweeps_noalloc(ctypes_ref(g), code, ms._ptr(du), ms._ptr(dt),
                                          ms._ptr(df), n, tb, ms._ptr(res), s)
    else:
        work = ms.jacobi_sweeps_workspace(du)
        rc = ms.lib.jacobi_sweeps_tb(ctypes_ref(g), code, ms._ptr(du), ms._ptr(dt), ms._ptr(df),
                                     n, tb, ms._ptr(res), ms._ptr(work), work.numel(), s)
    assert rc == ms.MS_OK, ms.last_error()
    torch.cuda.synchronize()
    passes = n if tb == 1 else n // 2 + n % 2
    out = du if passes % 2 == 0 else dt
    return host(out), host(res)


def ctypes_ref(g):
    return ctypes.byref(g)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("tb", [1, 2])
def test_noalloc_matches_the_workspace_entry_point_on_two_calls(dtype, tb):
    assert ms.lib.jacobi_sweeps_noalloc_scratch_bytes() >= \
        ms.lib.jacobi_sweeps_workspace_bytes(ctypes_ref(ms.Grid(8, 8, 8, 0, 10, 100)))
    cases = [((70, 45, 33), 7), ((19, 11, 6), 5)]  # second call: a smaller grid
    for (nx, ny, nz), n in cases:
        note(f"case: noalloc {nx}x{ny}x{nz} n={n} tb={tb} {dtype}")
        u_h, f_h = _problem(nx, ny, nz, nx, dtype)
        got, got_res = _run("noalloc", u_h, f_h, n, tb, dtype)
        want, want_res = _run("workspace", u_h, f_h, n, tb, dtype)
        assert np.array_equal(got, want)
        assert np.array_equal(got_res, want_res)
        assert np.all(np.isfinite(got_res))
        if dtype == torch.float64:
            traj = u_h
            for _ in range(n):
                traj = oracle.jacobi_sweep(traj, f_h)
            assert np.array_equal(got, traj)


def test_noalloc_python_binding_and_rejections():
    u_h, f_h = _problem(24, 20, 16, 5, torch.float64)
    du, dt, df = (ms.field_from(a) for a in (u_h, u_h, f_h))
    res = torch.zeros(5, dtype=torch.float64, device="cuda")
    out = ms.jacobi_sweeps_noalloc(du, dt, 4, f=df, res=res, temporal_block=2)
    torch.cuda.synchronize()
    want = u_h
    for _ in range(4):
        want = oracle.jacobi_sweep(want, f_h)
    assert np.array_equal(host(out), want)
    with pytest.raises(ms.MsError):
        ms.jacobi_sweeps_noalloc(du, dt, 4, f=df, temporal_block=3)
    with pytest.raises(ms.MsError):
        ms.jacobi_sweeps_noalloc(du, du, 2, f=df)
