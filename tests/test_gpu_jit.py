"""GPU parity of runtime-compiled stencil programs against the interpreter
in the oracle: bit for bit (each operation rounded once, in the text's
order, on both sides), for the Jacobi update, the three-output advection
region and seeded random programs, in FP64 and FP32, on ragged and padded
grids; and against the hand-written kernels on the benchmark grids."""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpuhelp import dev, empty_like_layout, host, note
from oracle import stencil_lang as sl
from stencil_programs import JACOBI, advection, random_program

pytestmark = pytest.mark.gpu

import paper_2310_01882_amd as ms  # noqa: E402


def _field(nx, ny, nz, seed, dtype=np.float64):
    a = synth.dirichlet_uniform(nx, ny, nz, seed)
    a[1:-1, 1:-1, 1:-1] = synth.rng(seed + 1).standard_normal((nz, ny, nx))
    return a.astype(dtype)


def _run(j, arrays, params=(), profiles=(), pad=(0, 0)):
    ins = [dev(a, *pad) for a in arrays]
    tdt = torch.float64 if arrays[0].dtype == np.float64 else torch.float32
    outs = [empty_like_layout(ins[0]) for _ in j.outputs]
    profs = [torch.from_numpy(np.ascontiguousarray(p, dtype=arrays[0].dtype)).cuda()
             for p in profiles]
    assert all(t.dtype == tdt for t in profs)
    j.apply(ins, outs, params, profs)
    torch.cuda.synchronize()
    return [host(o) for o in outs]


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 3, 4), (64, 4, 8), (65, 17, 9), (130, 9, 20),
                                  (63, 5, 41)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_jacobi_program_bit_exact(dims, dtype):
    note(f"case: jit jacobi {dims} {np.dtype(dtype).name}")
    u = _field(*dims, sum(dims), dtype)
    f = synth.gaussian_sources(*dims, 3, 7).astype(dtype)
    j = ms.JitStencil(JACOBI, torch.float64 if dtype == np.float64 else torch.float32)
    (got,) = _run(j, [u, f])
    (want,) = sl.run(JACOBI, [u, f], dtype=dtype)
    assert np.array_equal(got[1:-1, 1:-1, 1:-1], want)
    assert np.all(np.isnan(got[0]))  # the halo of the output is not written


def test_advection_program_bit_exact_and_equal_to_the_kernel():
    note("case: jit advection 70x20x9 padded")
    nx, ny, nz = 70, 20, 9
    u, v, w = synth.velocity_fields(nx, ny, nz, 3)
    t1, t2 = synth.tzc_arrays(nz, 4)
    j = ms.JitStencil(advection())
    got = _run(j, [u, v, w], [0.25, 0.5], [t1, t2], pad=(3, 2))
    want = oracle.advect_source(u, v, w, t1, t2, 0.25, 0.5)
    for g, w_ in zip(got, want):
        assert np.array_equal(g[1:-1, 1:-1, 1:-1], w_)


@pytest.mark.parametrize("seed", range(8))
def test_random_programs_bit_exact(seed):
    dtype = np.float64 if seed % 2 == 0 else np.float32
    note(f"case: jit random program seed {seed} {np.dtype(dtype).name}")
    text = random_program(seed)
    dims = (37, 11, 6)
    arrays = [_field(*dims, 100 * seed + n, dtype) for n in range(3)]
    params = [0.75, -1.5]
    prof = [np.linspace(0.5, 2.0, dims[2])]
    j = ms.JitStencil(text, torch.float64 if dtype == np.float64 else torch.float32)
    got = _run(j, arrays, params, prof)
    want = sl.run(text, arrays, params, prof, dtype=dtype)
    for g, w_ in zip(got, want):
        assert np.array_equal(g[1:-1, 1:-1, 1:-1], w_, equal_nan=True)


def test_full_size_jacobi_program_equals_the_sweep_kernel():
    """512^3, the sweep benchmark's input: the compiled program and one
    hand-written sweep give the same field."""
    note("case: jit jacobi 512^3 vs jacobi_sweeps")
    n = 512
    f_h = synth.gaussian_sources(n, n, n, 8, 1)
    u_h = synth.zeros(n, n, n)
    u_h[1:-1, 1:-1, 1:-1] = 3.0 * f_h[1:-1, 1:-1, 1:-1]
    u, f = ms.field_from(u_h), ms.field_from(f_h)
    j = ms.JitStencil(JACOBI)
    out = ms.alloc_field(n, n, n)
    j.apply([u, f], [out])
    tmp = ms.field_from(u_h)
    ref = ms.jacobi_sweeps(ms.field_from(u_h), tmp, 1, f=f)
    torch.cuda.synchronize()
    assert torch.equal(out[1:-1, 1:-1, 1:-1], ref[1:-1, 1:-1, 1:-1])


def test_full_size_advection_program_equals_the_advection_kernel():
    note("case: jit advection 512x512x256 vs advect_source")
    nx, ny, nz = 512, 512, 256
    u, v, w = (ms.field_from(a) for a in synth.velocity_fields(nx, ny, nz, 2))
    t1, t2 = (torch.from_numpy(a).cuda() for a in synth.tzc_arrays(nz, 3))
    j = ms.JitStencil(advection())
    outs = [ms.alloc_field(nx, ny, nz) for _ in range(3)]
    j.apply([u, v, w], outs, [0.25, 0.25], [t1, t2])
    refs = [ms.alloc_field(nx, ny, nz) for _ in range(3)]
    ms.advect_source(u, v, w, t1, t2, 0.25, 0.25, *refs)
    torch.cuda.synchronize()
    for a, b in zip(outs, refs):
        assert torch.equal(a[1:-1, 1:-1, 1:-1], b[1:-1, 1:-1, 1:-1])


def test_argument_errors():
    j = ms.JitStencil(JACOBI)
    u = dev(_field(8, 8, 8, 1))
    f = dev(_field(8, 8, 8, 2))
    o = empty_like_layout(u)
    with pytest.raises(ms.MsError) as e:
        j.apply([u], [o])  # one field short
    assert e.value.code == ms.MS_EINVAL
    with pytest.raises(ms.MsError, match="overlaps"):
        j.apply([u, f], [u])


def _vec_ok(ts):
    import ctypes
    arr = (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])
    out = ms.Tuning()
    g = ms.grid_of(ts[0])
    code = ms.MS_F64 if ts[0].dtype == torch.float64 else ms.MS_F32
    assert ms.lib.ms_sweep_shape(ctypes.byref(g), code, arr, len(ts), ctypes.byref(out)) == 0
    return out.vec_ok


@pytest.mark.parametrize("dtype,dims", [(np.float64, (300, 7, 6)), (np.float64, (128, 5, 9)),
                                        (np.float32, (600, 5, 4)), (np.float32, (256, 3, 11))])
@pytest.mark.parametrize("which", ["jacobi", "random"])
def test_vector_kernel_on_aligned_fields_with_ragged_tails(dtype, dims, which, monkeypatch):
    """Aligned fields take the vector kernel (2 FP64 / 4 FP32 cells per lane)
    for whole 64V-column tiles and the scalar kernel for the remaining
    columns; both together are bit-exact, and equal to the scalar kernel
    alone."""
    note(f"case: jit vector {which} {dims} {np.dtype(dtype).name}")
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    if which == "jacobi":
        text = JACOBI
        arrays = [_field(*dims, 5, dtype), synth.gaussian_sources(*dims, 3, 6).astype(dtype)]
        params, prof = [], []
    else:
        text = random_program(11 if dtype == np.float64 else 12)
        arrays = [_field(*dims, 40 + n, dtype) for n in range(3)]
        params, prof = [0.75, -1.5], [np.linspace(0.5, 2.0, dims[2])]
    ins = [ms.field_from(a, tdt) for a in arrays]
    j = ms.JitStencil(text, tdt)
    outs = [ms.alloc_field(*dims, tdt) for _ in j.outputs]
    assert _vec_ok(ins + outs) == (2 if dtype == np.float64 else 4)
    profs = [torch.from_numpy(np.ascontiguousarray(p, dtype=dtype)).cuda() for p in prof]
    j.apply(ins, outs, params, profs)
    want = sl.run(text, arrays, params, prof, dtype=dtype)
    for o, w_ in zip(outs, want):
        assert np.array_equal(host(o)[1:-1, 1:-1, 1:-1], w_, equal_nan=True)
    monkeypatch.setenv("MS_JIT_SCALAR", "1")
    outs2 = [ms.alloc_field(*dims, tdt) for _ in j.outputs]
    j.apply(ins, outs2, params, profs)
    torch.cuda.synchronize()
    for a, b in zip(outs, outs2):
        assert torch.equal(a[1:-1, 1:-1, 1:-1], b[1:-1, 1:-1, 1:-1])


@pytest.mark.parametrize("text,params,nprof", [
    ("param c; out o = c * 2;", [1.5], 0),
    ("profile t; out o = t - 1;", [], 1),
    ("field a; out o = a[0,0,1] - a[0,0,-1];", [], 0),
    ("field a, b; param p; out o = p; out q = b[1,1,1] / (2 + a * a);", [0.25], 0),
])
@pytest.mark.parametrize("aligned", [True, False])
def test_programs_without_some_kinds_of_inputs(text, params, nprof, aligned):
    """Programs with no fields, only a profile, z offsets only, or an output
    that reads nothing: both kernels (aligned fields take the vector one)."""
    note(f"case: jit {text!r} aligned={aligned}")
    dims = (300, 5, 7)
    prog = sl.parse(text)
    arrays = [_field(*dims, 60 + n) for n in range(len(prog["fields"]))]
    prof = [np.linspace(0.5, 2.0, dims[2])] * nprof
    j = ms.JitStencil(text)
    if aligned:
        ins = [ms.field_from(a) for a in arrays]
        outs = [ms.alloc_field(*dims) for _ in j.outputs]
    else:
        ins = [dev(a) for a in arrays]
        outs = [empty_like_layout(dev(synth.zeros(*dims))) for _ in j.outputs]
    profs = [torch.from_numpy(np.ascontiguousarray(p)).cuda() for p in prof]
    j.apply(ins, outs, params, profs)
    torch.cuda.synchronize()
    want = sl.run(text, arrays, params, prof, interior_shape=dims[::-1])
    for o, w_ in zip(outs, want):
        assert np.array_equal(host(o)[1:-1, 1:-1, 1:-1], w_)
