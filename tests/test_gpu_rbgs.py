"""GPU parity of the red-black Gauss-Seidel sweeps and solves against the
oracle: fields bit for bit (each half-sweep is the Jacobi expression in the
Jacobi operation order, no contraction on either side), norms to relative
1e-13 (summation order only), iteration counts exact unless a norm sits
within rounding of the tolerance."""

import numpy as np
import pytest
import torch

import oracle
import synth
from gpuhelp import dev, empty_like_layout, host, note

pytestmark = pytest.mark.gpu

import paper_2310_01882_amd as ms  # noqa: E402  (fails loudly if not built)

NORM_RTOL = 1e-13
STRADDLE = 1e-10


def _problem(nx, ny, nz, seed, with_f=True):
    u = synth.dirichlet_uniform(nx, ny, nz, seed)
    u[1:-1, 1:-1, 1:-1] = synth.rng(seed + 1).standard_normal((nz, ny, nx))
    f = synth.gaussian_sources(nx, ny, nz, 4, seed + 2) if with_f else None
    return u, f


def _run(u, f, n, dtype=np.float64, pad=(0, 0)):
    du = dev(u.astype(dtype), *pad)
    dt = empty_like_layout(du)
    dt.copy_(du)
    df = dev(f.astype(dtype), *pad) if f is not None else None
    res = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    out = ms.rbgs_sweeps(du, dt, n, f=df, res=res)
    torch.cuda.synchronize()
    assert (out is du) == (n % 2 == 0)
    return host(out), host(res)


TB_VARIANTS = {"columns": "2", "lds": "0", "registers": "3"}


@pytest.mark.parametrize("variant", list(TB_VARIANTS))
@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 3, 4), (64, 8, 8), (65, 17, 9), (130, 9, 20),
                                  (63, 15, 7), (200, 3, 70), (3, 2, 41), (61, 21, 10),
                                  (61, 90, 9)])
@pytest.mark.parametrize("with_f", [True, False])
def test_sweeps_bit_exact_on_ragged_grids(dims, with_f, variant, monkeypatch):
    monkeypatch.setenv("MS_TB_VARIANT", TB_VARIANTS[variant])
    note(f"case: rbgs sweeps {variant} {dims} f={with_f}")
    u, f = _problem(*dims, seed=sum(dims) + 3, with_f=with_f)
    for n in (0, 1, 2, 5):
        got, res = _run(u, f, n)
        want, hist = oracle.rbgs_sweeps(u, f, n)
        assert np.array_equal(got, want), n
        np.testing.assert_allclose(res, hist, rtol=NORM_RTOL, atol=0)


def test_padded_pitch_and_halo_untouched():
    note("case: rbgs padded pitch 70x13x11")
    u, f = _problem(70, 13, 11, 9)
    got, _ = _run(u, f, 3, pad=(5, 3))
    want, _ = oracle.rbgs_sweeps(u, f, 3)
    assert np.array_equal(got, want)
    mask = np.ones_like(u, bool)
    mask[1:-1, 1:-1, 1:-1] = False
    assert np.array_equal(got[mask], u[mask])


def test_fp32_storage_sweeps_bit_exact():
    note("case: rbgs FP32 70x33x20")
    nx, ny, nz = 70, 33, 20
    e = np.zeros((nz + 2, ny + 2, nx + 2), np.float32)
    e[1:-1, 1:-1, 1:-1] = synth.rng(13).standard_normal((nz, ny, nx)).astype(np.float32)
    rh = np.zeros_like(e)
    rh[1:-1, 1:-1, 1:-1] = synth.rng(14).standard_normal((nz, ny, nx)).astype(np.float32)
    got, res = _run(e, rh, 5, dtype=np.float32)
    want = e
    hist = [oracle.residual_norm_f32_storage(want, rh)]
    for _ in range(5):
        want = oracle.rbgs_sweep(want, rh)  # float32 arrays: float32 arithmetic
        hist.append(oracle.residual_norm_f32_storage(want, rh))
    assert want.dtype == np.float32
    assert np.array_equal(got, want)
    np.testing.assert_allclose(res, hist, rtol=NORM_RTOL)


def test_full_size_512cubed_sweeps_bit_exact():
    """512^3 interior, 8 Gaussian sources, zero Dirichlet halo, a non-zero
    start, the benchmark's launch configuration: two sweeps in full."""
    note("case: rbgs 512^3 x 2 sweeps (full compare)")
    n = 512
    f = synth.gaussian_sources(n, n, n, 8, 1)
    u = synth.zeros(n, n, n)
    u[1:-1, 1:-1, 1:-1] = f[1:-1, 1:-1, 1:-1] * 3.0
    got, res = _run(u, f, 2)
    want, hist = oracle.rbgs_sweeps(u, f, 2)
    assert np.array_equal(got, want)
    np.testing.assert_allclose(res, hist, rtol=NORM_RTOL)


def _count_ok(k_gpu, k_or, hist, res0, tol):
    if k_gpu == k_or:
        return True
    near = any(abs(hist[k] / res0 - tol) <= STRADDLE * tol
               for k in (k_or - 1, k_or) if 0 <= k < len(hist))
    return near and abs(k_gpu - k_or) == 1


@pytest.mark.parametrize("dims,tol", [((16, 16, 16), 1e-6), ((24, 20, 12), 1e-8),
                                      ((65, 9, 7), 1e-5), ((1, 1, 1), 1e-12)])
@pytest.mark.parametrize("use_graph", [1, 0])
def test_solve_count_and_field_match_oracle(dims, tol, use_graph):
    note(f"case: rbgs solve {dims} tol {tol} graph {use_graph}")
    u = synth.dirichlet_uniform(*dims, sum(dims))
    f = synth.gaussian_sources(*dims, 6, sum(dims) + 1)
    K, uk, hist, res0, ok = oracle.rbgs_solve(u, f, tol, 200000)
    assert ok
    du = dev(u)
    info = ms.jacobi_solve(du, dev(f), rel_tol=tol, max_sweeps=200000, use_graph=use_graph,
                           check_every=37, want_hist=True, method=ms.MS_METHOD_RBGS)
    assert info.status == ms.MS_OK
    assert _count_ok(info.sweeps, K, hist, res0, tol), (info.sweeps, K)
    assert info.res0 == pytest.approx(res0, rel=1e-13)
    if info.sweeps == K:
        assert np.array_equal(host(du), uk)
        np.testing.assert_allclose(info.hist, hist, rtol=1e-12)


def test_solve_takes_about_half_the_jacobi_sweeps():
    note("case: rbgs vs jacobi sweep counts 48x40x32")
    u = synth.zeros(48, 40, 32)
    f = synth.gaussian_sources(48, 40, 32, 8, 21)
    kj = ms.jacobi_solve(dev(u), dev(f), rel_tol=1e-8).sweeps
    kg = ms.jacobi_solve(dev(u), dev(f), rel_tol=1e-8, method=ms.MS_METHOD_RBGS).sweeps
    note(f"jacobi {kj} sweeps, red-black Gauss-Seidel {kg}")
    assert 0.4 < kg / kj < 0.6


@pytest.mark.parametrize("dims", [(24, 24, 24), (40, 18, 11)])
def test_refined_solve_reaches_1e8_checked_by_the_oracle(dims):
    note(f"case: rbgs refined {dims}")
    u = synth.zeros(*dims)
    f = synth.gaussian_sources(*dims, 8, 8)
    du = dev(u)
    info = ms.jacobi_solve(du, dev(f), precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8,
                           inner_eta=1e-4, method=ms.MS_METHOD_RBGS)
    assert info.status == ms.MS_OK
    x = host(du)
    res0 = oracle.residual_norm(oracle.zero_interior(u), f)
    assert oracle.residual_norm(x, f) / res0 <= 1e-8
    K, xs, _, _, ok = oracle.rbgs_solve(u, f, 1e-10, 500000)
    assert ok
    err = np.max(np.abs(x - xs)) / np.max(np.abs(xs))
    note(f"rbgs refined {dims}: outer {info.outer_iters} sweeps {info.sweeps} "
         f"rel {info.rel_final:.3e} field rel err {err:.3e}")
    assert err < 1e-6


def test_batched_solve_rejects_red_black():
    u = dev(synth.zeros(8, 8, 8))
    f = dev(synth.gaussian_sources(8, 8, 8, 2, 3))
    with pytest.raises(ms.MsError, match="Jacobi sweeps only"):
        ms.jacobi_solve_batched([u], [f], method=ms.MS_METHOD_RBGS)
    work = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(ms.MsError) as e:
        ms.jacobi_solve_batched([u], [f], work=work, method=ms.MS_METHOD_RBGS)
    assert e.value.code == ms.MS_EUNSUPPORTED
