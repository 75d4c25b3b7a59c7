"""GPU parity of the 7-point sweeps and the residual norm against the oracle.

Fields must match bit for bit (same operation order, no contraction on
either side). Norms differ only by summation order: relative 1e-13."""

import math

import numpy as np
import pytest
import torch

import oracle
import synth
from gpuhelp import dev, empty_like_layout, host, note

pytestmark = pytest.mark.gpu

import paper_2310_01882_amd as ms  # noqa: E402  (fails loudly if not built)

NORM_RTOL = 1e-13


def _problem(nx, ny, nz, seed, with_f=True, random_interior=True):
    u = synth.dirichlet_uniform(nx, ny, nz, seed)
    if random_interior:
        u[1:-1, 1:-1, 1:-1] = synth.rng(seed + 1).standard_normal((nz, ny, nx))
    f = synth.gaussian_sources(nx, ny, nz, 4, seed + 2) if with_f else None
    return u, f


def _run_sweeps(u, f, n, pad=(0, 0), dtype=np.float64):
    du = dev(u.astype(dtype), *pad)
    dt = empty_like_layout(du)
    dt.copy_(du)  # same Dirichlet halo in both buffers
    df = dev(f.astype(dtype), *pad) if f is not None else None
    res = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    out = ms.jacobi_sweeps(du, dt, n, f=df, res=res)
    torch.cuda.synchronize()
    return host(out), host(res)


def test_config0_64cubed_100_sweeps_bit_exact():
    """64^3 interior, Dirichlet halo ~U[0,1] (seed 0), zero interior, f = 0,
    exactly 100 sweeps: the field and the 101 residuals."""
    note("case: 64^3 x 100 sweeps, seed 0")
    u0 = synth.dirichlet_uniform(64, 64, 64, 0)
    got, res = _run_sweeps(u0, None, 100)
    want, hist = oracle.jacobi_sweeps(u0, None, 100)
    assert np.array_equal(got, want)
    np.testing.assert_allclose(res, hist, rtol=NORM_RTOL, atol=0)


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 3, 4), (65, 17, 9), (130, 33, 5), (64, 16, 4),
                                  (63, 15, 7), (200, 3, 70)])
@pytest.mark.parametrize("with_f", [True, False])
def test_ragged_grids_bit_exact(dims, with_f):
    note(f"case: sweeps {dims} f={with_f}")
    u, f = _problem(*dims, seed=sum(dims), with_f=with_f)
    for n in (1, 4):
        got, res = _run_sweeps(u, f, n)
        want, hist = oracle.jacobi_sweeps(u, f, n)
        assert np.array_equal(got, want), (dims, n)
        np.testing.assert_allclose(res, hist, rtol=NORM_RTOL, atol=1e-300)


def test_padded_pitch_bit_exact():
    note("case: padded pitch 37x21x11 pad (5, 3)")
    u, f = _problem(37, 21, 11, 5)
    got, res = _run_sweeps(u, f, 3, pad=(5, 3))
    want, hist = oracle.jacobi_sweeps(u, f, 3)
    assert np.array_equal(got, want)
    np.testing.assert_allclose(res, hist, rtol=NORM_RTOL)


def test_halo_untouched_and_zero_sweeps():
    u, f = _problem(20, 10, 6, 8)
    got, res = _run_sweeps(u, f, 0)
    assert np.array_equal(got, u)
    assert res[0] == pytest.approx(oracle.residual_norm(u, f), rel=NORM_RTOL)


def test_fp32_storage_sweeps_bit_exact():
    note("case: FP32 sweeps 70x33x20")
    nx, ny, nz = 70, 33, 20
    e = np.zeros((nz + 2, ny + 2, nx + 2), np.float32)
    e[1:-1, 1:-1, 1:-1] = synth.rng(3).standard_normal((nz, ny, nx)).astype(np.float32)
    rh = np.zeros_like(e)
    rh[1:-1, 1:-1, 1:-1] = synth.rng(4).standard_normal((nz, ny, nx)).astype(np.float32)
    got, res = _run_sweeps(e, rh, 5, dtype=np.float32)
    want = e
    hist = [oracle.residual_norm_f32_storage(want, rh)]
    for _ in range(5):
        want = oracle.sweep_f32(want, rh)
        hist.append(oracle.residual_norm_f32_storage(want, rh))
    assert np.array_equal(got, want)
    np.testing.assert_allclose(res, hist, rtol=NORM_RTOL)


@pytest.mark.parametrize("dims", [(1, 1, 1), (33, 18, 7), (128, 64, 32)])
def test_residual_norm_matches(dims):
    u, f = _problem(*dims, seed=11)
    for ff in (f, None):
        got = ms.residual_norm(dev(u), dev(ff) if ff is not None else None)
        assert got == pytest.approx(oracle.residual_norm(u, ff), rel=NORM_RTOL)
    # FP32 field: FP64 accumulation of exactly widened values
    u32 = u.astype(np.float32)
    f32 = f.astype(np.float32)
    got = ms.residual_norm(dev(u32), dev(f32))
    assert got == pytest.approx(oracle.residual_norm_f32_storage(u32, f32), rel=NORM_RTOL)


def test_residual_norm_is_deterministic():
    u, f = _problem(96, 80, 40, 12)
    du, df = dev(u), dev(f)
    vals = {ms.residual_norm(du, df) for _ in range(5)}
    assert len(vals) == 1


def test_linear_field_fixed_point_at_size():
    note("case: linear fixed point 256x256x128")
    nx, ny, nz = 256, 256, 128
    k, j, i = np.meshgrid(np.arange(-1, nz + 1), np.arange(-1, ny + 1), np.arange(-1, nx + 1),
                          indexing="ij")
    u = (3.0 + 2 * i - 5 * j + 7 * k).astype(np.float64)
    got, res = _run_sweeps(u, None, 10)
    assert np.array_equal(got, u)
    assert np.all(res == 0.0)


def test_eigenmode_decay_on_gpu():
    nx, ny, nz = 96, 80, 72
    u0 = synth.eigenmode(nx, ny, nz)
    rho = (math.cos(math.pi / (nx + 1)) + math.cos(math.pi / (ny + 1))
           + math.cos(math.pi / (nz + 1))) / 3.0
    got, res = _run_sweeps(u0, None, 50)
    assert np.max(np.abs(got - rho ** 50 * u0)) <= 8 * 50 * 2.0 ** -53
    for k in (0, 10, 50):
        assert res[k] / res[0] == pytest.approx(rho ** k, rel=1e-9)


GEOMETRIES = (
    [{"MS_SWEEP_VARIANT": "0", "MS_SWEEP_ROWS": r} for r in ("4", "8")]
    + [{"MS_SWEEP_VARIANT": "1", "MS_SWEEP_VEC": v, "MS_SWEEP_ROWS": r, "MS_SWEEP_WX": w}
       for v in ("1", "2", "4") for r in ("2", "4", "8") for w in ("1", "2", "4")]
)


@pytest.mark.parametrize("geom", GEOMETRIES, ids=lambda g: "-".join(g.values()))
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_every_tile_geometry_is_bit_exact(geom, dtype, monkeypatch):
    """Every tile shape the tuner may pick gives the oracle's bits, on aligned
    fields (vector lanes) and on ragged extents."""
    for key, val in geom.items():
        monkeypatch.setenv(key, val)
    monkeypatch.setenv("MS_SWEEP_ZC", "5")
    for dims in ((130, 37, 9), (64, 16, 8), (5, 3, 2), (300, 9, 11)):
        u, f = _problem(*dims, seed=dims[0])
        u, f = u.astype(dtype), f.astype(dtype)
        du, dt, df = ms.field_from(u), ms.field_from(u), ms.field_from(f)
        res = torch.zeros(4, dtype=torch.float64, device="cuda")
        out = ms.jacobi_sweeps(du, dt, 3, f=df, res=res)
        want = u
        hist = []
        for _ in range(3):
            if dtype == np.float64:
                hist.append(oracle.residual_norm(want, f))
                want = oracle.jacobi_sweep(want, f)
            else:
                hist.append(oracle.residual_norm_f32_storage(want, f))
                want = oracle.sweep_f32(want, f)
        assert np.array_equal(host(out), want), (geom, dims)
        np.testing.assert_allclose(host(res)[:3], hist, rtol=NORM_RTOL)


TB_VARIANTS = {"columns": "2", "lds": "0", "registers": "3"}


@pytest.mark.parametrize("variant", list(TB_VARIANTS))
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("dims", [(64, 8, 9), (130, 37, 11), (5, 3, 2), (1, 1, 1), (65, 17, 40),
                                  (200, 9, 3), (61, 21, 10), (121, 41, 17),
                                  (70, 95, 6)])
def test_temporal_blocking_is_bit_identical_to_plain_sweeps(dims, dtype, variant, monkeypatch):
    """Two sweeps fused per pass, in both kernel layouts: the same fields and
    norms as the oracle's plain sweeps, for even and odd sweep counts."""
    monkeypatch.setenv("MS_TB_VARIANT", TB_VARIANTS[variant])
    note(f"case: tb2 {variant} {dims} {dtype.__name__}")
    u, f = _problem(*dims, seed=3 * dims[0] + dims[2])
    u, f = u.astype(dtype), f.astype(dtype)
    for n in (1, 2, 3, 4, 7):
        du, dt, df = ms.field_from(u), ms.field_from(u), ms.field_from(f)
        res = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
        out = ms.jacobi_sweeps(du, dt, n, f=df, res=res, temporal_block=2)
        want, hist = u, []
        for _ in range(n):
            if dtype == np.float64:
                hist.append(oracle.residual_norm(want, f))
                want = oracle.jacobi_sweep(want, f)
            else:
                hist.append(oracle.residual_norm_f32_storage(want, f))
                want = oracle.sweep_f32(want, f)
        hist.append(oracle.residual_norm(want, f) if dtype == np.float64
                    else oracle.residual_norm_f32_storage(want, f))
        assert np.array_equal(host(out), want), (dims, n)
        np.testing.assert_allclose(host(res), hist, rtol=NORM_RTOL)


def test_autotuned_shape_is_used_and_bit_exact():
    nx, ny, nz = 200, 40, 30
    u, f = _problem(nx, ny, nz, seed=17)
    du, dt, df = ms.field_from(u), ms.field_from(u), ms.field_from(f)
    ms.tuning_clear()
    best = ms.autotune_sweeps(du, dt, df, sweeps_per_trial=2)
    assert best["nx"] == nx and best["us_per_sweep"] > 0
    assert ms.tuning_table() == [best]
    du, dt = ms.field_from(u), ms.field_from(u)
    res = torch.zeros(4, dtype=torch.float64, device="cuda")
    out = ms.jacobi_sweeps(du, dt, 3, f=df, res=res)
    want, hist = oracle.jacobi_sweeps(u, f, 3)
    assert np.array_equal(host(out), want)
    ms.tuning_clear()
