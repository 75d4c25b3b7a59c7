"""GPU convergence-controlled solves against the oracle: iteration counts,
fields at the accepted iterate, refinement to 1e-8, failure statuses."""

import math

import numpy as np
import pytest

import oracle
import synth
from gpuhelp import dev, host, note

pytestmark = pytest.mark.gpu

import paper_2310_01882_amd as ms  # noqa: E402

STRADDLE = 1e-10  # relative closeness to tol under which K +- 1 is accepted


def _poisson(nx, ny, nz, seed, halo=True, nsrc=6):
    u = synth.dirichlet_uniform(nx, ny, nz, seed) if halo else synth.zeros(nx, ny, nz)
    f = synth.gaussian_sources(nx, ny, nz, nsrc, seed + 1)
    return u, f


def _count_ok(k_gpu, k_or, hist, res0, tol):
    if k_gpu == k_or:
        return True
    near = any(abs(hist[k] / res0 - tol) <= STRADDLE * tol
               for k in (k_or - 1, k_or) if 0 <= k < len(hist))
    return near and abs(k_gpu - k_or) == 1


@pytest.mark.parametrize("dims,tol", [((16, 16, 16), 1e-6), ((24, 20, 12), 1e-8),
                                      ((65, 9, 7), 1e-5), ((1, 1, 1), 1e-12)])
@pytest.mark.parametrize("use_graph", [1, 0])
def test_f64_solve_count_and_field_match_oracle(dims, tol, use_graph):
    note(f"case: solve f64 {dims} tol {tol} graph {use_graph}")
    u, f = _poisson(*dims, seed=sum(dims))
    K, uk, hist, res0, ok = oracle.jacobi_solve(u, f, tol, 200000)
    assert ok
    du = dev(u)
    info = ms.jacobi_solve(du, dev(f), rel_tol=tol, max_sweeps=200000, use_graph=use_graph,
                           check_every=37, want_hist=True)
    assert info.status == ms.MS_OK
    assert _count_ok(info.sweeps, K, hist, res0, tol), (info.sweeps, K)
    assert info.res0 == pytest.approx(res0, rel=1e-13)
    if info.sweeps == K:
        assert np.array_equal(host(du), uk)
        np.testing.assert_allclose(info.hist, hist, rtol=1e-12)
        assert info.rel_final <= tol


def test_eigenmode_problem_iteration_count():
    nx, ny, nz = 40, 32, 24
    phi = synth.eigenmode(nx, ny, nz)
    rho = (math.cos(math.pi / (nx + 1)) + math.cos(math.pi / (ny + 1))
           + math.cos(math.pi / (nz + 1))) / 3.0
    f = np.zeros_like(phi)
    f[1:-1, 1:-1, 1:-1] = -6.0 * (1.0 - rho) * phi[1:-1, 1:-1, 1:-1]
    du = dev(np.zeros_like(phi))
    info = ms.jacobi_solve(du, dev(f), rel_tol=1e-6, max_sweeps=100000)
    assert abs(info.sweeps - math.ceil(math.log(1e-6) / math.log(rho))) <= 1
    # the answer approaches phi
    assert np.max(np.abs(host(du) - phi)) < 1e-5


def test_chunk_size_and_graph_do_not_change_the_result():
    u, f = _poisson(30, 22, 18, 3)
    outs = []
    for ce, g in ((1, 0), (7, 1), (64, 1), (1000, 1)):
        du = dev(u)
        info = ms.jacobi_solve(du, dev(f), rel_tol=1e-7, check_every=ce, use_graph=g)
        outs.append((info.sweeps, host(du).tobytes()))
    assert len(set(outs)) == 1


def test_not_converged_returns_the_capped_iterate():
    u, f = _poisson(20, 20, 20, 9)
    du = dev(u)
    info = ms.jacobi_solve(du, dev(f), rel_tol=1e-14, max_sweeps=33)
    assert info.status == ms.MS_NOT_CONVERGED and info.sweeps == 33
    want, _ = oracle.jacobi_sweeps(u, f, 33)
    assert np.array_equal(host(du), want)


def test_resume_is_bit_identical_to_an_uninterrupted_run():
    u, f = _poisson(26, 18, 14, 10)
    d1 = dev(u)
    full = ms.jacobi_solve(d1, dev(f), rel_tol=1e-8)
    d2 = dev(u)
    part = ms.jacobi_solve(d2, dev(f), rel_tol=1e-8, max_sweeps=full.sweeps // 3)
    assert part.status == ms.MS_NOT_CONVERGED
    rest = ms.jacobi_solve(d2, dev(f), rel_tol=1e-8)
    assert part.sweeps + rest.sweeps == full.sweeps
    assert np.array_equal(host(d1), host(d2))


def test_zero_reference_gives_zero_sweeps():
    u = synth.eigenmode(12, 12, 12)  # zero halo, f = 0 -> res0 = 0
    du = dev(u)
    info = ms.jacobi_solve(du, None, rel_tol=1e-8)
    assert info.status == ms.MS_OK and info.sweeps == 0 and info.res0 == 0.0
    assert np.array_equal(host(du), u)


def test_nonfinite_rhs_is_reported():
    u, f = _poisson(10, 10, 10, 4)
    f[5, 5, 5] = np.nan
    with pytest.raises(ms.MsError) as e:
        ms.jacobi_solve(dev(u), dev(f), rel_tol=1e-8)
    assert e.value.code == ms.MS_ENONFINITE


# ---------------------------------------------------------------- refinement

def _refined(u, f, **kw):
    du = dev(u)
    info = ms.jacobi_solve(du, dev(f), precision=ms.MS_SOLVE_F32_REFINED, want_hist=True, **kw)
    return du, info


@pytest.mark.parametrize("dims", [(24, 24, 24), (40, 18, 11)])
def test_refined_solve_reaches_1e8_checked_by_the_oracle(dims):
    note(f"case: refined {dims}")
    u, f = _poisson(*dims, seed=7, halo=False, nsrc=8)
    du, info = _refined(u, f, rel_tol=1e-8, inner_eta=1e-4)
    assert info.status == ms.MS_OK
    x = host(du)
    res0 = oracle.residual_norm(oracle.zero_interior(u), f)
    assert oracle.residual_norm(x, f) / res0 <= 1e-8
    # error against the oracle's FP64 solution at 1e-10
    K, xs, _, _, ok = oracle.jacobi_solve(u, f, 1e-10, 500000)
    assert ok
    err = np.max(np.abs(x - xs)) / np.max(np.abs(xs))
    note(f"refined {dims}: outer {info.outer_iters} sweeps {info.sweeps} "
         f"rel {info.rel_final:.3e} field rel err {err:.3e} (fp64 K at 1e-10: {K})")
    assert err < 1e-6


def test_refined_fields_replay_bit_exact_per_outer_step():
    """With the GPU's inner sweep counts replayed, the oracle reproduces
    every refinement step bit for bit (power-of-two scaling makes rhat and
    the update independent of the norm's rounding)."""
    u, f = _poisson(20, 16, 12, 5, halo=True, nsrc=5)
    counts = []
    prev = 0
    for outer in (1, 2):
        du, info = _refined(u, f, rel_tol=1e-12, inner_eta=1e-3, max_outer=outer)
        counts.append(info.sweeps - prev)
        prev = info.sweeps
        out = oracle.refined_solve(u, f, 1e-12, 1e-3, outer, 10 ** 7, 256, inner_counts=counts)
        assert np.array_equal(host(du), out["x"]), outer
    # and the counts follow the oracle's own stopping rule (straddle-tolerant)
    own = oracle.refined_solve(u, f, 1e-12, 1e-3, 2, 10 ** 7, 256)
    for a, b in zip(counts, own["inner"]):
        assert abs(a - b) <= 1


@pytest.mark.parametrize("dims,tol", [((16, 16, 16), 1e-6), ((33, 20, 12), 1e-7), ((9, 5, 3), 1e-9)])
def test_temporal_blocking_solve_matches_plain(dims, tol):
    u, f = _poisson(*dims, seed=sum(dims) + 1)
    res = []
    for tb in (1, 2):
        du = dev(u)
        info = ms.jacobi_solve(du, dev(f), rel_tol=tol, temporal_block=tb, check_every=13)
        res.append((info.sweeps, host(du)))
    assert res[0][0] == res[1][0]
    assert np.array_equal(res[0][1], res[1][1])
    K, uk, hist, res0, ok = oracle.jacobi_solve(u, f, tol, 200000)
    assert _count_ok(res[1][0], K, hist, res0, tol)


def test_temporal_blocking_refined_solve_matches_plain():
    u, f = _poisson(22, 18, 14, 6, halo=False, nsrc=4)
    out = []
    for tb in (1, 2):
        du, info = _refined(u, f, rel_tol=1e-8, temporal_block=tb)
        out.append((info.sweeps, info.outer_iters, host(du)))
    assert out[0][:2] == out[1][:2]
    assert np.array_equal(out[0][2], out[1][2])
