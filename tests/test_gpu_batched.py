"""GPU batched persistent solve: per-instance results against the oracle and
against single-instance solves."""

import numpy as np
import pytest

import oracle
import synth
from gpuhelp import dev, host, note

pytestmark = pytest.mark.gpu

import paper_2310_01882_amd as ms  # noqa: E402

DIMS = [(16, 16, 16), (24, 20, 12), (9, 5, 3), (32, 16, 8), (40, 18, 11), (12, 12, 30),
        (1, 1, 1), (70, 6, 5)]


def _instances(dims, seed0, halo=False):
    out = []
    for n, d in enumerate(dims):
        u = synth.dirichlet_uniform(*d, seed0 + n) if halo else synth.zeros(*d)
        f = synth.gaussian_sources(*d, 1 + n % 8, seed0 + 100 + n)
        out.append((u, f))
    return out


@pytest.mark.parametrize("halo", [False, True])
def test_batched_refined_matches_single_solves_and_oracle(halo):
    note(f"case: batched refined halo={halo}")
    probs = _instances(DIMS, 50, halo)
    xs = [dev(u) for u, _ in probs]
    fs = [dev(f) for _, f in probs]
    infos = ms.jacobi_solve_batched(xs, fs, precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8)
    for (u, f), x, info in zip(probs, xs, infos):
        assert info.status == ms.MS_OK
        res0 = oracle.residual_norm(oracle.zero_interior(u), f)
        got = host(x)
        assert oracle.residual_norm(got, f) <= 1e-8 * res0 * (1 + 1e-9)
        single = dev(u)
        s = ms.jacobi_solve(single, dev(f), precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8)
        assert (s.sweeps, s.outer_iters) == (info.sweeps, info.outer_iters)
        assert np.array_equal(host(single), got)


def test_batched_f64_counts_and_fields_match_oracle():
    probs = _instances(DIMS, 70, halo=True)
    xs = [dev(u) for u, _ in probs]
    fs = [dev(f) for _, f in probs]
    infos = ms.jacobi_solve_batched(xs, fs, precision=ms.MS_SOLVE_F64, rel_tol=1e-7)
    for (u, f), x, info in zip(probs, xs, infos):
        K, uk, hist, res0, ok = oracle.jacobi_solve(u, f, 1e-7, 10 ** 6)
        assert ok and info.status == ms.MS_OK
        assert info.sweeps == K or abs(hist[min(K, len(hist) - 1)] / res0 - 1e-7) < 1e-16
        if info.sweeps == K:
            assert np.array_equal(host(x), uk)
        assert info.res0 == pytest.approx(res0, rel=1e-13)


def test_many_small_instances_and_determinism():
    dims = synth.batch_sizes(64, 9, lo=6, hi=24)
    probs = _instances(dims, 300)
    runs = []
    for _ in range(2):
        xs = [dev(u) for u, _ in probs]
        fs = [dev(f) for _, f in probs]
        infos = ms.jacobi_solve_batched(xs, fs, precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8)
        runs.append(([i.sweeps for i in infos], [host(x).tobytes() for x in xs]))
        for (u, f), x, info in zip(probs, xs, infos):
            assert info.status == ms.MS_OK
            res0 = oracle.residual_norm(oracle.zero_interior(u), f)
            assert oracle.residual_norm(host(x), f) <= 1e-8 * res0 * (1 + 1e-9)
    assert runs[0] == runs[1]


def test_plan_gives_every_instance_a_team():
    dims = synth.batch_sizes(64, 4)
    xs = [ms.alloc_field(*d) for d in dims[:8]]
    teams, g = ms.batched_plan(xs, [None] * 8, precision=ms.MS_SOLVE_F32_REFINED)
    assert all(t >= 1 for t in teams) and sum(teams) == g
    # bigger instances (more cells x more sweeps) get at least as many blocks
    work = [np.prod(d) * max(d) ** 2 for d in dims[:8]]
    order = np.argsort(work)
    assert teams[order[-1]] >= teams[order[0]]


def _solve_with_shape(probs, shape, precision):
    """Batched solve with every instance's tile shape forced to `shape`
    ((tx, zsplit), or None for the library default)."""
    xs = [dev(u) for u, _ in probs]
    fs = [dev(f) for _, f in probs]
    ms.batch_tuning_clear()
    if shape is not None:
        teams, _ = ms.batched_plan(xs, fs, precision=precision, rel_tol=1e-8)
        ms.batch_tuning_load([dict(precision=precision, nx=x.shape[2] - 2, ny=x.shape[1] - 2,
                                   nz=x.shape[0] - 2, team=t, tx=shape[0], zsplit=shape[1])
                              for x, t in zip(xs, teams)])
    infos = ms.jacobi_solve_batched(xs, fs, precision=precision, rel_tol=1e-8)
    ms.batch_tuning_clear()
    return infos, [host(x) for x in xs]


@pytest.mark.parametrize("precision", [ms.MS_SOLVE_F32_REFINED, ms.MS_SOLVE_F64])
def test_every_tile_shape_gives_the_same_fields(precision):
    note(f"case: batched tile shapes precision={precision}")
    probs = _instances(DIMS, 90, halo=True)
    ref_infos, ref = _solve_with_shape(probs, None, precision)
    for shape in [(64, 8), (32, 1), (32, 4), (16, 2), (16, 8)]:
        infos, got = _solve_with_shape(probs, shape, precision)
        for a, b, fa, fb in zip(ref_infos, infos, ref, got):
            assert b.status == ms.MS_OK
            # the norms' summation order changes with the shape; the iterates do not
            assert (a.sweeps, a.outer_iters) == (b.sweeps, b.outer_iters), shape
            assert np.array_equal(fa, fb), shape


def test_autotune_picks_valid_shapes_and_leaves_x_alone():
    note("case: batched autotune 16 instances")
    dims = synth.batch_sizes(16, 4, lo=16, hi=96)
    probs = _instances(dims, 500)
    xs = [dev(u) for u, _ in probs]
    fs = [dev(f) for _, f in probs]
    before = [host(x) for x in xs]
    ms.batch_tuning_clear()
    best = ms.batched_autotune(xs, fs, sweeps_per_trial=8, precision=ms.MS_SOLVE_F32_REFINED,
                               rel_tol=1e-8)
    assert all(np.array_equal(host(x), b) for x, b in zip(xs, before))
    teams, _ = ms.batched_plan(xs, fs, precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8)
    assert [b["team"] for b in best] == teams
    for b, d in zip(best, dims):
        assert (b["nx"], b["ny"], b["nz"]) == d
        assert b["tx"] in (16, 32, 64) and b["zsplit"] in (1, 2, 4, 8)
        assert b["us_per_sweep"] > 0
    assert len(ms.batch_tuning_table()) == len(set((b["nx"], b["ny"], b["nz"], b["team"])
                                                   for b in best))
    infos = ms.jacobi_solve_batched(xs, fs, precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8)
    tuned = [host(x) for x in xs]
    ms.batch_tuning_clear()
    ref_infos, ref = _solve_with_shape(probs, None, ms.MS_SOLVE_F32_REFINED)
    for a, b, fa, fb, (u, f) in zip(ref_infos, infos, ref, tuned, probs):
        assert (a.sweeps, a.outer_iters) == (b.sweeps, b.outer_iters)
        assert np.array_equal(fa, fb)
        res0 = oracle.residual_norm(oracle.zero_interior(u), f)
        assert oracle.residual_norm(fb, f) <= 1e-8 * res0 * (1 + 1e-9)


def test_full_batch_of_64_uneven_instances_after_autotuning():
    """The benchmark's batch at full size: 64 instances, per-axis sizes
    log-uniform in [32, 256] (seed 4), 8 Gaussian sources each, FP32-refined
    to 1e-8 with autotuned tile shapes. Every instance's final residual is
    recomputed by the oracle; the three smallest are compared bit for bit
    with single-instance solves."""
    note("case: batched 64 instances, sizes log-uniform [32, 256], seed 4")
    dims = synth.batch_sizes(64, 4)
    probs = [(synth.zeros(*d), synth.gaussian_sources(*d, 8, 1000 + i))
             for i, d in enumerate(dims)]
    xs = [dev(u) for u, _ in probs]
    fs = [dev(f) for _, f in probs]
    opts = dict(precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8, max_outer=40)
    ms.batch_tuning_clear()
    ms.batched_autotune(xs, fs, sweeps_per_trial=10, **opts)
    infos = ms.jacobi_solve_batched(xs, fs, **opts)
    ms.batch_tuning_clear()
    for (u, f), x, info in zip(probs, xs, infos):
        assert info.status == ms.MS_OK
        res0 = oracle.residual_norm(oracle.zero_interior(u), f)
        assert info.res0 == pytest.approx(res0, rel=1e-12)
        assert oracle.residual_norm(host(x), f) <= 1e-8 * res0 * (1 + 1e-9)
    small = sorted(range(len(dims)), key=lambda i: np.prod(dims[i]))[:3]
    for i in small:
        u, f = probs[i]
        single = dev(u)
        s = ms.jacobi_solve(single, dev(f), **opts)
        assert (s.sweeps, s.outer_iters) == (infos[i].sweeps, infos[i].outer_iters)
        assert np.array_equal(host(single), host(xs[i]))
