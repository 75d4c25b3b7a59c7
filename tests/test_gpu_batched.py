"""GPU batched persistent solve: per-instance results against the oracle and
against single-instance solves."""

import numpy as np
import torch
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
    teams, g, groups = ms.batched_plan(xs, [None] * 8, precision=ms.MS_SOLVE_F32_REFINED,
                                       with_groups=True)
    size = {}
    for t, k in zip(teams, groups):
        assert t >= 1 and size.setdefault(k, t) == t
    assert sum(size.values()) == g
    # bigger instances (more cells x more sweeps) get at least as many blocks
    work = [np.prod(d) * max(d) ** 2 for d in dims[:8]]
    order = np.argsort(work)
    assert teams[order[-1]] >= teams[order[0]]


def test_more_instances_than_resident_blocks():
    """Teams run chains of instances, so a batch may hold more instances
    than the device has resident blocks; each still reaches the tolerance
    as the oracle measures it, and matches its single solve."""
    note("case: batched, 600 tiny instances")
    dims = synth.batch_sizes(600, 21, lo=2, hi=9)
    probs = _instances(dims, 700)
    xs = [dev(u) for u, _ in probs]
    fs = [dev(f) for _, f in probs]
    teams, g, groups = ms.batched_plan(xs, fs, precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8,
                                       with_groups=True)
    assert len(set(groups)) <= g < len(xs)
    infos = ms.jacobi_solve_batched(xs, fs, precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8)
    for (u, f), x, info in zip(probs, xs, infos):
        assert info.status == ms.MS_OK
        res0 = oracle.residual_norm(oracle.zero_interior(u), f)
        assert oracle.residual_norm(host(x), f) <= 1e-8 * res0 * (1 + 1e-9)
    for k in (0, 299, 599):
        u, f = probs[k]
        y = dev(u)
        one = ms.jacobi_solve(y, dev(f), precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8)
        assert (one.sweeps, one.outer_iters) == (infos[k].sweeps, infos[k].outer_iters)
        assert np.array_equal(host(y), host(xs[k]))


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


@pytest.mark.parametrize("shape", [None, (64, 4)])
def test_two_sweeps_per_barrier_gives_the_same_fields(monkeypatch, shape):
    """The FP32 inner solves sweep twice per team barrier by default (the
    second sweep's norm judged after the first's); MS_BATCH_TB=1 keeps one
    sweep per barrier. Same arithmetic per cell, so the same iterates,
    counts and fields; extents below, at and above the 60-column and 4-row
    wave tile, odd and even accepted iterates."""
    note(f"case: batched two sweeps per barrier, shape {shape}")
    dims = DIMS + [(130, 33, 20), (61, 9, 17), (60, 4, 2)]
    probs = _instances(dims, 110, halo=True)
    infos, got = _solve_with_shape(probs, shape, ms.MS_SOLVE_F32_REFINED)
    monkeypatch.setenv("MS_BATCH_TB", "1")
    ref_infos, ref = _solve_with_shape(probs, shape, ms.MS_SOLVE_F32_REFINED)
    for (u, f), a, b, fa, fb in zip(probs, ref_infos, infos, ref, got):
        assert b.status == ms.MS_OK
        assert (a.sweeps, a.outer_iters) == (b.sweeps, b.outer_iters)
        assert np.array_equal(fa, fb)
        res0 = oracle.residual_norm(oracle.zero_interior(u), f)
        assert oracle.residual_norm(fb, f) <= 1e-8 * res0 * (1 + 1e-9)


@pytest.mark.parametrize("precision", [ms.MS_SOLVE_F32_REFINED, ms.MS_SOLVE_F64])
def test_xcd_local_barriers_give_the_same_fields(monkeypatch, precision):
    """Teams whose blocks share an XCD synchronise through its L2 by default;
    MS_BATCH_XCD_BARRIER=0 keeps agent-scope fences for every team. Same
    counts and fields, on a batch big enough for multi-block teams."""
    note(f"case: batched XCD-local barriers precision={precision}")
    dims = [(200, 120, 60), (130, 64, 40), (64, 64, 64)] + DIMS
    probs = _instances(dims, 130, halo=True)
    teams, _ = ms.batched_plan([dev(u) for u, _ in probs], [dev(f) for _, f in probs],
                               precision=precision, rel_tol=1e-8)
    assert max(teams) > 1
    infos, got = _solve_with_shape(probs, None, precision)
    monkeypatch.setenv("MS_BATCH_XCD_BARRIER", "0")
    ref_infos, ref = _solve_with_shape(probs, None, precision)
    for a, b, fa, fb in zip(ref_infos, infos, ref, got):
        assert b.status == ms.MS_OK
        assert (a.sweeps, a.outer_iters) == (b.sweeps, b.outer_iters)
        assert np.array_equal(fa, fb)


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
    recomputed by the oracle; the four smallest are compared bit for bit
    with single-instance solves and with the oracle's own trajectory."""
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
    small = sorted(range(len(dims)), key=lambda i: np.prod(dims[i]))[:4]
    jobs = []
    for i in small:
        u, f = probs[i]
        single = dev(u)
        s = ms.jacobi_solve(single, dev(f), **opts)
        assert (s.sweeps, s.outer_iters) == (infos[i].sweeps, infos[i].outer_iters)
        assert np.array_equal(host(single), host(xs[i]))
        # inner sweep counts of every outer step: the same solve capped at
        # 1, 2, ... outer steps
        cum = [0]
        for m in range(1, s.outer_iters + 1):
            sm = ms.jacobi_solve(dev(u), dev(f), **dict(opts, max_outer=m))
            cum.append(sm.sweeps)
        counts = [b - a for a, b in zip(cum, cum[1:])]
        d = ms.solve_opts()
        jobs.append((i, dims[i], counts, 1e-8, d.inner_eta, 40, d.max_inner, d.stall_window))
    # The oracle's trajectory of the four smallest instances (the
    # configuration's check): replaying the device's inner counts gives the
    # device's answer bit for bit, and on the oracle's own residual history
    # every count is where the oracle's stopping rule stops (one sweep either
    # way only when the residual straddles the threshold within 1e-10).
    import concurrent.futures as cf
    import multiprocessing as mp
    import oracle_jobs
    with cf.ProcessPoolExecutor(len(jobs), mp_context=mp.get_context("spawn")) as pool:
        results = list(pool.map(oracle_jobs.batched_instance_replay, jobs))
    for job, (x, rhos, etas, rels) in zip(jobs, results):
        i, counts = job[0], job[2]
        note(f"oracle trajectory of batched instance {i} {dims[i]}: inner {counts}")
        assert np.array_equal(x, host(xs[i])), i
        assert rels[-1] <= 1e-8
        for c, rho, eta_o in zip(counts, rhos, etas):
            own = oracle_jobs.stops_at(rho, eta_o, job[7], job[6])
            assert own == c or (abs(own - c) == 1 and
                                oracle_jobs.straddles(rho, min(own, c), eta_o)), (i, c, own)


def test_plan_estimates_follow_the_slowest_mode_component():
    """The planner's sweep estimate is ln(tol ||r(u^0)|| / c1) / ln(rho), c1
    the starting residual's component along the slowest mode, kept within
    [1/10, 1] of ln(tol) / ln(rho), with r the residual of the zero-interior
    start: recomputed here from the oracle's residual, for an eigenmode
    right-hand side (c1 = ||r||: the bound), a Gaussian one with a random
    halo, a nonzero interior (ignored) and a problem already solved."""
    import math
    note("case: batched plan estimates")
    tol = 1e-8
    dims = [(20, 16, 12), (33, 17, 9), (24, 24, 24), (10, 9, 8)]
    probs = []
    phi = synth.eigenmode(*dims[0])
    f0 = np.zeros_like(phi)
    f0[1:-1, 1:-1, 1:-1] = phi[1:-1, 1:-1, 1:-1]
    probs.append((synth.zeros(*dims[0]), f0))
    probs.append((synth.dirichlet_uniform(*dims[1], 3), synth.gaussian_sources(*dims[1], 4, 4)))
    u2 = synth.zeros(*dims[2])
    u2[1:-1, 1:-1, 1:-1] = synth.rng(5).standard_normal((24, 24, 24)) * 1e-3
    probs.append((u2, synth.gaussian_sources(*dims[2], 6, 6)))
    probs.append((synth.zeros(*dims[3]), np.zeros_like(synth.zeros(*dims[3]))))
    xs = [dev(u) for u, _ in probs]
    fs = [dev(f) for _, f in probs]
    _, _, est = ms.batched_plan(xs, fs, with_estimates=True,
                                precision=ms.MS_SOLVE_F32_REFINED, rel_tol=tol)
    for (u, f), (nx, ny, nz), e in zip(probs, dims, est):
        rho = sum(math.cos(math.pi / (n + 1)) for n in (nx, ny, nz)) / 3.0
        upper = max(math.log(tol) / math.log(rho), 1.0)
        res0 = oracle.residual_norm(oracle.zero_interior(u), f)
        if res0 == 0.0:
            assert e == 1.0
            continue
        p1 = synth.eigenmode(nx, ny, nz)[1:-1, 1:-1, 1:-1]
        r = oracle.residual(oracle.zero_interior(u), f)
        c1 = abs(float((r * p1).sum())) / float(np.linalg.norm(p1))
        want = min(upper, max(math.log(tol * res0 / c1) / math.log(rho), upper / 10, 1.0))
        assert e == pytest.approx(want, rel=1e-9), (nx, ny, nz)
    assert est[0] == pytest.approx(
        math.log(tol) / math.log(sum(math.cos(math.pi / (n + 1)) for n in dims[0]) / 3.0),
        rel=1e-9)


@pytest.mark.parametrize("workers", [1, 3])
@pytest.mark.parametrize("kw", [dict(precision=ms.MS_SOLVE_F32_REFINED),
                                dict(precision=ms.MS_SOLVE_F64),
                                dict(precision=ms.MS_SOLVE_F64, method=ms.MS_METHOD_RBGS)],
                         ids=["f32r", "f64", "f64-rbgs"])
def test_stream_batch_equals_single_solves(workers, kw):
    """Instances solved on concurrent streams give what jacobi_solve gives
    one at a time: the same fields bit for bit and the same counts."""
    note(f"case: stream batch workers={workers} {kw}")
    dims = [(40, 30, 20), (9, 7, 5), (64, 33, 17), (20, 20, 20), (5, 60, 9), (33, 9, 41)]
    probs = _instances(dims, 700, halo=True)
    xs = [dev(u) for u, _ in probs]
    fs = [dev(f) for _, f in probs]
    infos = ms.jacobi_solve_batched_streams(xs, fs, workers=workers, rel_tol=1e-8, **kw)
    for (u, f), x, info in zip(probs, xs, infos):
        y = dev(u)
        ref = ms.jacobi_solve(y, dev(f), rel_tol=1e-8, **kw)
        assert (info.sweeps, info.outer_iters, info.status) == (ref.sweeps, ref.outer_iters,
                                                                 ref.status)
        assert torch.equal(x, y)


def test_stream_batch_reports_a_nonfinite_instance_and_solves_the_rest():
    dims = [(12, 10, 8), (16, 9, 7), (8, 8, 8)]
    probs = _instances(dims, 800)
    probs[1][1][3, 4, 5] = np.nan
    xs = [dev(u) for u, _ in probs]
    fs = [dev(f) for _, f in probs]
    with pytest.raises(ms.MsError) as e:
        ms.jacobi_solve_batched_streams(xs, fs, workers=2, rel_tol=1e-8)
    assert e.value.code == ms.MS_ENONFINITE
    for (u, f), x in zip([probs[0], probs[2]], [xs[0], xs[2]]):
        res0 = oracle.residual_norm(oracle.zero_interior(u), f)
        assert oracle.residual_norm(host(x), f) <= 1e-8 * res0 * (1 + 1e-9)
