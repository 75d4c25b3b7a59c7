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
