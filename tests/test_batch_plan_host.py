"""The batched planner on the host (no device): teams, chains and block
counts for given sweep estimates. Checked against its documented cost
models: with one sweep per team barrier (FP64) an instance of C cells and S
sweeps on t blocks costs C S / t, plus 8192 S when t > 1; with two sweeps
per barrier (FP32-refined) S / 2 x (rounds x (nz / p + 2) + 15 [t > 1]) for
the z split p that minimises rounds x levels. A team's chain costs the sum
over its instances."""

import math

import numpy as np
import pytest

import synth

ms = pytest.importorskip("paper_2310_01882_amd")

BARRIER = 8192.0
F64, F32R = ms.MS_SOLVE_F64, ms.MS_SOLVE_F32_REFINED


def _pair_levels(d, t):
    nx, ny, nz = d
    tiles = math.ceil(nx / 60) * math.ceil(ny / 4)
    best = None
    p = 1
    while p <= 16 and p <= nz:
        c = math.ceil(tiles * p / (16 * t)) * (nz / p + 2)
        if best is None or c < best * 0.999:
            best = c
        p *= 2
    return best


def _cost(d, s, t, precision=F32R):
    if precision == F32R:
        return s / 2 * (_pair_levels(d, t) + (15 if t > 1 else 0))
    c = float(np.prod(d))
    return c * s / t + (BARRIER * s if t > 1 else 0.0)


def _cap(d, blocks):
    return max(1, min(blocks, 8 * math.ceil(d[0] / 64) * math.ceil(d[1] / 16)))


def _estimates(dims, seed):
    """Sweep estimates of the size of the slowest-mode bound at 1e-8."""
    r = np.random.default_rng(seed)
    out = []
    for d in dims:
        rho = sum(math.cos(math.pi / (n + 1)) for n in d) / 3.0
        out.append(math.log(1e-8) / math.log(rho) * r.uniform(0.5, 1.0))
    return out


def _one_team_each(dims, est, blocks, precision=F32R):
    """Makespan of one team per instance, blocks handed out one at a time to
    the instance with the longest cost that one more block shortens."""
    def c(i, t):
        return _cost(dims[i], est[i], t, precision)
    team = [1] * len(dims)
    for _ in range(blocks - len(dims)):
        best = None
        for i in range(len(dims)):
            if team[i] >= _cap(dims[i], blocks) or c(i, team[i] + 1) >= c(i, team[i]):
                continue
            if best is None or c(i, team[i]) > c(best, team[best]):
                best = i
        if best is None:
            break
        team[best] += 1
    return max(c(i, t) for i, t in enumerate(team))


def _check_plan(dims, est, blocks, precision=F32R):
    teams, groups, g = ms.batched_plan_from_estimates(dims, est, blocks, precision)
    assert len(teams) == len(groups) == len(dims)
    size_of = {}
    load = {}
    for d, s, t, k in zip(dims, est, teams, groups):
        assert 1 <= t <= _cap(d, blocks)
        assert size_of.setdefault(k, t) == t  # one team size per group
        load[k] = load.get(k, 0.0) + _cost(d, s, t, precision)
    assert sorted(size_of) == list(range(len(size_of)))
    assert sum(size_of.values()) == g <= blocks
    return teams, groups, g, max(load.values())


@pytest.mark.parametrize("precision", [F32R, F64])
def test_benchmark_batch_plan_is_no_worse_than_one_team_each(precision):
    dims = synth.batch_sizes(64, 4)
    est = _estimates(dims, 1)
    teams, groups, g, makespan = _check_plan(dims, est, 256, precision)
    base = _one_team_each(dims, est, 256, precision)
    assert makespan <= base * (1 + 1e-9)
    # small instances share a team: fewer teams than instances
    assert len(set(groups)) < len(dims)
    print(f"teams {len(set(groups))} for {len(dims)} instances, {g} blocks; "
          f"estimated makespan {makespan / base:.3f} of one team each")
    # the same input gives the same plan
    assert ms.batched_plan_from_estimates(dims, est, 256, precision) == (teams, groups, g)


@pytest.mark.parametrize("precision", [F32R, F64])
@pytest.mark.parametrize("n,blocks", [(1, 256), (3, 1), (40, 7), (300, 64), (64, 256)])
def test_any_number_of_instances_fits_the_blocks(n, blocks, precision):
    dims = synth.batch_sizes(n, 11, lo=6, hi=200)
    est = _estimates(dims, n)
    teams, groups, g, makespan = _check_plan(dims, est, blocks, precision)
    if n <= blocks:
        assert makespan <= _one_team_each(dims, est, blocks, precision) * (1 + 1e-9)
    else:
        assert len(set(groups)) <= blocks
    # the makespan cannot beat the work spread over every block (teams of
    # more than one block only add barrier time to the work)
    work = sum(_cost(d, s, 1, precision) for d, s in zip(dims, est))
    assert makespan >= work / blocks * (1 - 1e-9)


def test_one_instance_takes_the_blocks_that_help():
    dims = [(256, 256, 256)]
    est = [20000.0]
    teams, groups, g, _ = _check_plan(dims, est, 256, F64)
    assert teams == [256] and groups == [0] and g == 256
    # with two sweeps per barrier: the fewest blocks with the fewest rounds
    # (5 x 64 tiles of 60 x 4 columns and rows, 16 waves per block)
    teams, _, g, _ = _check_plan(dims, est, 256, F32R)
    costs = [_cost(dims[0], est[0], t) for t in range(1, 257)]
    assert costs[teams[0] - 1] == min(costs)
    assert all(c > min(costs) for c in costs[:teams[0] - 1])
    # a tiny grid: a barrier per sweep costs more than splitting saves
    for p in (F64, F32R):
        teams, _, g, _ = _check_plan([(8, 8, 8)], [100.0], 256, p)
        assert teams == [1] and g == 1


def test_planner_rejects_bad_input():
    with pytest.raises(ms.MsError):
        ms.batched_plan_from_estimates([(8, 8, 8)], [100.0], 4, precision=7)
    with pytest.raises(ms.MsError):
        ms.batched_plan_from_estimates([(8, 8, 8)], [100.0], 0)
    with pytest.raises(ms.MsError):
        ms.batched_plan_from_estimates([(8, 8, 8)], [0.5], 4)
    with pytest.raises(ms.MsError):
        ms.batched_plan_from_estimates([(8, 8, 8)], [float("nan")], 4)
    with pytest.raises(ms.MsError):
        ms.batched_plan_from_estimates([(0, 8, 8)], [100.0], 4)
