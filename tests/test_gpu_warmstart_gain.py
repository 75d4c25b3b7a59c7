"""What the trained warm start gains over the solver without it, on the first
four held-out 128^3 instances (seeds 20000..20003, 1-8 Gaussian sources,
zero Dirichlet boundary; the training set used seeds 10000..11999), each
solved to a 1e-8 relative residual:
  B  FP32-refined Jacobi from the zero interior,
  C  the network's guess after four damped Jacobi sweeps, kept when its
     slowest-mode projection is below the zero interior's, then the same
     solver.
Checked: C reaches the tolerance as the oracle measures it; the guess lies
within 0.5 relative L2 error of B's answer on every instance; the guess is
kept on every one of them; C needs at most 97% of B's sweeps over the four
(the solves are deterministic, so the sweep counts are too); and where the
guess is set aside C is B bit for bit. Seconds are printed, not asserted."""

import os
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from gpuhelp import host, note

pytestmark = pytest.mark.gpu

import paper_2310_01882_amd as ms  # noqa: E402
from paper_2310_01882_amd import warmstart as wsm  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(ms.__file__), "weights", "warmstart_128.npz")
N = 128
SEEDS = (20000, 20001, 20002, 20003)


def _instance(seed):
    return synth.zeros(N, N, N), synth.gaussian_sources(N, N, N, synth.random_source_count(seed),
                                                       seed)


def _timed(fn):
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t


def test_trained_warm_start_gain_on_held_out_instances():
    assert os.path.exists(WEIGHTS), "the trained weights are part of the package"
    net = wsm.WarmStart.from_file(WEIGHTS, N, N, N)
    opts = dict(precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8)
    sweeps_b = sweeps_c = 0
    for seed in SEEDS:
        note(f"case: warm-start gain, held-out seed {seed}")
        u, f = _instance(seed)
        fd, u0 = ms.field_from(f), ms.field_from(u)
        xb = ms.field_from(u)
        b, tb = _timed(lambda: ms.jacobi_solve(xb, fd, **opts))
        xc = ms.field_from(u)

        def with_guess():
            used, meas = net.guess(u0, fd, xc, rule="slow_modes")
            return ms.jacobi_solve(xc, fd, **opts), used, meas

        (c, used, meas), tc = _timed(with_guess)
        used = bool(used.item())
        g = ms.field_from(u)
        net.guess(u0, fd, g, rule="force")
        gi, bi = g[1:-1, 1:-1, 1:-1], xb[1:-1, 1:-1, 1:-1]
        err = float(torch.linalg.norm(gi - bi) / torch.linalg.norm(bi))
        res0 = oracle.residual_norm(oracle.zero_interior(u), f)
        assert c.status == ms.MS_OK and b.status == ms.MS_OK
        assert oracle.residual_norm(host(xc), f) <= 1e-8 * res0 * (1 + 1e-9)
        assert err <= 0.5, (seed, err)
        if not used:
            assert (c.sweeps, c.outer_iters) == (b.sweeps, b.outer_iters)
            assert np.array_equal(host(xc), host(xb))
        assert used, (seed, [float(v) for v in meas.cpu()])
        sweeps_b += b.sweeps
        sweeps_c += c.sweeps
        print(f"seed {seed}: guess error {err:.3f}, slow-mode ratio "
              f"{meas[2].item() / meas[3].item():.3g}, kept {used}; B {b.sweeps} sweeps "
              f"{tb:.3f} s, C {c.sweeps} sweeps {tc:.3f} s ({(tb - tc) * 1e3:+.1f} ms)")
    print(f"four instances: C/B sweeps {sweeps_c / sweeps_b:.4f}")
    assert sweeps_c <= 0.97 * sweeps_b, (sweeps_c, sweeps_b)
