"""What the trained warm start gains over the solver without it, on held-out
128^3 instances (seeds 20000 + i, 1-8 Gaussian sources, zero Dirichlet
boundary), each solved to a 1e-8 relative residual:
  B  FP32-refined Jacobi from the zero interior,
  C  the network's guess, the zero interior instead when the guess's FP64
     residual is not below the zero interior's, then the same solver.
The test checks what must hold whatever the network learned -- C reaches
the tolerance as the oracle measures it, and when the fallback fires C is
B bit for bit -- and prints the measured gain (sweeps and seconds)."""

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
    for seed in (20000, 20001):
        note(f"case: warm-start gain, held-out seed {seed}")
        u, f = _instance(seed)
        fd = ms.field_from(f)
        xb = ms.field_from(u)
        b, tb = _timed(lambda: ms.jacobi_solve(xb, fd, **opts))
        xc = ms.field_from(u)

        def with_guess():
            used, meas = net.guess(xc, fd, xc, rule="residual")
            return ms.jacobi_solve(xc, fd, **opts), used, meas

        (c, used, meas), tc = _timed(with_guess)
        used = bool(used.item())
        ratio = meas[0].item() / meas[1].item()
        res0 = oracle.residual_norm(oracle.zero_interior(u), f)
        assert c.status == ms.MS_OK and b.status == ms.MS_OK
        assert oracle.residual_norm(host(xc), f) <= 1e-8 * res0 * (1 + 1e-9)
        if not used:
            assert (c.sweeps, c.outer_iters) == (b.sweeps, b.outer_iters)
            assert np.array_equal(host(xc), host(xb))
        print(f"seed {seed}: guess residual / zero residual {ratio:.3g}, guess used {used}; "
              f"B {b.sweeps} sweeps {tb:.3f} s, C {c.sweeps} sweeps {tc:.3f} s, "
              f"gain {b.sweeps - c.sweeps} sweeps ({(tb - tc) * 1e3:+.1f} ms)")
