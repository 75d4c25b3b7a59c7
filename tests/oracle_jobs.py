"""Oracle runs the GPU tests hand to worker processes (importable by a
spawned interpreter: numpy, synth and the oracle only)."""

import numpy as np

import oracle
import synth


def batched_instance_replay(args):
    """The oracle's FP32-refined solve of batched instance `index` (sizes
    from synth.batch_sizes(64, 4), 8 Gaussian sources, seed 1000 + index),
    replaying the given inner sweep counts. Returns (x, rho lists, eta per
    outer, rel per outer)."""
    index, dims, counts, tol, eta, max_outer, max_inner, stall = args
    u = synth.zeros(*dims)
    f = synth.gaussian_sources(*dims, 8, 1000 + index)
    out = oracle.refined_solve(u, f, tol, eta, max_outer, max_inner, stall,
                               inner_counts=counts)
    return out["x"], out["rho"], out["eta"], out["hist"]


def stops_at(rho, eta_o, stall, max_inner):
    """The inner stopping rule of the refinement applied to a residual
    history: the first j that stops."""
    for j in range(len(rho)):
        if rho[j] <= eta_o * rho[0] or j == max_inner:
            return j
        if j >= stall and rho[j] >= rho[j - stall]:
            return j
    return None


def straddles(rho, j, eta_o, rel=1e-10):
    """True if rho_j sits within `rel` of the stopping threshold."""
    thr = eta_o * rho[0]
    return abs(rho[j] - thr) <= rel * thr


__all__ = ["batched_instance_replay", "stops_at", "straddles", "np"]
