"""Train and evaluate the learned warm start on Jacobi-generated data.

    python -m paper_2310_01882_amd.train_warmstart train --n 128 --train 2000 \
        --epochs 24 --out weights.npz --report train_report.json
    python -m paper_2310_01882_amd.train_warmstart eval --n 128 --eval 200 \
        --weights weights.npz --report eval_report.json

Training instances: n^3 interior, zero Dirichlet boundary, right-hand side
= 1..8 Gaussian sources (count and sources from seed 10000 + i), solved to
a 1e-10 relative residual by the library's solver (FP32-storage Jacobi
sweeps inside FP64 refinement, instances on concurrent streams); the
network trains on them with warmstart_train_step (one instance per Adam
step). Held-out instances use seeds 20000 + i; each is solved to a 1e-8
relative residual five ways on the same GPU:
  A plain FP64 Jacobi from the zero interior,
  B FP32-refined Jacobi from the zero interior,
  C warmstart_forward (four damped sweeps on the guess, slowest-mode start
    rule), then B's solver,
  D the same forcing the guess,
  E the guess forced without the damped sweeps (what they contribute).
The report gives sweeps and seconds of each, the guess's relative error
against A's answer, its four start measures, and which start the residual
rule would have taken (the rules differ only in the decision: the solve
from either start is D's or B's, which are both measured).
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def instance(n, seed):
    import synth
    count = synth.random_source_count(seed)
    return synth.zeros(n, n, n), synth.gaussian_sources(n, n, n, count, seed)


def solve_targets(ms, n, seeds, batch, workers, tol):
    """(f, u_solved) device fields for every seed."""
    pairs = []
    for b0 in range(0, len(seeds), batch):
        t0 = time.perf_counter()
        chunk = seeds[b0:b0 + batch]
        probs = [instance(n, s) for s in chunk]
        xs = [ms.field_from(u) for u, _ in probs]
        fs = [ms.field_from(f) for _, f in probs]
        infos = ms.jacobi_solve_batched_streams(xs, fs, workers=workers,
                                                precision=ms.MS_SOLVE_F32_REFINED, rel_tol=tol,
                                                max_outer=40)
        for info in infos:
            if info.rel_final > tol:
                raise RuntimeError(f"target solve reached only {info.rel_final:.3e}")
        pairs.extend(zip(fs, xs))
        log(f"[train] solved targets {b0 + len(chunk)}/{len(seeds)} "
            f"({time.perf_counter() - t0:.1f} s; sweeps {min(i.sweeps for i in infos)}.."
            f"{max(i.sweeps for i in infos)})")
    return pairs


def lr_at(epoch, epochs, lr):
    """Step decay: full rate for 60% of the epochs, then a third, then a tenth."""
    if epoch < 0.6 * epochs:
        return lr
    return lr / 3 if epoch < 0.85 * epochs else lr / 10


def train(args):
    import numpy as np
    import torch

    import paper_2310_01882_amd as ms
    from paper_2310_01882_amd import warmstart as wsm

    n = args.n
    net = wsm.WarmStart(n, n, n, seed=args.seed)
    t0 = time.perf_counter()
    pairs = solve_targets(ms, n, [10000 + i for i in range(args.train)], args.batch,
                          args.workers, 1e-10)
    target_s = time.perf_counter() - t0
    zero = ms.alloc_field(n, n, n)
    order = np.random.Generator(np.random.PCG64(args.seed)).permutation
    t0 = time.perf_counter()
    losses = []
    for ep in range(args.epochs):
        lr = lr_at(ep, args.epochs, args.lr)
        tot = torch.zeros((), dtype=torch.float64, device="cuda")
        for i in order(len(pairs)):
            f, x = pairs[i]
            tot += net.train_step(zero, f, x, lr=lr)[0]
        losses.append(tot.item() / len(pairs))
        log(f"[train] epoch {ep + 1}/{args.epochs} (lr {lr:.1e}): mean loss {losses[-1]:.6e} "
            f"({time.perf_counter() - t0:.1f} s)")
    train_s = time.perf_counter() - t0
    meta = {"train_instances": args.train, "epochs": args.epochs, "lr": args.lr,
            "seed": args.seed, "out_scale": net.out_scale}
    net.save(args.out, meta=meta)
    report = dict(meta, n=n, target_tol=1e-10, target_seconds=target_s, train_seconds=train_s,
                  epoch_losses=losses, lr_schedule="full for 60% of epochs, /3, then /10",
                  weights=os.path.basename(args.out))
    with open(args.report, "w") as fh:
        json.dump(report, fh, indent=1)
    print(json.dumps({k: v for k, v in report.items() if k != "epoch_losses"}), flush=True)


NAMES = ("A_fp64", "B_fp32_refined", "C_cnn_slow_modes", "D_cnn_forced", "E_cnn_unsmoothed")


def evaluate(args):
    import torch

    import paper_2310_01882_amd as ms
    from paper_2310_01882_amd import warmstart as wsm

    n, tol = args.n, 1e-8
    params, out_scale, meta = wsm.WarmStart.load(args.weights)
    net = wsm.WarmStart(n, n, n, params=params, out_scale=out_scale)
    F32R = ms.MS_SOLVE_F32_REFINED
    rows = []
    seeds = [20000 + i for i in range(args.eval)]
    for rep, s in enumerate([seeds[0]] + seeds):  # the first pass warms graphs and caches
        u, f = instance(n, s)
        fd, u0 = ms.field_from(f), ms.field_from(u)
        row = {"seed": s}
        xa = None
        for name in NAMES:
            x = ms.field_from(u)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name[0] in "CDE":
                used, meas = net.guess(u0, fd, x, rule="slow_modes" if name[0] == "C" else "force",
                                       smooth=0 if name[0] == "E" else 4)
            prec = ms.MS_SOLVE_F64 if name == "A_fp64" else F32R
            info = ms.jacobi_solve(x, fd, precision=prec, rel_tol=tol)
            torch.cuda.synchronize()
            row[name] = {"seconds": time.perf_counter() - t0, "sweeps": info.sweeps,
                         "rel_final": info.rel_final, "outer": info.outer_iters}
            if name == "A_fp64":
                xa = x
            if name[0] in "CDE":
                m = [float(v) for v in meas.cpu()]
                row[name]["guess_used"] = bool(used.item())
                row[name]["measures"] = m
            if name == "D_cnn_forced":
                g2 = ms.field_from(u)
                net.guess(u0, fd, g2, rule="force")
                gi, ai = g2[1:-1, 1:-1, 1:-1], xa[1:-1, 1:-1, 1:-1]
                row["guess_rel_error"] = float(torch.linalg.norm(gi - ai) / torch.linalg.norm(ai))
                row["residual_rule_keeps_guess"] = m[0] < m[1]
                row["guess_rel_residual"] = m[0] / m[1]
                row["guess_rel_slow"] = m[2] / m[3]
        if rep == 0:
            continue
        rows.append(row)
        log(f"[eval] seed {s}: " + ", ".join(
            f"{k} {row[k]['seconds']:.3f}s/{row[k]['sweeps']}" for k in NAMES)
            + f"; guess rel error {row['guess_rel_error']:.3f}, "
              f"slow {row['guess_rel_slow']:.3f}, used {row['C_cnn_slow_modes']['guess_used']}")
    summ = {}
    for k in NAMES:
        ts = [r[k]["seconds"] for r in rows]
        sw = [r[k]["sweeps"] for r in rows]
        summ[k] = {"mean_seconds": statistics.mean(ts), "median_seconds": statistics.median(ts),
                   "mean_sweeps": statistics.mean(sw), "median_sweeps": statistics.median(sw),
                   "max_rel_final": max(r[k]["rel_final"] for r in rows)}
    summ["C_guess_used_fraction"] = (sum(r["C_cnn_slow_modes"]["guess_used"] for r in rows)
                                     / len(rows))
    summ["residual_rule_used_fraction"] = (sum(r["residual_rule_keeps_guess"] for r in rows)
                                           / len(rows))
    summ["mean_guess_rel_error"] = statistics.mean(r["guess_rel_error"] for r in rows)
    summ["median_guess_rel_error"] = statistics.median(r["guess_rel_error"] for r in rows)
    summ["mean_guess_rel_slow"] = statistics.mean(r["guess_rel_slow"] for r in rows)
    summ["C_vs_B_sweeps_saved_mean"] = (summ["B_fp32_refined"]["mean_sweeps"]
                                        - summ["C_cnn_slow_modes"]["mean_sweeps"])
    summ["C_vs_B_seconds_saved_mean"] = (summ["B_fp32_refined"]["mean_seconds"]
                                         - summ["C_cnn_slow_modes"]["mean_seconds"])
    report = {"n": n, "eval_instances": args.eval, "tol": tol, "weights": meta,
              "summary": summ, "rows": rows}
    with open(args.report, "w") as fh:
        json.dump(report, fh, indent=1)
    print(json.dumps(summ), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["train", "eval"])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--eval", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=24)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="warmstart.npz")
    ap.add_argument("--weights", default="warmstart.npz")
    ap.add_argument("--report", default="warmstart_report.json")
    args = ap.parse_args()
    train(args) if args.what == "train" else evaluate(args)


if __name__ == "__main__":
    main()
