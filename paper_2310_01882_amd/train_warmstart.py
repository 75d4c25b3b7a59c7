"""Train and evaluate the learned warm start on Jacobi-generated data.

    python -m paper_2310_01882_amd.train_warmstart --n 128 --train 256 \
        --eval 32 --epochs 8 --out weights.npz --report report.json

Training instances: n^3 interior, zero Dirichlet boundary, right-hand side
= 1..8 Gaussian sources (count and sources from seed 10000 + i). Targets:
the instances solved to a 1e-10 relative residual by the batched solver
(FP32-storage sweeps inside FP64 refinement), u / (s * lambda). Held-out
instances use seeds 20000 + i. For each held-out instance the report times
three solves to a 1e-8 relative residual on the same GPU:
  A plain FP64 Jacobi from the zero interior,
  B FP32-refined Jacobi from the zero interior,
  C the network's guess, then FP32-refined Jacobi (falls back to the zero
    interior when the guess's residual is not below the zero guess's),
  D the network's guess, then FP32-refined Jacobi, without the fallback.
The report also gives the guess's relative error against A's answer.
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


def solve_targets(ms, wsm, net, n, seeds, batch, tol):
    import torch
    fs, targets = [], []
    for b0 in range(0, len(seeds), batch):
        t0 = time.perf_counter()
        chunk = seeds[b0:b0 + batch]
        probs = [instance(n, s) for s in chunk]
        xs = [ms.field_from(u) for u, _ in probs]
        fdev = [ms.field_from(f) for _, f in probs]
        infos = ms.jacobi_solve_batched(xs, fdev, precision=ms.MS_SOLVE_F32_REFINED, rel_tol=tol,
                                        max_outer=40)
        for x, f, info in zip(xs, fdev, infos):
            if info.rel_final > tol:
                raise RuntimeError(f"target solve reached only {info.rel_final:.3e}")
            zero = torch.zeros_like(x)
            net.features(zero, f)
            targets.append(net.target(x).clone())
            fs.append(f)
        torch.cuda.synchronize()
        log(f"[train] solved targets {b0 + len(chunk)}/{len(seeds)} "
            f"({time.perf_counter() - t0:.1f} s; sweeps {min(i.sweeps for i in infos)}.."
            f"{max(i.sweeps for i in infos)})")
    return fs, targets


NAMES = ("A_fp64", "B_fp32_refined", "C_cnn_fp32_refined", "D_cnn_always")


def evaluate(ms, wsm, net, n, seeds, tol):
    import torch
    rows = []
    for s in seeds:
        u, f = instance(n, s)
        fd = ms.field_from(f)
        row = {"seed": s}
        xa = None
        for name in NAMES:
            x = ms.field_from(u)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            used_guess = False
            if name in ("C_cnn_fp32_refined", "D_cnn_always"):
                net.guess(x, fd, x)
                r_guess = ms.residual_norm(x, fd)
                r_zero = ms.residual_norm(ms.field_from(u), fd)
                used_guess = name == "D_cnn_always" or r_guess < r_zero
                if not used_guess:
                    x.copy_(ms.field_from(u))
                if xa is not None and name == "D_cnn_always":
                    gi, ai = x[1:-1, 1:-1, 1:-1], xa[1:-1, 1:-1, 1:-1]
                    row["guess_rel_error"] = float(torch.linalg.norm(gi - ai) /
                                                   torch.linalg.norm(ai))
            prec = ms.MS_SOLVE_F64 if name == "A_fp64" else ms.MS_SOLVE_F32_REFINED
            info = ms.jacobi_solve(x, fd, precision=prec, rel_tol=tol)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            row[name] = {"seconds": dt, "sweeps": info.sweeps, "rel_final": info.rel_final,
                         "outer": info.outer_iters}
            if name == "A_fp64":
                xa = x
            if name in ("C_cnn_fp32_refined", "D_cnn_always"):
                row[name]["guess_used"] = used_guess
                row[name]["guess_rel_residual"] = r_guess / r_zero if r_zero > 0 else 0.0
        rows.append(row)
        log(f"[eval] seed {s}: " + ", ".join(
            f"{k} {row[k]['seconds']:.3f}s/{row[k]['sweeps']}" for k in NAMES)
            + f"; guess rel error {row.get('guess_rel_error', float('nan')):.3e}")
    summ = {}
    for k in NAMES:
        ts = [r[k]["seconds"] for r in rows]
        sw = [r[k]["sweeps"] for r in rows]
        summ[k] = {"mean_seconds": statistics.mean(ts), "median_seconds": statistics.median(ts),
                   "mean_sweeps": statistics.mean(sw), "median_sweeps": statistics.median(sw),
                   "max_rel_final": max(r[k]["rel_final"] for r in rows)}
    summ["C_guess_used_fraction"] = sum(r["C_cnn_fp32_refined"]["guess_used"] for r in rows) / len(rows)
    summ["C_mean_guess_rel_residual"] = statistics.mean(
        r["C_cnn_fp32_refined"]["guess_rel_residual"] for r in rows)
    summ["mean_guess_rel_error"] = statistics.mean(r.get("guess_rel_error", float("nan"))
                                                   for r in rows)
    return summ, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--train", type=int, default=256)
    ap.add_argument("--eval", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="warmstart.npz")
    ap.add_argument("--report", default="warmstart_report.json")
    ap.add_argument("--weights", default=None, help="skip training, evaluate these weights")
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_2310_01882_amd as ms
    from paper_2310_01882_amd import warmstart as wsm

    n = args.n
    report = {"n": n, "train_instances": args.train, "eval_instances": args.eval,
              "epochs": args.epochs, "lr": args.lr}
    if args.weights:
        net = wsm.WarmStart(n, n, n, params=wsm.WarmStart.load_params(args.weights))
    else:
        net = wsm.WarmStart(n, n, n, seed=args.seed)
        t0 = time.perf_counter()
        fs, targets = solve_targets(ms, wsm, net, n, [10000 + i for i in range(args.train)],
                                    args.batch, 1e-10)
        report["target_seconds"] = time.perf_counter() - t0
        zero = ms.alloc_field(n, n, n)
        order = np.random.Generator(np.random.PCG64(args.seed)).permutation
        t0 = time.perf_counter()
        losses = []
        for ep in range(args.epochs):
            tot = torch.zeros((), dtype=torch.float64, device="cuda")
            for i in order(len(fs)):
                tot += net.train_step(zero, fs[i], targets[i], lr=args.lr)
            losses.append(tot.item() / len(fs))
            log(f"[train] epoch {ep + 1}/{args.epochs}: mean loss {losses[-1]:.6e} "
                f"({time.perf_counter() - t0:.1f} s)")
        report["train_seconds"] = time.perf_counter() - t0
        report["epoch_losses"] = losses
        net.save(args.out)
        del fs, targets
        torch.cuda.empty_cache()
    summ, rows = evaluate(ms, wsm, net, n, [20000 + i for i in range(args.eval)], 1e-8)
    report["summary"] = summ
    report["rows"] = rows
    with open(args.report, "w") as fh:
        json.dump(report, fh, indent=1)
    print(json.dumps(summ), flush=True)


if __name__ == "__main__":
    main()
