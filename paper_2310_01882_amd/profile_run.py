"""Small, fixed workloads for rocprofv3 runs (kernel traces and HBM counters).

    python -m paper_2310_01882_amd.profile_run sweep   [--dtype f64|f32] [--sweeps N] [--tb 1|2] [--rb]
    python -m paper_2310_01882_amd.profile_run advect  [--passes N]
    python -m paper_2310_01882_amd.profile_run batched [--streams W]
    python -m paper_2310_01882_amd.profile_run cnn     [--steps N]
    python -m paper_2310_01882_amd.profile_run jit     [--program jacobi|advection] [--passes N]
    python -m paper_2310_01882_amd.profile_run copy    [--mib M]

`sweep` runs N sweeps of the 512^3 Poisson workload (8 Gaussian sources,
seed 1, zero start) on aligned fields, with the launch geometry the
benchmark uses (--tb 2: two sweeps per pass; --rb: red-black Gauss-Seidel
sweeps instead). `advect` runs N passes of the
512 x 512 x 256 advection term. `batched` autotunes and then solves the
benchmark's batch (64 instances, sizes log-uniform in [32, 256], seed 4,
FP32-refined to 1e-8) once (--streams W: on W concurrent streams instead,
without the autotuning). `cnn` runs N training steps (forward, backward,
Adam) of the warm-start network on a 128^3 instance. `jit` compiles the
Jacobi (or advection) program of the stencil-program language and runs it N
times on the sweep (or advection) input. `copy` is the
calibration kernel of known size: one device-to-device tensor copy of M MiB
(reads M MiB, writes M MiB), used to scale the FETCH_SIZE / WRITE_SIZE
counters.
"""

from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["sweep", "advect", "batched", "cnn", "copy", "jit"])
    ap.add_argument("--tb", type=int, default=1, choices=[1, 2])
    ap.add_argument("--rb", action="store_true")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--sweeps", type=int, default=10)
    ap.add_argument("--passes", type=int, default=5)
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--program", default="jacobi", choices=["jacobi", "advection"])
    ap.add_argument("--streams", type=int, default=0)
    ap.add_argument("--n", type=int, default=512)
    args = ap.parse_args()

    import torch

    import paper_2310_01882_amd as ms
    import synth

    if args.what == "copy":
        n = args.mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"copy of {args.mib} MiB x 3 done", flush=True)
        return
    if args.what == "sweep":
        n = args.n
        dt = torch.float64 if args.dtype == "f64" else torch.float32
        f = ms.field_from(synth.gaussian_sources(n, n, n, 8, 1), dt)
        u = ms.alloc_field(n, n, n, dt)
        tmp = ms.alloc_field(n, n, n, dt)
        res = torch.zeros(args.sweeps + 1, dtype=torch.float64, device="cuda")
        if args.rb:
            ms.rbgs_sweeps(u, tmp, args.sweeps, f=f, res=res)
        else:
            ms.jacobi_sweeps(u, tmp, args.sweeps, f=f, res=res, temporal_block=args.tb)
        torch.cuda.synchronize()
        kind = "red-black Gauss-Seidel" if args.rb else f"temporal block {args.tb}"
        print(f"{args.sweeps} sweeps ({kind}) of {n}^3 ({args.dtype}) done; "
              f"final residual {res[-1].item():.6e}", flush=True)
        return
    if args.what == "batched":
        dims = synth.batch_sizes(64, 4)
        xs = [ms.field_from(synth.zeros(*d)) for d in dims]
        fs = [ms.field_from(synth.gaussian_sources(*d, 8, 1000 + i)) for i, d in enumerate(dims)]
        opts = dict(precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8, max_outer=40)
        if args.streams > 0:
            infos = ms.jacobi_solve_batched_streams(xs, fs, workers=args.streams, **opts)
            print(f"batched solve on {args.streams} streams done: "
                  f"{sum(i.sweeps for i in infos)} inner sweeps", flush=True)
            return
        ms.batched_autotune(xs, fs, sweeps_per_trial=20, **opts)
        print("batched autotune done", flush=True)
        infos = ms.jacobi_solve_batched(xs, fs, **opts)
        print(f"batched solve done: {sum(i.sweeps for i in infos)} inner sweeps", flush=True)
        return
    if args.what == "cnn":
        from paper_2310_01882_amd import warmstart as wsm
        n = 128
        net = wsm.WarmStart(n, n, n, seed=0)
        u = ms.alloc_field(n, n, n)
        f = ms.field_from(synth.gaussian_sources(n, n, n, 4, 7))
        solved = ms.alloc_field(n, n, n)  # a stand-in solution: the time does not depend on it
        for _ in range(args.steps):
            net.train_step(u, f, solved)
        torch.cuda.synchronize()
        print(f"{args.steps} warm-start training steps at {n}^3 done", flush=True)
        return
    if args.what == "jit":
        from paper_2310_01882_amd.programs import ADVECTION, JACOBI
        if args.program == "jacobi":
            n = args.n
            f = ms.field_from(synth.gaussian_sources(n, n, n, 8, 1))
            u = ms.alloc_field(n, n, n)
            o = ms.alloc_field(n, n, n)
            jac = ms.JitStencil(JACOBI)
            for _ in range(args.passes):
                jac.apply([u, f], [o])
            torch.cuda.synchronize()
            print(f"{args.passes} compiled Jacobi passes at {n}^3 done", flush=True)
            return
        nx, ny, nz = 512, 512, 256
        u, v, w = (ms.field_from(a) for a in synth.velocity_fields(nx, ny, nz, 2))
        t1, t2 = (torch.from_numpy(a).cuda() for a in synth.tzc_arrays(nz, 3))
        outs = [ms.alloc_field(nx, ny, nz) for _ in range(3)]
        adv = ms.JitStencil(ADVECTION)
        for _ in range(args.passes):
            adv.apply([u, v, w], outs, [0.25, 0.25], [t1, t2])
        torch.cuda.synchronize()
        print(f"{args.passes} compiled advection passes done", flush=True)
        return
    nx, ny, nz = 512, 512, 256
    u, v, w = (ms.field_from(a) for a in synth.velocity_fields(nx, ny, nz, 2))
    t1, t2 = (torch.from_numpy(a).cuda() for a in synth.tzc_arrays(nz, 3))
    outs = [ms.alloc_field(nx, ny, nz) for _ in range(3)]
    for _ in range(args.passes):
        ms.advect_source(u, v, w, t1, t2, 0.25, 0.25, *outs)
    torch.cuda.synchronize()
    print(f"{args.passes} advection passes done", flush=True)


if __name__ == "__main__":
    main()
