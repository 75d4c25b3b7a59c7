#!/usr/bin/env python3
"""Benchmark of the stencil hot path on one MI355X.

Default workload (the headline): 7-point FP64 Jacobi on a 512^3 interior
with a one-cell zero Dirichlet halo, right-hand side = 8 Gaussian sources
(seed 1), zero start; one step = 1000 sweeps, each with the residual norm
of its input fused in, plus the trailing residual of the last iterate.
Inputs are generated on the host, copied to HBM, and resident before the
timed region. Prints ONE JSON line on stdout (progress goes to stderr).

    python bench.py [--steps K] [--warmup W] [--mode jacobi|f32|advect|solve|batched]

Other modes time the FP32-storage sweeps (same grid), the advection source
term (512 x 512 x 256, one pass per step), the time to a 1e-8 relative
residual at 128^3 for plain FP64 vs FP32-refined solves, and the batched
persistent solve of 64 uneven instances (FP32-refined to 1e-8; one step =
one batch).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
METRIC = "GLUP/s + %HBM peak, 512\u00b3 Jacobi; time-to-1e-8 residual plain vs learned/FP32"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def traffic_for(kernel_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when absent or taken on different kernel sources."""
    from paper_2310_01882_amd.profile_summary import source_hash
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel_key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != source_hash(kernel_key):
        return None
    return rec.get("bytes_per_launch")


def cpu_threads():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def event_time(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        fn()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / 1e3  # seconds


def bench_jacobi(args, dtype_name="f64"):
    import numpy as np
    import torch
    import paper_2310_01882_amd as ms
    import synth

    n, sweeps = args.n, args.sweeps
    np_dt = np.float64 if dtype_name == "f64" else np.float32
    log(f"[bench] generating 512^3-class inputs n={n} ({dtype_name})")
    f_h = synth.gaussian_sources(n, n, n, 8, 1)
    u_h = synth.zeros(n, n, n)
    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype_name == "f64" else torch.float32
    # aligned layout: interior rows start on 128-byte boundaries
    u = ms.field_from(u_h, tdt)
    tmp = ms.field_from(u_h, tdt)
    f = ms.field_from(f_h, tdt)
    res = torch.zeros(sweeps + 1, dtype=torch.float64, device=dev)
    work = ms.jacobi_sweeps_workspace(u)
    stream = torch.cuda.current_stream()

    def step():
        ms.jacobi_sweeps(u, tmp, sweeps, f=f, res=res, work=work, stream=stream)

    log(f"[bench] warmup {args.warmup} + timed {args.steps} steps of {sweeps} sweeps")
    secs = event_time(step, args.steps, args.warmup, stream)
    # the same workload with two sweeps fused per pass (temporal blocking)
    tb_secs = event_time(lambda: ms.jacobi_sweeps(u, tmp, sweeps, f=f, res=res, work=work,
                                                  stream=stream, temporal_block=2),
                         args.steps, args.warmup, stream)
    tb_glups = n ** 3 * sweeps * args.steps / tb_secs / 1e9
    # red-black Gauss-Seidel sweeps on the same inputs (one sweep per pass)
    gs_secs = event_time(lambda: ms.rbgs_sweeps(u, tmp, sweeps, f=f, res=res, work=work,
                                                stream=stream),
                         args.steps, args.warmup, stream)
    cells = n ** 3
    lups = cells * sweeps * args.steps
    glups = lups / secs / 1e9
    bpl = 24 if dtype_name == "f64" else 12  # read u and f, write u'
    launch_s = secs / (sweeps * args.steps)  # every sweep launch, trailing passes included
    achieved = bpl * cells / launch_s / 1e9
    log(f"[bench] {glups:.1f} GLUP/s, {achieved:.0f} GB/s algorithmic, "
        f"{launch_s * 1e6:.1f} us per sweep launch; final residual {res[-1].item():.6e}")
    key = f"jacobi7_{dtype_name}_{n}"
    traffic = traffic_for(key)
    tb_traffic = traffic_for(f"jacobi7tb2_{dtype_name}_{n}")
    gs_traffic = traffic_for(f"jacobi7rbgs_{dtype_name}_{n}")
    gs_launch = gs_secs / (sweeps * args.steps)
    ceiling = stream_ceiling()
    cpu = None
    del u, tmp, f
    torch.cuda.empty_cache()
    ttt = None if args.no_solve else time_to_tolerance(args)
    if not args.no_cpu_baseline:
        workers = min(16, cpu_threads())
        cpu = cpu_baseline_jacobi_all_cores(u_h, f_h, np_dt, args.cpu_sweeps_all, workers)
        log(f"[bench] cpu baseline on {workers} processes: {cpu['value']} GLUP/s")
        cpu["one_core"] = cpu_baseline_jacobi(u_h, f_h, np_dt, args.cpu_sweeps)
    out = {
        "metric": METRIC if dtype_name == "f64"
        else "GLUP/s (FP32-storage 7-point Jacobi sweeps, 512^3, FP64 norms)",
        "value": round(glups, 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_name,
        "data": "synthetic",
        "config": {
            "workload": f"jacobi7_{dtype_name}_{n}cubed_{sweeps}sweeps",
            "interior": [n, n, n],
            "halo": 1,
            "sweeps_per_step": sweeps,
            "rhs": "8 Gaussian sources (seed 1)",
            "boundary": "zero Dirichlet",
            "residual": "fused per sweep + trailing pass",
            "parallelism": "single GPU",
        },
        "gb_per_s_algorithmic": round(achieved, 1),
        "pct_hbm_peak": round(100 * achieved / HBM_PEAK_GBS, 2),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "sweep_rt_kernel<%s> (register-tiled)" % ("double" if dtype_name == "f64" else "float"),
            "bytes_per_launch_algorithmic": bpl * cells,
            "avg_launch_us": round(launch_s * 1e6, 3),
        },
        "cpu_baseline": cpu,
        "paper_context": ("the paper's only absolute figure for this sweep: about 70 GLUP/s "
                          "(70,000 MCells/s) on 8192 cores of ARCHER2 (64 nodes of 2x64-core "
                          "AMD EPYC 7742), 17e9 cells, MPI (Section 4.4); other hardware and "
                          "scale, context only"),
        "temporal_block_2": {
            "glups": round(tb_glups, 3),
            "ms_per_step": round(tb_secs / args.steps * 1e3, 4),
            "gb_per_s_algorithmic": round(bpl / 2 * n ** 3 * sweeps * args.steps / tb_secs / 1e9, 1),
            "traffic_per_pass": tb_traffic,
            "gb_per_s_measured": (round(tb_traffic * (sweeps // 2) * args.steps / tb_secs / 1e9, 1)
                                  if tb_traffic else None),
            "note": "two sweeps per pass over memory: 12 B/LUP (FP64) algorithmic",
        },
        "red_black_gauss_seidel": {
            "kernel": "sweep_tbw_kernel<%s, true, true>" % ("double" if dtype_name == "f64"
                                                           else "float"),
            "glups": round(cells * sweeps * args.steps / gs_secs / 1e9, 3),
            "ms_per_step": round(gs_secs / args.steps * 1e3, 4),
            "avg_launch_us": round(gs_launch * 1e6, 3),
            "gb_per_s_algorithmic": round(bpl * cells / gs_launch / 1e9, 1),
            "traffic_per_sweep": gs_traffic,
            "gb_per_s_measured": round(gs_traffic / gs_launch / 1e9, 1) if gs_traffic else None,
            "note": ("one red-black Gauss-Seidel sweep per pass over memory, "
                     f"{bpl} B/LUP algorithmic; asymptotically one such sweep reduces the "
                     "error as much as two Jacobi sweeps (rate rho_J^2)"),
        },
        "hbm_stream_ceiling": ceiling,
        "time_to_1e8_128cubed": ttt,
        "host": host_info(),
    }
    return out


def bench_slab(args):
    """One rank's z-slab share of the 512^3 FP64 sweep (design only: the
    multi-GPU exchange is not built). Its own mode, so that the headline
    run's kernel statistics cover the 512^3 sweep alone."""
    import torch
    import synth
    n = args.n
    f_h = synth.gaussian_sources(n, n, n, 8, 1)
    out = slab_share(n, torch.float64, f_h)
    return {"metric": "GLUP/s (one rank's 512x512x64 z-slab of the 512^3 FP64 sweep)",
            "value": out["glups"], "unit": "GLUP/s", "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": round(out["us_per_sweep"] * 200 / 1e3, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "jacobi7_f64_512x512x64_slab", "parallelism": "single GPU"},
            "slab": out}


def slab_share(n, tdt, f_full, ranks=8, sweeps=200):
    """One rank's share of the same grid split into `ranks` z-slabs
    (n x n x n/ranks interior, the same sources cut to the slab), swept alone:
    the kernel time a multi-GPU sweep would overlap its halo exchange with.
    A z-slab's halo is one contiguous plane (plane pitch sz), so no pack or
    unpack kernel is needed; the exchange itself is not implemented here."""
    import torch
    import paper_2310_01882_amd as ms
    import synth
    nz = n // ranks
    f_h = f_full[: nz + 2]
    u = ms.field_from(synth.zeros(n, n, nz), tdt)
    tmp = ms.field_from(synth.zeros(n, n, nz), tdt)
    f = ms.field_from(f_h, tdt)
    work = ms.jacobi_sweeps_workspace(u)
    stream = torch.cuda.current_stream()
    secs = event_time(lambda: ms.jacobi_sweeps(u, tmp, sweeps, f=f, work=work, stream=stream),
                      1, 1, stream)
    us = secs / sweeps * 1e6
    plane_bytes = u.stride(0) * u.element_size()
    return {"interior": [n, n, nz], "us_per_sweep": round(us, 2),
            "glups": round(n * n * nz / us / 1e3, 2),
            "halo_plane_bytes": plane_bytes,
            "halo_plane_us_at_153_gbs_xgmi": round(plane_bytes / 153e3, 2)}


def stream_ceiling(mib=1024, reps=20):
    """Achievable HBM bandwidth on this device for the stencils' access
    patterns, from the library's own streaming kernel (ms_stream_probe):
    read-1/write-1 and read-2/write-1 over `mib` MiB arrays, GB/s of bytes
    moved, best over a few grid sizes, timed with events."""
    import torch
    import paper_2310_01882_amd as ms
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    out = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    res = {}
    for name, two in (("read1_write1", False), ("read2_write1", True)):
        best, how = 0.0, None
        for form in (0, 1, 2, 3):
            for blocks in (512, 1024, 2048, 4096):
                def step():
                    ms.stream_probe(a, out, b if two else None, blocks=blocks, form=form,
                                    stream=stream)
                secs = event_time(step, reps, 2, stream)
                gbs = (3 if two else 2) * n * 8 * reps / secs / 1e9
                if gbs > best:
                    best, how = gbs, {"form": form, "blocks": blocks}
        res[name + "_gbs"] = round(best, 1)
        res[name + "_best"] = how
    del a, b, out
    torch.cuda.empty_cache()
    res["kernel"] = "ms_stream_probe (16-byte lanes, nontemporal stores; best form and grid)"
    return res


def host_info():
    """CPU model, threads this process may use, ROCm and HIP versions."""
    import torch
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    rocm = None
    try:
        with open("/opt/rocm/.info/version") as fh:
            rocm = fh.read().strip()
    except OSError:
        pass
    return {"cpu_model": model, "host_threads": cpu_threads(), "rocm": rocm,
            "torch_hip": getattr(torch.version, "hip", None), "torch": torch.__version__}


# ---- the oracle on all host cores: z-slabs of one field in shared memory,
# one process per slab, one sweep (with the residual of its input) per round

_SLAB = {}


def _slab_init(names, shape, dtype):
    from multiprocessing import shared_memory
    import numpy as np
    _SLAB["shm"] = [shared_memory.SharedMemory(name=n) for n in names]
    _SLAB["arr"] = [np.ndarray(shape, dtype=dtype, buffer=m.buf) for m in _SLAB["shm"]]


def _slab_sweep(task):
    """One oracle sweep of planes z0+1 .. z1 (halo-padded indices) of buffer
    `src` into `dst`; returns the slab's sum of squared residuals of the
    input (the oracle's residual on the slab)."""
    import numpy as np
    import oracle
    src, dst, z0, z1 = task
    u, out, f = _SLAB["arr"][src], _SLAB["arr"][dst], _SLAB["arr"][2]
    view, fv = u[z0:z1 + 2], f[z0:z1 + 2]
    if u.dtype == np.float64:
        r = oracle.residual(view, fv)
        new = oracle.jacobi_sweep(view, fv)
    else:
        r = oracle.residual(view.astype(np.float64), fv.astype(np.float64))
        new = oracle.sweep_f32(view, fv)
    out[z0 + 1:z1 + 1, 1:-1, 1:-1] = new[1:-1, 1:-1, 1:-1]
    return float(np.sum(r * r))


def cpu_baseline_jacobi_all_cores(u_h, f_h, np_dt, nsweeps, workers):
    """The oracle as it stands on `workers` host processes: the field is cut
    into z-slabs, each process sweeps its slab with the oracle's own
    jacobi_sweep and residual, the slabs' residual sums are added in slab
    order. Returns the baseline record (and checks that the result equals
    the oracle's whole-field sweeps on a few planes)."""
    import multiprocessing as mp
    from multiprocessing import shared_memory
    import numpy as np
    shape = u_h.shape
    nbytes = int(np.prod(shape)) * np.dtype(np_dt).itemsize
    shms = [shared_memory.SharedMemory(create=True, size=nbytes) for _ in range(3)]
    try:
        arrs = [np.ndarray(shape, dtype=np_dt, buffer=m.buf) for m in shms]
        arrs[0][...] = u_h
        arrs[1][...] = u_h
        arrs[2][...] = f_h
        nz = shape[0] - 2
        cuts = [round(nz * i / workers) for i in range(workers + 1)]
        ctx = mp.get_context("spawn")
        with ctx.Pool(workers, initializer=_slab_init,
                      initargs=([m.name for m in shms], shape, np_dt)) as pool:
            pool.map(_slab_sweep, [(0, 1, cuts[i], cuts[i + 1]) for i in range(workers)])
            arrs[1][...] = u_h  # the warm-up pass above is not counted
            t = time.perf_counter()
            norms = []
            for k in range(nsweeps):
                src, dst = k % 2, 1 - k % 2
                parts = pool.map(_slab_sweep, [(src, dst, cuts[i], cuts[i + 1])
                                              for i in range(workers)])
                norms.append(math.sqrt(sum(parts)))
            dt = time.perf_counter() - t
        cells = (shape[0] - 2) * (shape[1] - 2) * (shape[2] - 2)
        return {"value": round(cells * nsweeps / dt / 1e9, 5), "unit": "GLUP/s",
                "cores": workers, "kind": "oracle",
                "sample": (f"{nsweeps} sweeps + residual norms of the same 512^3 input: the "
                           f"oracle's own sweep and residual on {workers} z-slabs, one process "
                           "per slab (numpy)"),
                "seconds": round(dt, 2), "final_residual": norms[-1]}
    finally:
        for m in shms:
            m.close()
            m.unlink()


def cpu_baseline_jacobi(u_h, f_h, np_dt, nsweeps):
    """The oracle as it stands, timed on the host on a bounded sample of the
    same workload: ``nsweeps`` sweeps of the same 512^3 input, each with its
    residual norm (what one GPU sweep launch computes)."""
    import numpy as np
    import oracle
    log(f"[bench] cpu baseline: {nsweeps} oracle sweeps of the same input")
    u = u_h.astype(np_dt)
    f = f_h.astype(np_dt)
    cells = (u.shape[0] - 2) * (u.shape[1] - 2) * (u.shape[2] - 2)
    t = time.perf_counter()
    for _ in range(nsweeps):
        if np_dt == np.float64:
            oracle.residual_norm(u, f)
            u = oracle.jacobi_sweep(u, f)
        else:
            oracle.residual_norm_f32_storage(u, f)
            u = oracle.sweep_f32(u, f)
    dt = time.perf_counter() - t
    return {
        "value": round(cells * nsweeps / dt / 1e9, 5),
        "unit": "GLUP/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{nsweeps} sweeps + residual norms of the 512^3 input (numpy, one thread)",
        "seconds": round(dt, 2),
        "host_threads_available": cpu_threads(),
    }


def bench_advect(args):
    import numpy as np
    import torch
    import paper_2310_01882_amd as ms
    import synth

    nx, ny, nz = 512, 512, 256
    log("[bench] generating advection inputs 512x512x256")
    u_h, v_h, w_h = synth.velocity_fields(nx, ny, nz, 2)
    t1_h, t2_h = synth.tzc_arrays(nz, 3)
    dev = torch.device("cuda:0")
    u, v, w = (ms.field_from(a) for a in (u_h, v_h, w_h))
    t1, t2 = torch.from_numpy(t1_h).to(dev), torch.from_numpy(t2_h).to(dev)
    su, sv, sw = (ms.alloc_field(nx, ny, nz) for _ in range(3))
    stream = torch.cuda.current_stream()

    def step():
        ms.advect_source(u, v, w, t1, t2, 0.25, 0.25, su, sv, sw, stream=stream)

    passes = max(args.steps, 1) * 20
    secs = event_time(step, passes, max(args.warmup, 1) * 5, stream)
    cells = nx * ny * nz
    gcells = cells * passes / secs / 1e9
    achieved = 48 * cells / (secs / passes) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        sl = slice(0, 34)  # 32 interior levels
        t = time.perf_counter()
        oracle.advect_source(u_h[sl], v_h[sl], w_h[sl], t1_h[:32], t2_h[:32], 0.25, 0.25)
        dt = time.perf_counter() - t
        cpu = {"value": round(nx * ny * 32 / dt / 1e9, 5), "unit": "Gcell/s", "cores": 1,
               "kind": "oracle", "sample": "one pass over 32 of the 256 levels (numpy, one thread)",
               "seconds": round(dt, 2)}
    return {
        "metric": "Gcell/s (fused 3-field advection source term, FP64)",
        "value": round(gcells, 3), "unit": "Gcell/s", "n_gpus": 1, "steps": passes,
        "warmup": max(args.warmup, 1) * 5, "ms_per_step": round(secs / passes * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "pw_advection_512x512x256", "interior": [nx, ny, nz],
                   "fields": "16-sinusoid u,v,w (seed 2); tzc1,tzc2 ~U[0.5,2] (seed 3)",
                   "tcx": 0.25, "tcy": 0.25, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_for("advect_512x512x256"),
                     "kernel": "advect_staged_kernel", "bytes_per_launch_algorithmic": 48 * cells,
                     "avg_launch_us": round(secs / passes * 1e6, 3)},
        "cpu_baseline": cpu,
    }


def bench_jit(args):
    """Runtime-compiled stencil programs: the Jacobi update and the
    three-field advection region written in the stencil-program language,
    compiled with hipRTC, run on the benchmark inputs (512^3 FP64; advection
    512 x 512 x 256). `value` is the compiled Jacobi program's throughput;
    the hand-written kernels are timed beside it on the same inputs."""
    import torch
    import paper_2310_01882_amd as ms
    import synth
    from paper_2310_01882_amd.programs import ADVECTION, JACOBI

    n = args.n
    f_h = synth.gaussian_sources(n, n, n, 8, 1)
    u_h = synth.zeros(n, n, n)
    u, f = ms.field_from(u_h), ms.field_from(f_h)
    out, tmp = ms.alloc_field(n, n, n), ms.alloc_field(n, n, n)
    stream = torch.cuda.current_stream()
    t = time.perf_counter()
    jac = ms.JitStencil(JACOBI)
    t_jac = time.perf_counter() - t
    t = time.perf_counter()
    adv = ms.JitStencil(ADVECTION)
    t_adv = time.perf_counter() - t
    launches = max(args.steps, 1) * 100
    warm = max(args.warmup, 1) * 10
    secs = event_time(lambda: jac.apply([u, f], [out], stream=stream), launches, warm, stream)
    hand = event_time(lambda: ms.jacobi_sweeps(u, tmp, 1, f=f, stream=stream), launches, warm,
                      stream)
    cells = n ** 3
    launch_s = secs / launches
    achieved = 24 * cells / launch_s / 1e9
    nx, ny, nz = 512, 512, 256
    uu, vv, ww = (ms.field_from(a) for a in synth.velocity_fields(nx, ny, nz, 2))
    t1, t2 = (torch.from_numpy(a).cuda() for a in synth.tzc_arrays(nz, 3))
    outs = [ms.alloc_field(nx, ny, nz) for _ in range(3)]
    apasses = max(args.steps, 1) * 20
    asecs = event_time(lambda: adv.apply([uu, vv, ww], outs, [0.25, 0.25], [t1, t2],
                                         stream=stream), apasses, warm, stream)
    ahand = event_time(lambda: ms.advect_source(uu, vv, ww, t1, t2, 0.25, 0.25, *outs,
                                                stream=stream), apasses, warm, stream)
    acells = nx * ny * nz
    log(f"[bench] compiled Jacobi {launch_s * 1e6:.1f} us (hand-written "
        f"{hand / launches * 1e6:.1f}); compiled advection {asecs / apasses * 1e6:.1f} us "
        f"(hand-written {ahand / apasses * 1e6:.1f})")
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import stencil_lang
        reps = 3
        log(f"[bench] cpu baseline: {reps} interpreter runs of the Jacobi program at {n}^3")
        t = time.perf_counter()
        for _ in range(reps):
            stencil_lang.run(JACOBI, [u_h, f_h])
        dt = time.perf_counter() - t
        cpu = {"value": round(cells * reps / dt / 1e9, 5), "unit": "GLUP/s", "cores": 1,
               "kind": "oracle", "sample": f"{reps} runs of the Jacobi program on the {n}^3 "
               "input by the oracle's interpreter (numpy, one thread)", "seconds": round(dt, 2)}
    return {
        "metric": "GLUP/s (runtime-compiled 7-point Jacobi program, 512^3 FP64)",
        "value": round(cells / launch_s / 1e9, 3), "unit": "GLUP/s", "n_gpus": 1,
        "steps": launches, "warmup": warm, "ms_per_step": round(launch_s * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"jit_jacobi7_f64_{n}cubed", "interior": [n, n, n],
                   "rhs": "8 Gaussian sources (seed 1)", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_for(f"jit_jacobi_f64_{n}"), "kernel": "ms_jit_kernel_v",
                     "bytes_per_launch_algorithmic": 24 * cells,
                     "avg_launch_us": round(launch_s * 1e6, 3)},
        "compile_seconds": {"jacobi": round(t_jac, 3), "advection": round(t_adv, 3)},
        "hand_written_sweep_us": round(hand / launches * 1e6, 3),
        "advection": {"workload": "pw_advection_512x512x256",
                      "us_per_pass": round(asecs / apasses * 1e6, 3),
                      "gcells": round(acells * apasses / asecs / 1e9, 3),
                      "gb_per_s_algorithmic": round(48 * acells / (asecs / apasses) / 1e9, 1),
                      "traffic": traffic_for("jit_advect_512x512x256"),
                      "hand_written_us": round(ahand / apasses * 1e6, 3)},
        "cpu_baseline": cpu,
    }


def bench_streamed(args):
    """The 512^3 FP64 sweep input held in pinned host memory and swept
    through the device in z slabs (sweeps_per_pass sweeps per trip, slabs of
    slab_planes planes): PCIe-inclusive throughput of a field the device
    does not hold, next to the same sweeps resident in HBM."""
    import torch
    import paper_2310_01882_amd as ms
    import synth

    n = args.n
    f_h = synth.gaussian_sources(n, n, n, 8, 1)
    u_h = synth.zeros(n, n, n)
    hu = torch.from_numpy(u_h).pin_memory()
    ht = torch.from_numpy(u_h).pin_memory()
    hf = torch.from_numpy(f_h).pin_memory()
    sweeps = 64
    rows = {}
    for T, S in ((16, 64), (32, 64), (32, 128), (64, 128)):
        ms.jacobi_sweeps_streamed(hu, ht, T, f=hf, sweeps_per_pass=T, slab_planes=S)  # warm-up
        t = time.perf_counter()
        ms.jacobi_sweeps_streamed(hu, ht, sweeps, f=hf, sweeps_per_pass=T, slab_planes=S)
        dt = time.perf_counter() - t
        rows[f"T{T}_S{S}"] = {"seconds": round(dt, 4),
                              "glups": round(n ** 3 * sweeps / dt / 1e9, 3),
                              "pcie_gb_per_s": round(24 * (n + 2) ** 3 * (sweeps // T) / dt / 1e9,
                                                     1)}
        log(f"[bench] streamed T={T} S={S}: {dt:.3f} s for {sweeps} sweeps "
            f"({rows[f'T{T}_S{S}']['glups']} GLUP/s)")
    best = max(rows, key=lambda k: rows[k]["glups"])
    return {"metric": "GLUP/s (512^3 FP64 Jacobi sweeps of a host-resident field, PCIe included)",
            "value": rows[best]["glups"], "unit": "GLUP/s", "n_gpus": 1, "steps": sweeps,
            "warmup": 1, "ms_per_step": round(rows[best]["seconds"] / sweeps * 1e3, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "jacobi7_f64_512cubed_host_resident", "value_is": best,
                       "parallelism": "single GPU"},
            "runs": rows}


WEIGHTS = os.path.join(ROOT, "paper_2310_01882_amd", "weights", "warmstart_128.npz")


def time_to_tolerance(args, seeds=(20000, 20001, 20002, 20003), tol=1e-8):
    """The metric's second half: seconds to a 1e-8 relative residual at 128^3
    on held-out warm-start instances (seeds 20000+, 1-8 Gaussian sources,
    zero Dirichlet boundary, zero start), solved three ways on this GPU with
    the library defaults (two sweeps per pass):
      A plain FP64 Jacobi,
      B FP32-storage Jacobi inside FP64 refinement,
      C the learned warm start (warmstart_forward: features, network, guess,
        slowest-mode start rule; inside the timed region), then B's solver;
    and, beside them, with red-black Gauss-Seidel sweeps inside the same
    refinement (the library's extension of the paper's Jacobi iteration):
      D from the zero interior, E after the warm start.
    One warm-up solve of each kind first (graphs, caches)."""
    import statistics
    import torch
    import paper_2310_01882_amd as ms
    from paper_2310_01882_amd import warmstart as wsm
    import synth

    n = 128
    net = wsm.WarmStart.from_file(WEIGHTS, n, n, n) if os.path.exists(WEIGHTS) else None
    F64, F32R = ms.MS_SOLVE_F64, ms.MS_SOLVE_F32_REFINED
    names = (["A_fp64", "B_fp32_refined"] + (["C_cnn_fp32_refined"] if net else [])
             + ["D_fp32_refined_rbgs"] + (["E_cnn_fp32_refined_rbgs"] if net else []))
    rows = []
    for rep, seed in enumerate((seeds[0],) + tuple(seeds)):
        u_h = synth.zeros(n, n, n)
        f_h = synth.gaussian_sources(n, n, n, synth.random_source_count(seed), seed)
        f, u0 = ms.field_from(f_h), ms.field_from(u_h)
        row = {"seed": seed}
        for name in names:
            x = ms.field_from(u_h)
            torch.cuda.synchronize()
            t = time.perf_counter()
            cnn = "cnn" in name
            if cnn:
                used, _ = net.guess(u0, f, x, rule="slow_modes")
            method = ms.MS_METHOD_RBGS if name.endswith("rbgs") else ms.MS_METHOD_JACOBI
            info = ms.jacobi_solve(x, f, precision=F64 if name.startswith("A") else F32R,
                                   rel_tol=tol if rep else 1e-3, method=method)
            torch.cuda.synchronize()
            row[name] = {"seconds": round(time.perf_counter() - t, 4), "sweeps": info.sweeps,
                         "rel_final": info.rel_final}
            if cnn:
                row[name]["guess_used"] = bool(used.item())
        if rep:
            rows.append(row)
            log(f"[bench] 128^3 seed {seed}: " + ", ".join(
                f"{k} {row[k]['seconds']:.3f} s / {row[k]['sweeps']}" for k in names))
    out = {"interior": [n, n, n], "tol": tol, "seeds": list(seeds),
           "rhs": "1-8 Gaussian sources per seed (held-out warm-start instances)",
           "boundary": "zero Dirichlet", "start": "zero interior"}
    for name in names:
        out[name] = {"mean_seconds": round(statistics.mean(r[name]["seconds"] for r in rows), 4),
                     "mean_sweeps": statistics.mean(r[name]["sweeps"] for r in rows),
                     "max_rel_final": max(r[name]["rel_final"] for r in rows)}
    if net:
        for name in ("C_cnn_fp32_refined", "E_cnn_fp32_refined_rbgs"):
            out[name]["guess_used"] = [r[name]["guess_used"] for r in rows]
        out["weights"] = os.path.relpath(WEIGHTS, ROOT)
    # the Jacobi pipeline the metric names (C, else B), and the fastest overall
    best = "C_cnn_fp32_refined" if net else "B_fp32_refined"
    out["speedup_vs_A"] = round(out["A_fp64"]["mean_seconds"] / out[best]["mean_seconds"], 3)
    fastest = min(names, key=lambda k: out[k]["mean_seconds"])
    out["fastest"] = {"name": fastest, "speedup_vs_A": round(
        out["A_fp64"]["mean_seconds"] / out[fastest]["mean_seconds"], 3)}
    out["rows"] = rows
    return out


def bench_solve(args):
    """Time to a 1e-8 relative residual at 128^3 (8 Gaussian sources, seed 1,
    zero Dirichlet boundary, zero start) on aligned fields, median of
    --solve-reps timed solves after one warm-up each:
      fp64                     plain FP64 Jacobi, one sweep per pass
      fp64_tb2                 the same with two sweeps per pass (the library default)
      fp32_refined(_tb2)       FP32 sweeps inside FP64 refinement
      fp32_refined_persistent  the same through the persistent batched kernel
      fp64_rbgs, fp32_refined_rbgs
                               red-black Gauss-Seidel sweeps instead of Jacobi
                               (plain FP64, and inside the refinement); reported
                               beside the Jacobi variants, not used for `value`
      cnn_fp32_refined         the trained warm start's guess (zero interior
                               if its residual is not smaller), then the
                               fastest FP32-refined variant; the guess's
                               features and forward pass are inside the
                               timed region (needs the committed weights)
    `value` is cnn_fp32_refined when the weights are present, else the
    fastest FP32-refined variant; `speedup_vs_fp64` compares it with the
    faster plain FP64 schedule."""
    import statistics
    import torch
    import paper_2310_01882_amd as ms
    import synth

    n = args.solve_n
    f_h = synth.gaussian_sources(n, n, n, 8, 1)
    u_h = synth.zeros(n, n, n)
    f = ms.field_from(f_h)
    u0 = ms.field_from(u_h)

    def fresh():  # a new aligned field holding the zero start (clone() drops the padding)
        return ms.field_from(u_h)

    # tile shapes from the autotuner for both storage precisions (the FP32
    # inner sweeps run on workspace grids with the same extents and alignment)
    t0 = time.perf_counter()
    tuned = {"f64": ms.autotune_sweeps(fresh(), fresh(), f)}
    f32 = ms.field_from(f_h, torch.float32)
    tuned["f32"] = ms.autotune_sweeps(ms.field_from(u_h, torch.float32),
                                      ms.field_from(u_h, torch.float32), f32)
    log(f"[bench] autotuned sweep shapes in {time.perf_counter() - t0:.2f} s: {tuned}")
    F64, F32R = ms.MS_SOLVE_F64, ms.MS_SOLVE_F32_REFINED
    # reference answer for the field errors: FP64 Jacobi to a 1e-10 relative residual
    x_ref = fresh()
    ms.jacobi_solve(x_ref, f, precision=F64, rel_tol=1e-10)
    ref_norm = torch.linalg.vector_norm(x_ref).item()

    def field_error(x):
        return torch.linalg.vector_norm(x - x_ref).item() / ref_norm

    RB = ms.MS_METHOD_RBGS
    variants = [("fp64", dict(precision=F64, temporal_block=1)),
                ("fp64_tb2", dict(precision=F64, temporal_block=2)),
                ("fp32_refined", dict(precision=F32R, temporal_block=1)),
                ("fp32_refined_tb2", dict(precision=F32R, temporal_block=2)),
                ("fp64_rbgs", dict(precision=F64, method=RB)),
                ("fp32_refined_rbgs", dict(precision=F32R, method=RB))]
    rows = {}

    def record(name, times, info, x):
        dt = statistics.median(times)
        rows[name] = {"seconds": round(dt, 4), "seconds_all": [round(t, 4) for t in times],
                      "sweeps": info.sweeps, "outer": info.outer_iters,
                      "rel_final": info.rel_final,
                      "field_rel_error_vs_fp64_1e-10": field_error(x),
                      "glups": round(n ** 3 * info.sweeps / dt / 1e9, 2)}
        log(f"[bench] {name}: {dt:.3f} s, {info.sweeps} sweeps, rel {info.rel_final:.3e}")

    for name, kw in variants:
        work = ms.jacobi_workspace(u0, ms.solve_opts(**kw))
        ms.jacobi_solve(fresh(), f, work=work, rel_tol=1e-3, **kw)  # warm-up (graphs, caches)
        times = []
        for _ in range(args.solve_reps):
            u = fresh()
            torch.cuda.synchronize()
            t = time.perf_counter()
            info = ms.jacobi_solve(u, f, work=work, rel_tol=1e-8, **kw)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
        record(name, times, info, u)
    times = []
    for rep in range(args.solve_reps + 1):
        u = fresh()
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = ms.jacobi_solve_batched([u], [f], precision=F32R, rel_tol=1e-8 if rep else 1e-3)[0]
        torch.cuda.synchronize()
        if rep:
            times.append(time.perf_counter() - t)
    record("fp32_refined_persistent", times, info, u)
    fp32_names = ["fp32_refined", "fp32_refined_tb2", "fp32_refined_persistent"]
    best32 = min(fp32_names, key=lambda k: rows[k]["seconds"])
    value_name = best32
    if os.path.exists(WEIGHTS):
        from paper_2310_01882_amd import warmstart as wsm
        net = wsm.WarmStart.from_file(WEIGHTS, n, n, n)
        kw = dict(variants)[best32] if best32 != "fp32_refined_persistent" else None
        times, used = [], []
        for rep in range(args.solve_reps + 1):
            x = fresh()
            torch.cuda.synchronize()
            t = time.perf_counter()
            use, _ = net.guess(x, f, x)
            tol = 1e-8 if rep else 1e-3
            if kw is None:
                info = ms.jacobi_solve_batched([x], [f], precision=F32R, rel_tol=tol)[0]
            else:
                info = ms.jacobi_solve(x, f, rel_tol=tol, **kw)
            torch.cuda.synchronize()
            if rep:
                times.append(time.perf_counter() - t)
                used.append(bool(use.item()))
        record("cnn_fp32_refined", times, info, x)
        rows["cnn_fp32_refined"]["solver"] = best32
        rows["cnn_fp32_refined"]["guess_used"] = used
        value_name = "cnn_fp32_refined"
    v = rows[value_name]["seconds"]
    return {
        "metric": "seconds to 1e-8 relative residual (128^3 Poisson): learned/FP32 vs plain FP64",
        "value": v, "unit": "s", "n_gpus": 1, "steps": args.solve_reps, "warmup": 1,
        "ms_per_step": round(v * 1e3, 2), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"poisson_{n}cubed_to_1e-8", "rhs": "8 Gaussian sources (seed 1)",
                   "boundary": "zero Dirichlet", "value_is": value_name,
                   "parallelism": "single GPU"},
        "sweep_shapes": tuned,
        "speedup_vs_fp64": round(min(rows["fp64"]["seconds"],
                                     rows["fp64_tb2"]["seconds"]) / v, 3),
        "solves": rows,
    }


def est_sweeps(dims, tol=1e-8):
    """Jacobi sweeps for the slowest mode to decay by `tol`: the upper bound
    the batched planner's data-aware estimate is kept under."""
    rho = sum(math.cos(math.pi / (n + 1)) for n in dims) / 3.0
    return math.log(tol) / math.log(rho)


def bench_batched(args):
    """64 instances, per-axis sizes log-uniform in [32, 256] (seed 4), each with
    8 Gaussian sources (seed 1000 + i) and a zero Dirichlet boundary, solved
    from zero to a 1e-8 relative residual by FP32 sweeps inside FP64
    refinement, two ways: all in one persistent launch per step (tile shapes
    from the batched autotuner, run once before the timed region), and on
    4, 8 and 16 concurrent streams (each instance solved as jacobi_solve
    does, largest estimated work first). `value` is the persistent launch (the
    configuration's form); the streams figure is reported beside it."""
    import numpy as np
    import torch
    import paper_2310_01882_amd as ms
    import synth

    dims = synth.batch_sizes(64, 4)
    log(f"[bench] generating 64 batched instances ({sum(a * b * c for a, b, c in dims) / 1e6:.1f}"
        " M cells)")
    probs = [(synth.zeros(*d), synth.gaussian_sources(*d, 8, 1000 + i))
             for i, d in enumerate(dims)]
    x0 = [ms.field_from(u) for u, _ in probs]
    xs = [ms.field_from(u) for u, _ in probs]
    fs = [ms.field_from(f) for _, f in probs]
    opts = dict(precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8, max_outer=40)
    stream = torch.cuda.current_stream()
    cells = np.array([a * b * c for a, b, c in dims], dtype=np.float64)

    def reset():
        for x, a in zip(xs, x0):
            x.copy_(a)
        torch.cuda.synchronize()

    def timed_batch(label):
        reset()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        infos = ms.jacobi_solve_batched(xs, fs, stream=stream, **opts)
        e1.record(stream)
        torch.cuda.synchronize()
        dt = e0.elapsed_time(e1) / 1e3
        log(f"[bench] {label}: {dt:.3f} s, sweeps {min(i.sweeps for i in infos)}.."
            f"{max(i.sweeps for i in infos)}, worst rel {max(i.rel_final for i in infos):.3e}")
        return dt, infos

    ms.batch_tuning_clear()
    untuned_s, _ = timed_batch("default tile shapes")
    t = time.perf_counter()
    best = ms.batched_autotune(xs, fs, sweeps_per_trial=20, **opts)
    tune_s = time.perf_counter() - t
    shapes = {}
    for b in best:
        key = f"{b['tx']}x{b['zsplit']}"
        shapes[key] = shapes.get(key, 0) + 1
    log(f"[bench] autotune {tune_s:.2f} s; shapes (tx x zsplit): {shapes}")
    for _ in range(args.warmup):
        timed_batch("warm-up")
    secs, infos = [], None
    for k in range(args.steps):
        dt, infos = timed_batch(f"step {k + 1}/{args.steps}")
        secs.append(dt)
    mean_s = sum(secs) / len(secs)
    # the same batch on concurrent streams (a side figure: not one launch)
    stream_s, stream_infos = {}, {}
    for rep, w in enumerate((8, 4, 8, 16)):  # the first run warms up graphs and caches
        reset()
        t = time.perf_counter()
        sinfos = ms.jacobi_solve_batched_streams(xs, fs, workers=w, stream=stream, **opts)
        torch.cuda.synchronize()
        dt = round(time.perf_counter() - t, 4)
        log(f"[bench] streams x{w}{' (warm-up)' if rep == 0 else ''}: {dt:.3f} s, sweeps "
            f"{min(i.sweeps for i in sinfos)}..{max(i.sweeps for i in sinfos)}, worst rel "
            f"{max(i.rel_final for i in sinfos):.3e}")
        if rep:
            stream_s[w], stream_infos[w] = dt, sinfos
    best_w = min(stream_s, key=stream_s.get)
    # per-team finish times (device clock): the batch ends with its slowest team
    fin = np.array([i.seconds for i in infos])
    teams, grid_blocks, planned, groups = ms.batched_plan(xs, fs, with_estimates=True,
                                                          with_groups=True, **opts)
    # a team runs its chain of instances one after the other: it is busy
    # until its last instance finishes
    team_end, team_size = {}, {}
    for e, t, k in zip(fin, teams, groups):
        team_end[k] = max(team_end.get(k, 0.0), float(e))
        team_size[k] = t
    order = np.argsort(-fin)
    for i in order[:4]:
        log(f"[bench]   slowest: instance {i} dims {dims[i]} team {teams[i]} sweeps "
            f"{infos[i].sweeps} finished at {fin[i]:.2f} s")
    # The configuration asks for one persistent launch: that is `value`. The
    # stream-parallel run is reported beside it with its own sweep counts.
    def work_of(inf, inner_bytes):
        sw = np.array([i.sweeps for i in inf], dtype=np.float64)
        ou = np.array([i.outer_iters for i in inf], dtype=np.float64)
        # algorithmic HBM bytes: inner_bytes per FP32 inner update (e, rhat in
        # and e out once per pass: 12, or 6 with two sweeps per pass); per
        # outer step 16 (norm: x, f) + 24 (rhat: x, f in; rhat, e0 out) + 20
        # (update: x, e in; x out) per cell; 16 per cell for the first norm
        return (sw, ou, float((cells * sw).sum()),
                float((cells * (inner_bytes * sw + 60 * ou + 16)).sum()))

    # the persistent kernel sweeps twice per pass unless MS_BATCH_TB=1; the
    # stream path's column kernel always does
    per_pass = 1 if os.environ.get("MS_BATCH_TB") == "1" else 2
    sweeps, outer, lups, nbytes = work_of(infos, 12 / per_pass)
    value_s = mean_s
    value_is = "persistent"
    glups = lups / value_s / 1e9
    achieved = nbytes / value_s / 1e9
    _, _, s_lups, s_bytes = work_of(stream_infos[best_w], 6)
    streams_side = {"workers": best_w, "seconds": stream_s[best_w],
                    "glups": round(s_lups / stream_s[best_w] / 1e9, 3),
                    "gb_per_s_algorithmic": round(s_bytes / stream_s[best_w] / 1e9, 1),
                    "note": "each instance a plain jacobi_solve, instances on concurrent "
                            "streams (not one launch); warm-up run excluded"}
    # the same instances one by one through the single-instance solve
    seq = None
    if not args.no_sequential:
        reset()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for x, f in zip(xs, fs):
            ms.jacobi_solve(x, f, stream=stream, **opts)
        t1.record(stream)
        torch.cuda.synchronize()
        seq = round(t0.elapsed_time(t1) / 1e3, 4)
        log(f"[bench] the same 64 solves one by one: {seq:.3f} s")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        sample = probs[:6]
        t = time.perf_counter()
        lup = 0
        for u, f in sample:
            uf, ff = u.astype(np.float32), f.astype(np.float32)
            for _ in range(2):
                oracle.residual_norm_f32_storage(uf, ff)
                uf = oracle.sweep_f32(uf, ff)
            lup += 2 * (u.shape[0] - 2) * (u.shape[1] - 2) * (u.shape[2] - 2)
        dt = time.perf_counter() - t
        cpu = {"value": round(lup / dt / 1e9, 5), "unit": "GLUP/s", "cores": 1, "kind": "oracle",
               "sample": "2 FP32 sweeps + FP64 norms of each of the first 6 instances "
                         "(numpy, one thread)", "seconds": round(dt, 2)}
    return {
        "metric": "GLUP/s (batched FP32-refined Poisson solves to 1e-8, 64 instances)",
        "value": round(glups, 3), "unit": "GLUP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(value_s * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "batched_poisson_64x_loguniform_32_256_to_1e-8",
                   "instances": 64, "size_seed": 4, "cells": int(cells.sum()),
                   "rhs": "8 Gaussian sources per instance (seed 1000+i)",
                   "boundary": "zero Dirichlet", "parallelism": "single GPU",
                   "value_is": value_is, "inner_sweeps_per_pass": per_pass},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_for("batched_64x"),
                     "kernel": f"batched_kernel<{str(per_pass == 2).lower()}> (one persistent "
                               "launch per step)",
                     "bytes_per_launch_algorithmic": nbytes,
                     "avg_launch_us": round(value_s * 1e6, 1)},
        "cpu_baseline": cpu,
        "streams": streams_side,
        "batch": {"seconds_tuned": round(mean_s, 4), "seconds_default_shapes": round(untuned_s, 4),
                  "seconds_streams": stream_s,
                  "autotune_seconds": round(tune_s, 3), "shapes": shapes,
                  "seconds_one_by_one": seq, "total_inner_sweeps": int(sweeps.sum()),
                  "max_sweeps": int(sweeps.max()), "outer_max": int(outer.max()),
                  "worst_rel_final": max(i.rel_final for i in infos),
                  "grid_blocks": grid_blocks, "teams": len(team_size),
                  "team_finish_seconds": {"min": round(min(team_end.values()), 3),
                                          "median": round(float(np.median(
                                              list(team_end.values()))), 3),
                                          "max": round(max(team_end.values()), 3)},
                  "block_seconds_busy_fraction": round(
                      sum(team_end[k] * team_size[k] for k in team_end) /
                      (max(team_end.values()) * grid_blocks), 3),
                  "instances": [{"dims": list(d), "team": t, "group": k,
                                 "shape": [b["tx"], b["zsplit"]],
                                 "sweeps": i.sweeps, "est_sweeps": round(pe),
                                 "est_sweeps_slowest_mode_bound": round(est_sweeps(d)),
                                 "finish_s": round(float(e), 3)}
                                for d, t, k, b, i, e, pe in zip(dims, teams, groups, best,
                                                                infos, fin, planned)],
                  "plan_estimate_error": {
                      "mean_abs": round(float(np.mean([abs(pe / i.sweeps - 1)
                                                       for pe, i in zip(planned, infos)])), 4),
                      "bound_mean_abs": round(float(np.mean([abs(est_sweeps(d) / i.sweeps - 1)
                                                             for d, i in zip(dims, infos)])), 4)}},
    }


def bench_refined512(args):
    """The 512^3 configuration solved to a 1e-8 relative residual by FP32
    sweeps inside FP64 refinement (about a million sweeps, several minutes);
    the answer's FP64 residual is recomputed by a separate residual pass."""
    import numpy as np
    import torch
    import paper_2310_01882_amd as ms
    import synth

    n = args.n
    f_h = synth.gaussian_sources(n, n, n, 8, 1)
    u_h = synth.zeros(n, n, n)
    f = ms.field_from(f_h)
    u = ms.field_from(u_h)
    f32 = ms.field_from(f_h, torch.float32)
    tuned = ms.autotune_sweeps(ms.field_from(u_h, torch.float32),
                               ms.field_from(u_h, torch.float32), f32)
    del f32
    torch.cuda.empty_cache()
    log(f"[bench] FP32 sweep shape {tuned}")
    # Solved in calls of at most `chunk` inner sweeps, each resuming from the
    # previous answer (the tolerance is relative to the zero interior's
    # residual, so it does not move), with a progress line after each call.
    chunk = 100000
    opts = dict(precision=ms.MS_SOLVE_F32_REFINED, rel_tol=1e-8, temporal_block=args.tb,
                max_sweeps=chunk)
    work = ms.jacobi_workspace(u, ms.solve_opts(**opts))
    torch.cuda.synchronize()
    t = time.perf_counter()
    total, outer = 0, 0
    while True:
        info = ms.jacobi_solve(u, f, work=work, **opts)
        total += info.sweeps
        outer += info.outer_iters
        log(f"[bench]   {time.perf_counter() - t:.1f} s: {total} inner sweeps, "
            f"rel {info.rel_final:.3e}")
        if info.status == ms.MS_OK:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    info.sweeps, info.outer_iters = total, outer
    log(f"[bench] solved in {dt:.1f} s: {info.sweeps} inner sweeps, {info.outer_iters} outer, "
        f"rel {info.rel_final:.3e}")
    # the answer's FP64 residual, recomputed by the library's residual kernel
    zero = ms.field_from(u_h)
    rel = ms.residual_norm(u, f) / ms.residual_norm(zero, f)
    log(f"[bench] recomputed relative residual {rel:.3e}")
    return {
        "metric": "seconds to 1e-8 relative residual (512^3 Poisson, FP32 storage + FP64 refinement)",
        "value": round(dt, 2), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(dt * 1e3, 1), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"poisson_{n}cubed_fp32_refined_to_1e-8",
                   "rhs": "8 Gaussian sources (seed 1)", "boundary": "zero Dirichlet",
                   "temporal_block": args.tb, "calls_of_at_most_sweeps": chunk,
                   "parallelism": "single GPU"},
        "sweeps": info.sweeps, "outer": info.outer_iters, "rel_final": info.rel_final,
        "recomputed_rel_residual": rel, "glups": round(n ** 3 * info.sweeps / dt / 1e9, 2),
        "sweep_shape": tuned,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", choices=["jacobi", "f32", "advect", "solve", "batched",
                                       "refined512", "slab", "jit", "streamed"], default="jacobi")
    ap.add_argument("--tb", type=int, default=1, choices=[1, 2],
                    help="refined512 mode: sweeps per pass")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--sweeps", type=int, default=1000)
    ap.add_argument("--solve-n", type=int, default=128)
    ap.add_argument("--solve-reps", type=int, default=3)
    ap.add_argument("--cpu-sweeps", type=int, default=8)
    ap.add_argument("--cpu-sweeps-all", type=int, default=24,
                    help="sweeps of the all-core oracle baseline")
    ap.add_argument("--no-solve", action="store_true",
                    help="jacobi mode: skip the 128^3 time-to-tolerance comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batched mode: skip the one-by-one comparison")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on one GPU only; the multi-GPU halo-exchange path is a design "
              "(no collectives are implemented), so --gpus must be 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.mode == "jacobi":
        out = bench_jacobi(args, "f64")
    elif args.mode == "f32":
        out = bench_jacobi(args, "f32")
    elif args.mode == "advect":
        out = bench_advect(args)
    elif args.mode == "batched":
        out = bench_batched(args)
    elif args.mode == "refined512":
        out = bench_refined512(args)
    elif args.mode == "slab":
        out = bench_slab(args)
    elif args.mode == "jit":
        out = bench_jit(args)
    elif args.mode == "streamed":
        out = bench_streamed(args)
    else:
        out = bench_solve(args)
    out["device"] = torch.cuda.get_device_name(0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
