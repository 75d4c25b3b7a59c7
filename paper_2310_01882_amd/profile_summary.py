"""Turns rocprofv3 CSV output into the short summaries kept under profiles/.

    python -m paper_2310_01882_amd.profile_summary stats  OUT.md  KERNEL_STATS_CSV  "COMMAND"
    python -m paper_2310_01882_amd.profile_summary traffic KEY KERNEL_SUBSTR \
        FETCH_CSV WRITE_CSV COPY_FETCH_CSV COPY_WRITE_CSV COPY_MIB OUT.md "COMMANDS"

    python -m paper_2310_01882_amd.profile_summary counters OUT.md "TITLE" "COMMANDS" CSV...

`stats` writes the per-kernel table (calls, average and total duration) of a
--kernel-trace --stats run. `traffic` reads FETCH_SIZE and WRITE_SIZE (KiB per
dispatch) for the kernels whose name contains KERNEL_SUBSTR, scales each by
the factor that makes the same counter read the known size of a plain
device copy of COPY_MIB MiB, and records bytes per launch in
profiles/traffic.json under KEY, together with a hash of the kernel sources
the figure was taken on (the benchmark reports null once they change).
`counters` tabulates every counter of one or more --pmc runs per kernel
(average per dispatch) and, where SQ_VALU_MFMA_BUSY_CYCLES and
SQ_BUSY_CYCLES are both present, the share of the MFMA pipes kept busy
(MFMA busy cycles over 1024 SIMDs x SQ_BUSY_CYCLES / 32 shader engines).
"""

from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PROFILES = os.path.join(ROOT, "profiles")

SOURCES = {
    "jacobi7": ["jacobi.hip", "ms_internal.hpp", "common.hip", "march.hpp"],
    "advect": ["advect.hip"],
    "batched": ["batched.hip", "ms_internal.hpp", "march.hpp"],
    "conv": ["cnn.hip"],
    "jit": ["jit.hip", "programs.py"],
}


def source_hash(key: str) -> str:
    names = SOURCES[next((k for k in SOURCES if key.startswith(k)), "jacobi7")]
    h = hashlib.sha256()
    for n in names:
        path = os.path.join(HERE, "csrc", n)
        if not os.path.exists(path):
            path = os.path.join(HERE, n)
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name: str, width: int = 90) -> str:
    return name if len(name) <= width else name[: width - 3] + "..."


def stats(out_md: str, stats_csv: str, command: str):
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# Kernel time summary: {os.path.basename(out_md)[:-3]}", "",
             f"Command: `{command}`", "",
             "| kernel | calls | avg (us) | total (ms) | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        calls = int(r["Calls"])
        tot_ns = float(r["TotalDurationNs"])
        avg_ns = float(r["AverageNs"])
        pct = float(r.get("Percentage", 0.0))
        lines.append(f"| `{_short(r['Name'])}` | {calls} | {avg_ns / 1e3:.1f} | "
                     f"{tot_ns / 1e6:.2f} | {pct:.1f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _per_kernel(path: str, counter: str):
    agg = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def _mean_for(agg, substr):
    vals = [v for k, vs in agg.items() if substr in k for v in vs]
    if not vals:
        raise SystemExit(f"no dispatch of a kernel matching {substr!r}")
    return sum(vals) / len(vals), len(vals)


def traffic(key, substr, fetch_csv, write_csv, cfetch_csv, cwrite_csv, copy_mib, out_md,
            commands):
    copy_kib = float(copy_mib) * 1024.0
    cf, _ = _mean_for(_per_kernel(cfetch_csv, "FETCH_SIZE"), "copy")
    cw, _ = _mean_for(_per_kernel(cwrite_csv, "WRITE_SIZE"), "copy")
    kf, nf = _mean_for(_per_kernel(fetch_csv, "FETCH_SIZE"), substr)
    kw, nw = _mean_for(_per_kernel(write_csv, "WRITE_SIZE"), substr)
    fscale, wscale = copy_kib / cf, copy_kib / cw
    fetch_b = kf * fscale * 1024.0
    write_b = kw * wscale * 1024.0
    rec = {
        "bytes_per_launch": round(fetch_b + write_b),
        "fetch_bytes_per_launch": round(fetch_b),
        "write_bytes_per_launch": round(write_b),
        "fetch_kib_raw": kf, "write_kib_raw": kw,
        "fetch_scale": fscale, "write_scale": wscale,
        "dispatches": [nf, nw],
        "source_hash": source_hash(key),
    }
    path = os.path.join(PROFILES, "traffic.json")
    db = json.load(open(path)) if os.path.exists(path) else {}
    db[key] = rec
    json.dump(db, open(path, "w"), indent=1, sort_keys=True)
    lines = [f"# HBM traffic: {key}", "",
             "Commands (FETCH_SIZE run, WRITE_SIZE run, and the copy calibration runs):", ""]
    lines += [f"    {c}" for c in commands.split(";;")]
    lines += ["",
              f"Copy calibration: a {copy_mib} MiB device copy reads FETCH_SIZE {cf:.0f} KiB "
              f"and WRITE_SIZE {cw:.0f} KiB per dispatch; scale factors fetch {fscale:.4f}, "
              f"write {wscale:.4f}.", "",
              f"Kernel `{substr}`: FETCH_SIZE {kf:.0f} KiB ({nf} dispatches), WRITE_SIZE "
              f"{kw:.0f} KiB ({nw} dispatches) per dispatch.", "",
              f"Scaled HBM bytes per launch: fetch {fetch_b / 1e9:.4f} GB, write "
              f"{write_b / 1e9:.4f} GB, total {(fetch_b + write_b) / 1e9:.4f} GB.", "",
              f"Kernel source hash: {rec['source_hash']}"]
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counters(out_md: str, title: str, commands: str, *csvs: str):
    table = defaultdict(dict)
    names = []
    for path in csvs:
        agg = defaultdict(lambda: defaultdict(list))
        for r in csv.DictReader(open(path)):
            agg[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
        for kern, per in agg.items():
            for ctr, vals in per.items():
                table[kern][ctr] = sum(vals) / len(vals)
                if ctr not in names:
                    names.append(ctr)
    mfma = "SQ_VALU_MFMA_BUSY_CYCLES" in names and "SQ_BUSY_CYCLES" in names
    head = names + (["MFMA busy share"] if mfma else [])
    lines = [f"# {title}", "", "Commands (one run per line):", ""]
    lines += [f"    {c}" for c in commands.split(";;")]
    lines += ["", "Average per dispatch, summed over the device as rocprofv3 reports them.", "",
              "| kernel | " + " | ".join(head) + " |", "|---|" + "---:|" * len(head)]
    for kern in sorted(table):
        row = table[kern]
        cells = [f"{row[c]:.3g}" if c in row else "" for c in names]
        if mfma:
            busy = row.get("SQ_BUSY_CYCLES", 0.0)
            share = row.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (1024 * busy / 32) if busy else 0
            cells.append(f"{100 * share:.0f}%")
        lines.append(f"| `{_short(kern, 60)}` | " + " | ".join(cells) + " |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(*sys.argv[2:5])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:11])
    elif sys.argv[1] == "counters":
        counters(*sys.argv[2:])
    else:
        raise SystemExit(__doc__)
