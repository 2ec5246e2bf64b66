"""Summaries of rocprofv3 output (CSV) for the association kernels.

    python -m paper_1805_01559_amd.profiling stats <dir> [--top N]
    python -m paper_1805_01559_amd.profiling traffic <fetch_dir> <write_dir> <kernel-substring> \
        --bytes <algorithmic bytes per launch> [--copy-bytes 536870912]

    python -m paper_1805_01559_amd.profiling valu <pmc_dir> <kernel-substring> --cells <cells per dispatch>
    python -m paper_1805_01559_amd.profiling timeline <trace_dir> <kernel-substring> [--index -3] [--after 12]

`stats` prints the kernel table of a `--kernel-trace --stats` run.
`timeline` interleaves the HIP API calls and the kernels of a
`--runtime-trace --kernel-trace` run around one dispatch of a kernel (the
`--index`-th, Python-style), from the end of the dispatch before it to the end
of the `--after`-th one after it, in microseconds from the first event.
`valu` turns a `--pmc` run of SQ_INSTS_* counters into lane-instructions per
cell of one kernel (median wave-instructions per working dispatch x 64 /
cells).
`traffic` turns two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs into HBM bytes
per launch of one kernel (`--first N`: its first N dispatches only). Both counters are in KiB per dispatch; each is
scaled by what it reads for the largest plain device copy in the same run
(a copy of known size: it reads and writes `--copy-bytes / 2` each), so that
the figure is in bytes the copy would have moved. The kernel's figure is the
median over its dispatches, which drops the launches of a chunk that stop at
once. Also prints a JSON line that bench.py can pick up.
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


SWEEP_SOURCES = ("kernels.h", "cost_sources.h", "device_common.h")
COOP_SOURCES = ("persist_kernels.h", "kernels.h", "cost_sources.h", "device_common.h")


def source_hash(files=SWEEP_SOURCES) -> str:
    """Hash of the sources that define a kernel: a traffic figure taken from
    counters is valid only for this hash."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def sweep_source_hash() -> str:
    return source_hash(SWEEP_SOURCES)


def _find(d: str, suffix: str) -> str:
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffix} under {d}")


def stats(d: str, top: int = 15) -> str:
    rows = list(csv.DictReader(open(_find(d, "kernel_stats.csv"))))
    out = ["| kernel | calls | avg us | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = r["Name"].replace("|", "/")
        if len(name) > 110:
            name = name[:107] + "..."
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out)


def _counter(d: str):
    return list(csv.DictReader(open(_find(d, "counter_collection.csv"))))


def traffic(fetch_dir: str, write_dir: str, kernel: str, alg_bytes: float, copy_bytes: float,
            sources=SWEEP_SOURCES, first: int = 0) -> dict:
    res = {}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter(d) if r["Counter_Name"] == name]
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        cal_kib = max(copies) if copies else None
        mine = sorted((int(r["Dispatch_Id"]), float(r["Counter_Value"])) for r in rows if kernel in r["Kernel_Name"])
        vals = [v for _, v in (mine[:first] if first > 0 else mine)]
        if not vals or not cal_kib:
            raise SystemExit(f"{name}: no dispatches of '{kernel}' or no copy calibration in {d}")
        factor = (copy_bytes / 2) / (cal_kib * 1024.0)
        res[name] = dict(median_kib=statistics.median(vals), dispatches=len(vals), copy_kib=cal_kib,
                         factor=factor, bytes=statistics.median(vals) * 1024.0 * factor)
    total = res["FETCH_SIZE"]["bytes"] + res["WRITE_SIZE"]["bytes"]
    return dict(kernel=kernel, algorithmic_bytes=alg_bytes, hbm_bytes=total, ratio=total / alg_bytes,
                fetch=res["FETCH_SIZE"], write=res["WRITE_SIZE"], sources=list(sources),
                source_hash=source_hash(sources))


def valu(d: str, kernel: str, cells: float) -> dict:
    """Median per dispatch of every SQ_INSTS_* counter of the kernels whose
    name contains `kernel`, as lane-instructions per cell, over the dispatches
    that did a sweep's work: those with at least half the largest
    SQ_INSTS_VALU (a captured chunk's launches after the stop exit at once)."""
    rows = [r for r in _counter(d) if kernel in r["Kernel_Name"] and r["Counter_Name"].startswith("SQ_INSTS_")]
    if not rows:
        raise SystemExit(f"no SQ_INSTS_ counters of '{kernel}' in {d}")
    total = {r["Dispatch_Id"]: float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == "SQ_INSTS_VALU"}
    if total:
        top = max(total.values())
        busy = {k for k, v in total.items() if v >= 0.5 * top}
        rows = [r for r in rows if r["Dispatch_Id"] in busy]
    out = {}
    for name in sorted({r["Counter_Name"] for r in rows}):
        vals = [float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == name]
        out[name] = dict(dispatches=len(vals), median_wave_insts=statistics.median(vals),
                         lane_insts_per_cell=statistics.median(vals) * 64.0 / cells)
    names = {r["Kernel_Name"] for r in rows}
    return dict(kernel=kernel, kernels_matched=sorted(names), cells=cells, counters=out)


def timeline(d: str, kernel: str, index: int = -3, after: int = 12) -> str:
    api = list(csv.DictReader(open(_find(d, "hip_api_trace.csv"))))
    ker = sorted(csv.DictReader(open(_find(d, "kernel_trace.csv"))), key=lambda r: int(r["Start_Timestamp"]))
    hits = [i for i, r in enumerate(ker) if kernel in r["Kernel_Name"]]
    if not hits:
        raise SystemExit(f"no dispatch of '{kernel}' in {d}")
    i = hits[index]
    lo = int(ker[i - 1]["End_Timestamp"]) if i > 0 else int(ker[i]["Start_Timestamp"])
    hi = int(ker[min(len(ker) - 1, i + after)]["End_Timestamp"])
    ev = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), "API", r["Function"]) for r in api
          if lo <= int(r["Start_Timestamp"]) <= hi]
    ev += [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), "GPU", r["Kernel_Name"].split("(")[0]) for r in ker
           if lo <= int(r["Start_Timestamp"]) <= hi]
    ev.sort()
    t0 = ev[0][0]
    out = ["| start (us) | duration (us) | | call or kernel |", "|---:|---:|---|---|"]
    for s, e, k, n in ev:
        out.append(f"| {(s - t0) / 1e3:.1f} | {(e - s) / 1e3:.1f} | {k} | `{n[:90]}` |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--top", type=int, default=15)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("kernel")
    b.add_argument("--bytes", type=float, required=True)
    b.add_argument("--copy-bytes", type=float, default=float(2 * (256 << 20)))
    b.add_argument("--coop", action="store_true", help="the kernel is the cooperative phase (persist_kernels.h)")
    b.add_argument("--first", type=int, default=0,
                   help="use only the kernel's first N dispatches (the bench's main leg runs first)")
    c = sub.add_parser("valu")
    c.add_argument("dir")
    c.add_argument("kernel")
    c.add_argument("--cells", type=float, required=True)
    t = sub.add_parser("timeline")
    t.add_argument("dir")
    t.add_argument("kernel")
    t.add_argument("--index", type=int, default=-3)
    t.add_argument("--after", type=int, default=12)
    args = ap.parse_args(argv)
    if args.cmd == "timeline":
        print(timeline(args.dir, args.kernel, args.index, args.after))
    elif args.cmd == "stats":
        print(stats(args.dir, args.top))
    elif args.cmd == "valu":
        v = valu(args.dir, args.kernel, args.cells)
        for k in v["kernels_matched"]:
            print(f"kernel: {k}")
        for name, x in v["counters"].items():
            print(f"{name}: {x['lane_insts_per_cell']:.2f} lane-instructions per cell "
                  f"(median {x['median_wave_insts']:.4g} wave-instructions over {x['dispatches']} dispatches)")
    else:
        t = traffic(args.fetch_dir, args.write_dir, args.kernel, args.bytes, args.copy_bytes,
                    COOP_SOURCES if args.coop else SWEEP_SOURCES, args.first)
        f, w = t["fetch"], t["write"]
        print(f"kernel: {t['kernel']}")
        print(f"FETCH_SIZE median {f['median_kib']:.1f} KiB over {f['dispatches']} dispatches; copy reads "
              f"{f['copy_kib']:.1f} KiB for 256 MiB -> factor {f['factor']:.4f}")
        print(f"WRITE_SIZE median {w['median_kib']:.1f} KiB; copy writes {w['copy_kib']:.1f} KiB -> factor "
              f"{w['factor']:.4f}")
        print(f"HBM bytes per launch {t['hbm_bytes']:.4g} vs algorithmic {t['algorithmic_bytes']:.4g} "
              f"(ratio {t['ratio']:.3f})")
        print(json.dumps(t))


if __name__ == "__main__":
    sys.exit(main())
