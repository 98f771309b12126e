"""Profiling runs of the lattice kernel and the coupled step (rocprofv3).

  run:        lattice-kernel launches (LB-only steps) on a named workload, then copies of
              a known number of bytes by a plain copy kernel, for one counter pass:
                rocprofv3 --pmc FETCH_SIZE --output-format csv -d D -o fetch -- \
                    python3 -m paper_0710_1272_amd.profile_lattice run --workload c3 --storage f32
                rocprofv3 --pmc WRITE_SIZE ... (same program)
  summarize:  reads the two counter CSVs, scales each counter by what it reads for the
              copy (bytes moved / counter), and records bytes per lattice launch in
              profiles/traffic.json with the hash of the kernel source it was taken on.
  trace:      coupled steps of a named workload in the benchmark's configuration (autotuned
              launch shapes, graph launches, the workload's chains), for a kernel trace:
                rocprofv3 --kernel-trace --stats --output-format csv -d D -o c3 -- \
                    python3 -m paper_0710_1272_amd.profile_lattice trace --workload c3 --storage f32
  trace-summary: per-kernel durations over the last --window dispatches of each kernel in a
              kernel-trace CSV (the timed steps, after the autotuner's trials).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_BYTES = 1 << 30  # 1 GiB read + 1 GiB written per copy
LAUNCHES = 20
COPIES = 4


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("lb_kernels.hip", "lbmd_device.hpp"):
        with open(os.path.join(ROOT, "paper_0710_1272_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(name: str, storage: str):
    from workloads import configs as WC

    st = {"f32": WC.STORE_F32, "f16dev": WC.STORE_F16, "bf16dev": WC.STORE_BF16}[storage]
    if name == "c4":
        return WC.c4_batched(256, st), st
    w = {"c2": WC.c2_translocation, "c3": WC.c3_translocation, "c5": WC.c5_large}[name](st)
    return w, st


def run(args):
    import torch

    from paper_0710_1272_amd import lbmd as B
    from workloads import configs as WC

    w, st = workload(args.workload, args.storage)
    reps = [WC.Replica(r.box, [], r.seed) for r in w.replicas]
    mapping = {"flat": B.LB_MAP_FLAT, "rows": B.LB_MAP_ROWS, "shifted": B.LB_MAP_SHIFTED,
               "flat2": B.LB_MAP_FLAT2}[args.mapping]
    sim = B.Simulation(reps, w.md, st, {}, mapping=mapping, xcd_order=args.xcd)
    for _ in range(LAUNCHES):
        sim.step(1, coupled=False)
    torch.cuda.synchronize()
    sim.close()
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(COPIES):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"profile_lattice: {w.name} {args.storage}: {LAUNCHES} lattice launches, "
          f"{COPIES} copies of {COPY_BYTES} bytes", flush=True)


def trace(args):
    """Coupled steps in the benchmark's configuration, after a warm-up, in blocks of at most
    100 graph-launched steps."""
    import numpy as np
    import torch

    from paper_0710_1272_amd import lbmd as B
    from workloads import generate as G

    import dataclasses

    w, st = workload(args.workload, args.storage)
    md = dataclasses.replace(w.md, stencil=1) if args.trilinear else w.md
    beads = np.concatenate([G.replica_beads(r, md) for r in w.replicas])
    sim = B.Simulation(w.replicas, md, st, {"bead_r": beads}, flags=B.LB_CFG_AUTOTUNE)
    sim.step(args.warmup)
    done = 0
    while done < args.steps:
        k = min(100, args.steps - done)
        sim.prepare(k)
        sim.step(k)
        sim.conserved()
        done += k
    torch.cuda.synchronize()
    print(f"profile_lattice trace: {w.name} {args.storage}: {args.warmup} + {args.steps} coupled steps, "
          f"launch shape {sim.launch_shape()}", flush=True)
    sim.close()


def trace_summary(args):
    """Mean and median duration of each kernel's last `window` dispatches in a kernel-trace
    CSV, and the spacing of the last dispatches of the most frequent kernel."""
    rows = {}
    with open(args.trace_csv) as fh:
        for r in csv.DictReader(fh):
            rows.setdefault(r["Kernel_Name"], []).append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    out = []
    for name, ts in rows.items():
        ts.sort()
        last = ts[-args.window:]
        d = sorted(e - b for b, e in last)
        out.append((sum(d) / len(d), name, len(ts), len(last), d[len(d) // 2]))
    out.sort(reverse=True)
    print("| kernel | dispatches | last | mean ns (last) | median ns (last) |")
    print("|---|---|---|---|---|")
    for mean, name, n, k, med in out:
        print(f"| `{name[:90]}` | {n} | {k} | {mean:.0f} | {med} |")


def _per_dispatch(path, counter):
    lat, cop = [], []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"]) * 1024.0  # the counter reads KiB
            name = r["Kernel_Name"]
            if "k_stream_collide" in name:
                lat.append(v)
            elif "copy" in name.lower() or "elementwise" in name.lower():
                cop.append(v)
    return lat, cop


def summarize(args):
    w, st = workload(args.workload, args.storage)
    lat_f, cop_f = _per_dispatch(args.fetch_csv, "FETCH_SIZE")
    lat_w, cop_w = _per_dispatch(args.write_csv, "WRITE_SIZE")
    # the copy kernels with the largest counts are the 1 GiB copies
    cop_f = sorted(cop_f)[-COPIES:]
    cop_w = sorted(cop_w)[-COPIES:]
    sf = COPY_BYTES / (sum(cop_f) / len(cop_f))
    sw = COPY_BYTES / (sum(cop_w) / len(cop_w))
    fetch = sf * sum(lat_f) / len(lat_f)
    write = sw * sum(lat_w) / len(lat_w)
    alg = w.fluid_nodes * 19 * {0: 8, 1: 4, 2: 2, 3: 2}[st]
    entry = {"bytes_per_launch": round(fetch + write), "fetch_bytes": round(fetch),
             "write_bytes": round(write), "alg_bytes": 2 * alg, "fetch_over_alg": round(fetch / alg, 4),
             "write_over_alg": round(write / alg, 4), "fetch_scale": round(sf, 4),
             "write_scale": round(sw, 4), "launches": len(lat_f), "mapping": args.mapping, "xcd_order": args.xcd,
             "kernel_hash": kernel_source_hash()}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        data = {}
    data[f"{w.name}:{args.storage}"] = entry
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(json.dumps({f"{w.name}:{args.storage}": entry}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["run", "summarize", "trace", "trace-summary"])
    ap.add_argument("--workload", default="c3", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f16dev", "bf16dev"])
    ap.add_argument("--mapping", default="flat", choices=["flat", "rows", "shifted", "flat2"],
                    help="thread-to-node mapping of the lattice launches in run mode")
    ap.add_argument("--xcd", type=int, default=0,
                    help="XCD tile order of the lattice launches in run mode (LB_XCD_*, or a chunk "
                         "size > 0; the default lets the library choose)")
    ap.add_argument("--steps", type=int, default=100, help="timed coupled steps (trace)")
    ap.add_argument("--warmup", type=int, default=20, help="coupled steps before them (trace)")
    ap.add_argument("--trilinear", action="store_true", help="the trilinear stencil (trace)")
    ap.add_argument("--fetch-csv")
    ap.add_argument("--write-csv")
    ap.add_argument("--trace-csv")
    ap.add_argument("--window", type=int, default=100)
    args = ap.parse_args()
    {"run": run, "summarize": summarize, "trace": trace, "trace-summary": trace_summary}[args.mode](args)


if __name__ == "__main__":
    main()
