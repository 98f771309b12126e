"""Benchmark of the coupled D3Q19 LB / bead-dynamics step on one MI355X.

Default workload: the 128x64x64 translocation box (one wall with a 3x3 pore, one
N=100 bead chain, M=20 MD substeps per LB step, FP32 populations).  A step is one
coupled LB step (nearest-node interpolation, M bead substeps, spread of the
reaction force, stream-collide with bounce-back / free-slip), with the FP64
conserved-moment reduction and translocation read-out every 100 steps.

Prints one JSON line: MLUPS (fluid node updates per second / 1e6) of the whole
job, the lattice kernel's roofline figures (algorithmic bytes / measured kernel
time vs the 8 TB/s HBM peak), the FP64 oracle timed on the host cores, and the
16-bit storage variants of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E nominal
BYTES_PER_ELEM = {0: 8, 1: 4, 2: 2, 3: 2}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("lb_kernels.hip", "lbmd_device.hpp"):
        with open(os.path.join(ROOT, "paper_0710_1272_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, storage: str):
    """HBM bytes per lattice-kernel launch from the committed rocprofv3 counter runs,
    or None when they were taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(f"{workload}:{storage}")
    if not e or e.get("kernel_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def build_case(workload, storage):
    import numpy as np

    from paper_0710_1272_amd import lbmd as B
    from workloads import generate as G

    beads = [G.replica_beads(r, workload.md) for r in workload.replicas]
    allb = np.concatenate(beads) if beads else np.zeros((0, 3))
    init = {"bead_r": allb} if len(allb) else {}
    sim = B.Simulation(workload.replicas, workload.md, storage, init)
    return sim


def time_steps(sim, steps, diag_every=100):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(diag_every, steps - done)
        sim.step(k)
        done += k
        sim.conserved()     # FP64 mass/momentum reduction (synchronises)
        sim.transloc()      # N_T, centre of mass, completion step
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def lattice_kernel_time(sim, launches=200):
    """Average duration of the lattice kernel: HIP events recorded on the stream the
    kernel is launched on, around single LB-only steps (one launch each)."""
    import torch

    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(launches)]
    for _ in range(10):
        sim.step(1, coupled=False)
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        sim.step(1, coupled=False)
        b.record(stream)
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    return sum(ms) / len(ms) / 1e3, ms[len(ms) // 2] / 1e3


def cpu_baseline(workload, seconds=12.0):
    """The FP64 oracle on the same workload, timed on this host's cores."""
    import numpy as np

    from oracle import oracle as O
    from workloads import generate as G

    rep = workload.replicas[0]
    box = rep.box
    beads = G.replica_beads(rep, workload.md)
    f0 = O.equilibrium_populations(box, np.full(box.nodes, box.rho0), np.zeros((3, box.nodes)))
    sim = O.Sim(box, workload.md, rep.chain_len, f0, beads, seed=rep.seed)
    sim.step(1)
    n, t0 = 0, time.perf_counter()
    while True:
        sim.step(1)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= seconds and n >= 3:
            break
    return {"value": round(box.fluid_nodes() * n / dt / 1e6, 4), "unit": "MLUPS",
            "cores": O.threads(), "kind": "oracle",
            "sample": f"{n} coupled steps of the {workload.name} workload from its initial state "
                      f"(FP64 oracle, OpenMP over z-planes of the lattice loop)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c5"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-variants", action="store_true", help="skip the 16-bit storage variants")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from workloads import configs as WC

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    make = {"c2": WC.c2_translocation, "c3": WC.c3_translocation, "c5": WC.c5_large}[args.workload]
    w = make(WC.STORE_F32)
    fluid = w.fluid_nodes

    print(f"# building {w.name} (fp32)", file=sys.stderr, flush=True)
    sim = build_case(w, WC.STORE_F32)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    print(f"# timing {args.steps} coupled steps", file=sys.stderr, flush=True)
    dt = time_steps(sim, args.steps)
    mlups = fluid * args.steps / dt / 1e6
    k_avg, k_med = lattice_kernel_time(sim)
    bytes_launch = fluid * 2 * 19 * BYTES_PER_ELEM[WC.STORE_F32]
    achieved = bytes_launch / k_avg / 1e9
    traffic = measured_traffic(w.name, "f32")
    sim.close()

    variants = {}
    if not args.no_variants:
        for st in (WC.STORE_F16, WC.STORE_BF16):
            name = WC.STORE_NAMES[st]
            print(f"# variant {name}", file=sys.stderr, flush=True)
            s2 = build_case(w, st)
            s2.step(args.warmup)
            d2 = time_steps(s2, args.steps)
            ka, _ = lattice_kernel_time(s2)
            b2 = fluid * 2 * 19 * BYTES_PER_ELEM[st]
            variants[name] = {"mlups": round(fluid * args.steps / d2 / 1e6, 1),
                              "ms_per_step": round(d2 / args.steps * 1e3, 5),
                              "speedup_vs_f32": round(dt / d2, 3),
                              "lattice_kernel_us": round(ka * 1e6, 2),
                              "lattice_kernel_gbs": round(b2 / ka / 1e9, 1)}
            s2.close()

    out = {
        "metric": "coupled D3Q19 step MLUPS & % HBM peak; fp32 vs fp16-store; replicas/s",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "box": [w.replicas[0].box.nx, w.replicas[0].box.ny,
                                               w.replicas[0].box.nz],
                   "fluid_nodes": fluid, "beads": w.replicas[0].n_beads, "md_substeps": w.md.M,
                   "storage": "f32", "diag_every": 100},
        "roofline": {"bound": "hbm", "kernel": "k_stream_collide",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "alg_bytes_per_launch": bytes_launch,
                     "kernel_us_avg": round(k_avg * 1e6, 2), "kernel_us_median": round(k_med * 1e6, 2)},
        "variants": variants,
        "paper_context": "0.262 MLUPS coupled (N=100, 80x40x40 box) on a serial 2 GHz Opteron",
    }
    if not args.no_cpu:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
