"""Benchmark of the coupled D3Q19 LB / bead-dynamics step on one MI355X.

Headline workload: the 512^3 box with two pore walls, an N = 800 chain and 64 crowder
chains of 25 beads, FP32 populations (20.4 GB of populations read and written per step,
far beyond the 256 MB last-level cache).  A step is one coupled LB step (nearest-node
interpolation, M = 20 bead substeps, spread of the reaction force, stream-collide with
bounce-back and free-slip faces); the FP64 conserved-moment reduction and the
translocation read-out run after every block of at most 100 steps.  Every HIP graph the
timed steps launch is captured before the timed region.

Prints one JSON line: MLUPS (fluid node updates per second / 1e6) of the whole job; the
lattice kernel's roofline (algorithmic bytes / measured kernel time against the 8 TB/s
HBM peak) and the same for the whole coupled step; the FP64 oracle timed on the host
cores; and, under "workloads", the 128x64x64 and 256x128x128 boxes in FP32, FP16 and BF16
storage and the 256-replica batch, each speedup next to its measured error against FP64
storage of the same inputs.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E nominal
BYTES_PER_ELEM = {0: 8, 1: 4, 2: 2, 3: 2}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
DIAG_EVERY = 100


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    """The host CPU as /proc/cpuinfo names it, with its family / model / stepping numbers
    (a virtual machine may report only the brand) and the logical CPUs visible."""
    info = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if ":" in line:
                    k, v = line.split(":", 1)
                    info.setdefault(k.strip(), v.strip())
    except OSError:
        pass
    name = info.get("model name") or platform.processor() or "unknown"
    ids = [f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info]
    return f"{name} ({', '.join(ids + [f'{os.cpu_count()} logical CPUs visible'])})"


def measured_traffic(workload: str, storage: str):
    """HBM bytes per lattice-kernel launch from the committed rocprofv3 counter runs,
    or None when they were taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    from paper_0710_1272_amd.profile_lattice import kernel_source_hash

    e = t.get(f"{workload}:{storage}")
    if not e or e.get("kernel_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def build_case(workload, storage, beads=True, flags=None, init=None):
    import numpy as np

    from paper_0710_1272_amd import lbmd as B
    from workloads import generate as G

    init = dict(init or {})
    if beads:
        b = [G.replica_beads(r, workload.md) for r in workload.replicas]
        allb = np.concatenate(b) if b else np.zeros((0, 3))
        if len(allb):
            init["bead_r"] = allb
    return B.Simulation(workload.replicas, workload.md, storage, init,
                        flags=B.LB_CFG_AUTOTUNE if flags is None else flags)


def chunks(steps):
    out, done = [], 0
    while done < steps:
        k = min(DIAG_EVERY, steps - done)
        out.append(k)
        done += k
    return out


def time_steps(sim, steps):
    """Seconds for `steps` coupled steps, with the FP64 conserved sums and the translocation
    read-out after every block of at most DIAG_EVERY steps.  The graphs of every block length
    are captured first, outside the timed region."""
    import torch

    for k in sorted(set(chunks(steps))):
        sim.prepare(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in chunks(steps):
        sim.step(k)
        sim.conserved()     # FP64 mass/momentum reduction (synchronises)
        sim.transloc()      # N_T, centre of mass, completion step
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def event_time(fn, n, warm=5):
    """Average duration of fn() (one kernel launch on the current stream) from HIP
    events recorded on that stream around each call."""
    import torch

    stream = torch.cuda.current_stream()
    for _ in range(warm):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    return sum(ms) / len(ms) / 1e3, ms[len(ms) // 2] / 1e3


def lattice_roofline(sim, fluid, storage, n=96):
    """Average lattice-kernel duration: HIP events on the launch stream (the caller's, where
    the library launches its graphs) around n back-to-back LB-only steps (one lattice launch
    each, graph-launched), best of 3, and, for reference, around single launches."""
    import torch

    stream = torch.cuda.current_stream()
    sim.prepare(n, coupled=False)
    sim.prepare(1, coupled=False)
    sim.step(16, coupled=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = 1e30
    for _ in range(3):
        torch.cuda.synchronize()
        e0.record(stream)
        sim.step(n, coupled=False)
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3 / n)
    single, _ = event_time(lambda: sim.step(1, coupled=False), 20)
    # the same-pattern reference (lb_pattern_copy): the sweep's loads and stores over every node
    # (solid ones included) with no arithmetic, in the same launch shape, alternating between
    # the two buffers as the sweeps do; it leaves the populations without meaning, so it comes
    # last and the caller only reads the launch shape and closes the context afterwards
    pat = 1e30
    for _ in range(3):
        torch.cuda.synchronize()
        e0.record(stream)
        for _k in range(n):
            sim.pattern_copy(alternate=True)
        e1.record(stream)
        torch.cuda.synchronize()
        pat = min(pat, e0.elapsed_time(e1) / 1e3 / n)
    alg = fluid * 2 * 19 * BYTES_PER_ELEM[storage]
    pat_bytes = sum(r.box.nodes for r in sim.replicas) * 2 * 19 * BYTES_PER_ELEM[storage]
    pat_gbs = pat_bytes / pat / 1e9
    return {"kernel_us_avg": round(best * 1e6, 2), "kernel_us_single_launch": round(single * 1e6, 2),
            "alg_bytes_per_launch": alg, "achieved_gbs": round(alg / best / 1e9, 1),
            "frac": round(alg / best / 1e9 / HBM_PEAK_GBS, 4),
            "same_pattern_gbs": round(pat_gbs, 1), "frac_of_same_pattern": round(alg / best / 1e9 / pat_gbs, 4)}


def accuracy(workload, storage, steps=10, picks=None, batched=False):
    """Error of `storage` against FP64 storage of the same inputs after `steps` coupled steps
    from a random small flow (|u| <= 0.01, rho = 1 +- 0.01) with the workload's chains: the
    largest velocity difference over fluid nodes divided by max|u| of the FP64 run, and the
    largest bead-position difference.  The FP64 path is the one the parity tests hold to the
    FP64 oracle at 1e-11.  picks: replicas to compare (all by default); batched: the whole
    batch runs in `storage` at once, each picked replica alone in FP64."""
    import numpy as np

    from workloads import configs as WC
    from workloads import generate as G

    reps = workload.replicas
    picks = list(range(len(reps))) if picks is None else list(picks)
    flows = {k: G.random_small_flow(reps[k].box, 700 + k, du=0.01) for k in range(len(reps))
             if batched or k in picks}
    beads = {k: G.replica_beads(reps[k], workload.md) for k in flows}

    def run(idx, st):
        init = dict(rho=np.concatenate([flows[k][0] for k in idx]),
                    u=np.concatenate([flows[k][1].ravel() for k in idx]),
                    bead_r=np.concatenate([beads[k] for k in idx]))
        w = WC.Workload(workload.name, [reps[k] for k in idx], workload.md, st, steps)
        sim = build_case(w, st, beads=False, flags=0, init=init)
        sim.step(steps)
        out = {k: (sim.fields(j), sim.beads(j)[0]) for j, k in enumerate(idx) if k in picks}
        err, _ = sim.status()
        sim.close()
        return out, err

    got, err = {}, 0
    if batched:
        got, err = run(list(range(len(reps))), storage)
    else:
        for k in picks:
            g, e = run([k], storage)
            got.update(g)
            err |= e
    ve, dr = 0.0, 0.0
    for k in picks:
        ref, e = run([k], WC.STORE_F64)
        err |= e
        ((_, u_s), r_s), ((rho_d, u_d), r_d) = got[k], ref[k]
        fluid = rho_d > 0  # solid nodes read 0
        ve = max(ve, float(np.max(np.abs(u_s[:, fluid] - u_d[:, fluid])) / np.max(np.abs(u_d[:, fluid]))))
        dr = max(dr, float(np.max(np.abs(r_s - r_d))) if len(r_d) else 0.0)
    return {"vel_err_over_max_u": float(f"{ve:.3g}"), "bead_drift_max": float(f"{dr:.3g}"),
            "steps": steps, "replicas_compared": len(picks), "error_word": int(err)}


def large_box_16bit(storage, f32_step_s, steps=50):
    """The 512^3 two-wall workload with 16-bit deviation storage: coupled MLUPS, speedup over
    the FP32 headline step, the lattice roofline, and the error against FP64 storage of the
    same inputs (a random small flow and the workload's chains) after 10 coupled steps, over
    sampled z-slabs (bulk, both walls with their pores, the faces): the box is too large to
    read back whole at FP64."""
    import numpy as np
    import torch

    from workloads import configs as WC
    from workloads import generate as G

    w = WC.c5_large(storage)
    log(f"workload {w.name} {WC.STORE_NAMES[storage]}")
    sim = build_case(w, storage)
    sim.step(10)
    dt = time_steps(sim, steps)
    e = {"mlups": round(w.fluid_nodes * steps / dt / 1e6, 1), "ms_per_step": round(dt / steps * 1e3, 4),
         "speedup_vs_f32": round(f32_step_s / (dt / steps), 3)}
    e["lattice"] = lattice_roofline(sim, w.fluid_nodes, storage, n=16)
    e["launch"] = sim.launch_shape()
    sim.close()
    torch.cuda.empty_cache()
    # accuracy against FP64 storage on sampled slabs of 4 z-planes
    rep = w.replicas[0]
    box = rep.box
    rho, u = G.random_small_flow(box, 700, du=0.01)
    beads = G.replica_beads(rep, w.md)
    nxy = box.nx * box.ny
    slabs = [0, box.nz // 4, box.nz // 2 - 2, box.nz - 4]
    res = {}
    for st in (storage, WC.STORE_F64):
        s2 = build_case(w, st, beads=False, flags=0, init={"rho": rho, "u": u.ravel(), "bead_r": beads})
        s2.step(10)
        res[st] = ([s2.fields_range(z * nxy, 4 * nxy) for z in slabs], s2.beads()[0], s2.status()[0])
        s2.close()
        torch.cuda.empty_cache()
    ve = 0.0
    for (rho_s, u_s), (rho_d, u_d) in zip(res[storage][0], res[WC.STORE_F64][0]):
        fl = rho_d > 0
        ve = max(ve, float(np.max(np.abs(u_s[:, fl] - u_d[:, fl])) / np.max(np.abs(u_d[:, fl]))))
    e["accuracy_vs_f64"] = {"vel_err_over_max_u": float(f"{ve:.3g}"),
                            "bead_drift_max": float(f"{np.max(np.abs(res[storage][1] - res[WC.STORE_F64][1])):.3g}"),
                            "steps": 10, "sample": f"z-slabs of 4 planes at z = {slabs} (all x, y)",
                            "error_word": int(res[storage][2] | res[WC.STORE_F64][2])}
    return e


def translocation_times(storage, n=512, cap=4000, check=250):
    """Completion steps of n independent translocation events (48^3 pore boxes, N = 32) run
    as one batch: mean and standard error of the completed ones."""
    import numpy as np

    from workloads import configs as WC

    w = WC.ensemble48_n32(n, WC.ENSEMBLE_SEED_GPU, storage)
    sim = build_case(w, storage, flags=0)
    steps = 0
    t = np.full(n, -1)
    while steps < cap:
        sim.step(check)
        steps += check
        t = np.array([sim.transloc(r)["t_done"] for r in range(n)])
        if np.all(t > 0):
            break
    sim.close()
    done = t[t > 0]
    return {"events": n, "completed": int(len(done)), "mean_steps": round(float(done.mean()), 2),
            "se_steps": round(float(done.std(ddof=1) / np.sqrt(len(done))), 2)}


def cpu_baseline(workload):
    """The FP64 oracle on the headline workload, timed on this host's cores, on a bounded
    sample: LB-only steps of a 512x512x64 slab of the box (the lattice loop is linear in the
    volume and runs OpenMP over z-planes) and bead steps (M substeps) of the full bead
    population; the estimated time of one whole coupled step is 8 slab steps plus one bead
    step."""
    import numpy as np

    from oracle import oracle as O
    from workloads import configs as WC
    from workloads import generate as G

    rep = workload.replicas[0]
    box = rep.box
    slab = WC.Box(box.nx, box.ny, box.nz // 8, box.bc, box.walls, box.tau, box.rho0)
    f0 = O.equilibrium_populations(slab, np.full(slab.nodes, slab.rho0), np.zeros((3, slab.nodes)))
    lb = O.Sim(slab, workload.md, np.zeros(0, dtype=np.int32), f0, np.zeros((0, 3)), seed=rep.seed)
    lb.step(1, coupled=False)
    t_lb = []
    for _ in range(3):
        t0 = time.perf_counter()
        lb.step(1, coupled=False)
        t_lb.append(time.perf_counter() - t0)
    del lb, f0
    beads = G.replica_beads(rep, workload.md)
    r, v, u = beads.copy(), np.zeros_like(beads), np.zeros_like(beads)
    t_md = []
    for k in range(3):
        t0 = time.perf_counter()
        O.md_substeps(box, workload.md, rep.chain_len, r, v, u, k, rep.seed)
        t_md.append(time.perf_counter() - t0)
    t_step = 8 * float(np.median(t_lb)) + float(np.median(t_md))
    return {"value": round(box.fluid_nodes() / t_step / 1e6, 4), "unit": "MLUPS",
            "cores": O.threads(), "cpu": cpu_model(), "kind": "oracle",
            "sample": f"FP64 oracle: 3 LB-only steps of a {slab.nx}x{slab.ny}x{slab.nz} slab of the "
                      f"{workload.name} box (median {np.median(t_lb):.3f} s, OpenMP over z-planes) and 3 bead "
                      f"steps of its {len(beads)} beads (median {np.median(t_md):.3f} s, one thread); "
                      f"coupled step estimated as 8 slab steps + 1 bead step = {t_step:.2f} s"}


def storage_set(workload, steps, out, key, with_roofline=True, acc_kw=None):
    """FP32, FP16 and BF16 storage of one workload: coupled MLUPS, speedup over FP32, the
    lattice kernel's roofline and the error against FP64 storage."""
    import torch

    from workloads import configs as WC

    base = None
    for st in (WC.STORE_F32, WC.STORE_F16, WC.STORE_BF16):
        name = WC.STORE_NAMES[st]
        log(f"workload {workload.name} {name}")
        sim = build_case(workload, st)
        sim.step(20)
        dt = time_steps(sim, steps)
        e = {"mlups": round(workload.fluid_nodes * steps / dt / 1e6, 1), "ms_per_step": round(dt / steps * 1e3, 4)}
        if with_roofline:
            e["lattice"] = lattice_roofline(sim, workload.fluid_nodes, st)
        e["launch"] = sim.launch_shape()
        sim.close()
        if base is None:
            base = dt
        else:
            e["speedup_vs_f32"] = round(base / dt, 3)
        e["accuracy_vs_f64"] = accuracy(workload, st, **(acc_kw or {}))
        out[f"{key}:{name}"] = e
        torch.cuda.empty_cache()


def extra_workloads(f32_step_s):
    """The other configurations: 128x64x64 and 256x128x128 in FP32/FP16/BF16, the 256-replica
    batch against the same replicas one at a time in FP32, the paper's rigid chain, the
    thermal fluid, the no-solvent comparison and translocation times per storage format."""
    import dataclasses

    import numpy as np
    import torch

    from workloads import configs as WC

    out = {}
    out["large512_two_walls:f16dev"] = large_box_16bit(WC.STORE_F16, f32_step_s)
    storage_set(WC.c2_translocation(WC.STORE_F32), 1000, out, "pore128x64x64_n100")
    storage_set(WC.c3_translocation(WC.STORE_F32), 300, out, "pore256x128x128_n400")

    w = WC.c4_batched(256, WC.STORE_F16)
    log(f"workload {w.name} (building 256 chains)")
    sim = build_case(w, WC.STORE_F16)
    sim.step(5)
    n = 60
    dt = time_steps(sim, n)
    rl = lattice_roofline(sim, w.fluid_nodes, WC.STORE_F16, n=16)
    batched = len(w.replicas) * n / dt
    e = {"replica_steps_per_s": round(batched, 1), "mlups": round(w.fluid_nodes * n / dt / 1e6, 1),
         "ms_per_step": round(dt / n * 1e3, 4), "lattice": rl, "launch": sim.launch_shape()}
    sim.close()
    torch.cuda.empty_cache()
    # the plain form: replicas one at a time in FP32; the mean step time of 8 replicas at
    # evenly spaced size ranks estimates that of the whole batch
    order = np.argsort([r.box.nodes * 1000 + r.n_beads for r in w.replicas])
    picks = [int(order[round(k * (len(order) - 1) / 7)]) for k in range(8)]
    times = []
    for k in picks:
        one = dataclasses.replace(w, replicas=[w.replicas[k]])
        s1 = build_case(one, WC.STORE_F32)
        s1.step(20)
        times.append(time_steps(s1, 200) / 200)
        s1.close()
    seq = 1.0 / float(np.mean(times))
    e["single_f32_replica_steps_per_s"] = round(seq, 1)
    e["speedup_vs_single_f32"] = round(batched / seq, 2)
    e["single_f32_sample"] = "8 replicas at evenly spaced size ranks, each alone in FP32 storage (autotuned)"
    log("accuracy of the batch (3 sampled replicas)")
    e["accuracy_vs_f64"] = accuracy(w, WC.STORE_F16, picks=[int(order[0]), int(order[len(order) // 2]),
                                                            int(order[-1])], batched=True)
    out[f"{w.name}:f16dev"] = e
    torch.cuda.empty_cache()

    # the paper's own polymer model (rigid bonds by SHAKE/RATTLE, M = 5) on 128x64x64 / N=100
    w = WC.c2_paper_polymer(WC.STORE_F32)
    log(f"workload {w.name} f32")
    sim = build_case(w, WC.STORE_F32)
    sim.step(50)
    dt = time_steps(sim, 1000)
    md_avg, _ = event_time(sim.md_step, 30)
    out[f"{w.name}:f32"] = {"mlups": round(w.fluid_nodes * 1000 / dt / 1e6, 1), "ms_per_step": round(dt, 5),
                            "md_substeps": w.md.M, "bead_kernel_us": round(md_avg * 1e6, 2),
                            "launch": sim.launch_shape()}
    sim.close()
    # the fluctuating lattice (thermal source F_p at kT = 1e-4) on the same 128x64x64 / N=100 set-up
    w = WC.c2_translocation(WC.STORE_F32)
    rep = w.replicas[0]
    w = dataclasses.replace(w, name=w.name + "_thermal",
                            replicas=[dataclasses.replace(rep, box=dataclasses.replace(rep.box, fluid_kT=1e-4))])
    log(f"workload {w.name} f32")
    sim = build_case(w, WC.STORE_F32)
    sim.step(50)
    dt = time_steps(sim, 1000)
    out[f"{w.name}:f32"] = {"mlups": round(w.fluid_nodes * 1000 / dt / 1e6, 1), "ms_per_step": round(dt, 5),
                            "fluid_kT": 1e-4, "lattice_only_step": lattice_roofline(sim, w.fluid_nodes,
                                                                                     WC.STORE_F32, n=96),
                            "launch": sim.launch_shape()}
    sim.close()
    torch.cuda.empty_cache()
    return out


def no_hydro():
    """Beads alone in a fluid at rest (the no-solvent comparison of Sec. III) against the
    coupled step, on the 512-replica translocation ensemble (48^3 boxes, N = 32)."""
    import torch

    from workloads import configs as WC

    w = WC.ensemble48_n32(512, WC.ENSEMBLE_SEED_GPU, WC.STORE_F32)
    log(f"no-solvent comparison on {w.name}")
    sim = build_case(w, WC.STORE_F32)
    n = 200
    res = {}
    for hydro in (True, False):
        sim.step(10, hydro=hydro)
        sim.prepare(n, hydro=hydro)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(n, hydro=hydro)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res["coupled" if hydro else "no_solvent"] = {
            "replica_steps_per_s": round(len(w.replicas) * n / dt, 1), "ms_per_step": round(dt / n * 1e3, 4)}
    res["workload"] = w.name
    res["speedup_without_solvent"] = round(res["no_solvent"]["replica_steps_per_s"]
                                           / res["coupled"]["replica_steps_per_s"], 2)
    sim.close()
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-extras", action="store_true", help="skip the other workloads")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs the coupled step on one GPU; --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from workloads import configs as WC

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    w = WC.c5_large(WC.STORE_F32)
    fluid = w.fluid_nodes
    rep = w.replicas[0]

    log(f"building {w.name} (fp32, {rep.n_beads} beads)")
    sim = build_case(w, WC.STORE_F32)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    log(f"timing {args.steps} coupled steps")
    dt = time_steps(sim, args.steps)
    step_s = dt / args.steps
    mlups = fluid * args.steps / dt / 1e6
    err_word, _ = sim.status()
    md_avg, _ = event_time(sim.md_step, 10)
    log("lattice roofline")
    rl = lattice_roofline(sim, fluid, WC.STORE_F32, n=16)
    shape = sim.launch_shape()
    traffic = measured_traffic(w.name, "f32")
    sim.close()
    torch.cuda.empty_cache()
    alg = rl["alg_bytes_per_launch"]

    out = {
        "metric": "coupled D3Q19 step MLUPS & % HBM peak; fp32 vs fp16-store; replicas/s",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "box": [rep.box.nx, rep.box.ny, rep.box.nz],
                   "walls": len(rep.box.walls), "fluid_nodes": fluid, "beads": rep.n_beads,
                   "chains": f"{rep.chain_len[0]} + {len(rep.chain_len) - 1} x {rep.chain_len[1]}",
                   "md_substeps": w.md.M, "storage": "f32", "diag_every": DIAG_EVERY, "launch": shape,
                   "precision_note": "populations stored and collided in FP32; bead positions, the "
                                     "conserved sums and the centre of mass in FP64 (bead velocities and "
                                     "forces FP32); beyond FP64 reductions, positions are FP64 because "
                                     "they integrate 1e5-1e6 small increments, and the rigid-bond "
                                     "multipliers and trilinear weights (options not used here) are "
                                     "FP64 too"},
        "roofline": {"bound": "hbm", "kernel": "k_stream_collide",
                     "achieved": rl["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": rl["frac"], "traffic": traffic, "alg_bytes_per_launch": alg,
                     "kernel_us_avg": rl["kernel_us_avg"], "kernel_us_single_launch": rl["kernel_us_single_launch"],
                     "coupled_step_frac": round(alg / step_s / 1e9 / HBM_PEAK_GBS, 4),
                     "same_pattern_gbs": rl["same_pattern_gbs"], "frac_of_same_pattern": rl["frac_of_same_pattern"],
                     "note": "achieved = 2 x 19 x 4 B per fluid node / the lattice kernel's average duration "
                             "(HIP events on its launch stream); coupled_step_frac = the same bytes / the "
                             "timed coupled step; same_pattern_gbs = the sweep's loads and stores without "
                             "arithmetic (lb_pattern_copy, same launch shape); traffic = FETCH_SIZE + "
                             "WRITE_SIZE per launch from the committed counter runs (flat mapping, 256-thread "
                             "blocks, contiguous XCD ranges; null if the kernel source changed since); the bead "
                             f"kernel alone takes {md_avg * 1e6:.0f} us per step (md_step, events), hidden "
                             "under the sweep in the coupled step"},
        "error_word": err_word,
        "paper_context": "0.262 MLUPS coupled (N=100, 80x40x40 box) on a serial 2 GHz Opteron",
    }
    if not args.no_extras:
        out["workloads"] = extra_workloads(step_s)
        out["no_solvent"] = no_hydro()
        tt = {}
        for st in (WC.STORE_F64, WC.STORE_F32, WC.STORE_F16, WC.STORE_BF16):
            log(f"translocation times {WC.STORE_NAMES[st]}")
            tt[WC.STORE_NAMES[st]] = translocation_times(st)
        out["translocation_time_48cube_n32"] = tt
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
