"""Ensemble analysis of translocation runs (Sec. III of arXiv:0710.1272), on the observable
record the bead kernel writes (LB_MOM_OBSERVABLES) and the completion steps.

* most probable translocation time: the peak of each length's duration histogram (the
  distributions are skewed towards long times, so the paper takes the peak, not the mean);
* scaling tau(N) ~ N^alpha over lengths;
* blob radii R_U, R_T of the untranslocated and translocated parts and the effective radius
  R_E = (R_T^(1/mu) + R_U^(1/mu))^mu with the Flory exponent mu = 0.6 (the R_E equation);
* work rates S_H (eq. Shydro), S_E (eq. Selec) and gamma K along each event, on time scaled
  by the event's own duration;
* retraction: a chain that falls back to the cis side after part of it has crossed.

Host-side numpy on what the GPU recorded; ``python -m paper_0710_1272_amd.ensemble`` runs the
translocation ensembles on the GPU (one replica per event, all events of a length batched).
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

FLORY_MU = 0.6
# columns of an observable row (the order of LB_MOM_OBSERVABLES)
STEP, N_T, S_H, S_E, K, R_U2, R_T2, X_COM = range(8)


def most_probable_time(times: Sequence[float], grid_points: int = 4096) -> float:
    """Peak of the duration histogram, as the mode of a Gaussian kernel density estimate
    with Silverman's bandwidth 0.9 min(sd, IQR/1.34) n^(-1/5) (a histogram's peak depends
    on its binning; the smoothed density's does not)."""
    t = np.asarray(times, dtype=np.float64)
    if len(t) < 2:
        raise ValueError("need at least two events")
    sd = t.std(ddof=1)
    q75, q25 = np.percentile(t, [75, 25])
    spread = min(sd, (q75 - q25) / 1.34) if q75 > q25 else sd
    h = 0.9 * spread * len(t) ** -0.2
    if not h > 0:
        return float(t[0])
    grid = np.linspace(t.min(), t.max(), grid_points)
    dens = np.zeros_like(grid)
    for lo in range(0, len(t), 512):  # bounded memory for large samples
        z = (grid[:, None] - t[None, lo:lo + 512]) / h
        dens += np.exp(-0.5 * z * z).sum(axis=1)
    return float(grid[int(np.argmax(dens))])


def scaling_exponent(lengths: Sequence[float], taus: Sequence[float]) -> Tuple[float, float, float]:
    """tau(N) = A N^alpha fitted by least squares on log tau = alpha log N + log A.
    Returns (alpha, standard error of alpha, A)."""
    x = np.log(np.asarray(lengths, dtype=np.float64))
    y = np.log(np.asarray(taus, dtype=np.float64))
    n = len(x)
    if n < 2:
        raise ValueError("need at least two lengths")
    xm, ym = x.mean(), y.mean()
    sxx = np.sum((x - xm) ** 2)
    alpha = float(np.sum((x - xm) * (y - ym)) / sxx)
    c = ym - alpha * xm
    resid = y - (alpha * x + c)
    se = float(np.sqrt(np.sum(resid ** 2) / (n - 2) / sxx)) if n > 2 else float("nan")
    return alpha, se, float(np.exp(c))


def effective_radius(r_u: np.ndarray, r_t: np.ndarray, mu: float = FLORY_MU) -> np.ndarray:
    """R_E = (R_T^(1/mu) + R_U^(1/mu))^mu: constant while both blobs follow R_I ~ N_I^mu."""
    r_u = np.asarray(r_u, dtype=np.float64)
    r_t = np.asarray(r_t, dtype=np.float64)
    return (r_t ** (1.0 / mu) + r_u ** (1.0 / mu)) ** mu


def retracted(n_t: Sequence[float], n_beads: int, threshold: Optional[int] = None) -> bool:
    """Whether a chain anti-translocated after a partial passage: N_T reached the threshold
    (default max(2, N/10) beads) and later fell back to 0."""
    thr = max(2, n_beads // 10) if threshold is None else threshold
    seen = False
    for v in n_t:
        if v >= thr:
            seen = True
        elif seen and v == 0:
            return True
    return False


def event_rows(rows: np.ndarray, t_done: int) -> np.ndarray:
    """The rows of one event: recorded steps up to its completion step."""
    return rows[(rows[:, STEP] >= 1) & (rows[:, STEP] <= t_done)]


def event_summary(rows: np.ndarray, t_done: int, gamma: float) -> Dict[str, float]:
    """Per-event means of S_H, S_E and gamma K over the event, and the radius ratio
    R_T(t = 1) / R_U(t = 0) (first and last recorded rows of the event)."""
    ev = event_rows(rows, t_done)
    if len(ev) == 0:
        raise ValueError("no recorded rows inside the event")
    return {"S_H": float(ev[:, S_H].mean()), "S_E": float(ev[:, S_E].mean()),
            "gammaK": float(gamma * ev[:, K].mean()),
            "R_T_end_over_R_U_start": float(np.sqrt(ev[-1, R_T2]) / np.sqrt(ev[0, R_U2]))
            if ev[0, R_U2] > 0 else float("nan"),
            "S_H_positive_fraction": float(np.mean(ev[:, S_H] > 0)),
            "S_E_negative_fraction": float(np.mean(ev[:, S_E] < 0))}


def scaled_profile(events: Iterable[Tuple[np.ndarray, int]], gamma: float, bins: int = 20) -> Dict[str, np.ndarray]:
    """Averages over events of R_U, R_T, R_E, S_H, S_E and gamma K as functions of the time
    scaled by each event's duration (t = step / t_done in (0, 1], `bins` equal bins)."""
    keys = ("R_U", "R_T", "R_E", "S_H", "S_E", "gammaK")
    acc = {k: np.zeros(bins) for k in keys}
    cnt = np.zeros(bins)
    for rows, t_done in events:
        ev = event_rows(rows, t_done)
        if len(ev) == 0:
            continue
        s = ev[:, STEP] / float(t_done)
        b = np.minimum((s * bins).astype(int), bins - 1)
        ru, rt = np.sqrt(ev[:, R_U2]), np.sqrt(ev[:, R_T2])
        vals = {"R_U": ru, "R_T": rt, "R_E": effective_radius(ru, rt), "S_H": ev[:, S_H],
                "S_E": ev[:, S_E], "gammaK": gamma * ev[:, K]}
        for k in keys:
            np.add.at(acc[k], b, vals[k])
        np.add.at(cnt, b, 1.0)
    out = {k: np.where(cnt > 0, acc[k] / np.maximum(cnt, 1), np.nan) for k in keys}
    out["t"] = (np.arange(bins) + 0.5) / bins
    out["rows"] = cnt
    return out


# ---------------------------------------------------------------------------------------
# GPU ensembles
# ---------------------------------------------------------------------------------------
def run_length(box, md, n_beads: int, events: int, seed0: int, storage: int, step_cap: int,
               hydro: bool = True, obs_every: int = 10, check_every: int = 500,
               log=print) -> Dict[str, object]:
    """All events of one chain length as one batch of replicas (each its own box and seed),
    stepped until every event completed or the cap; returns completion steps and the
    observable records."""
    from paper_0710_1272_amd import lbmd as B
    from workloads import configs as WC
    from workloads import generate as G

    reps = [WC.Replica(box, [n_beads], seed0 + k) for k in range(events)]
    beads = np.concatenate([G.replica_beads(r, md) for r in reps])
    cap_rows = step_cap // obs_every + 1
    t0 = time.perf_counter()
    with B.Simulation(reps, md, storage, {"bead_r": beads}, flags=B.LB_CFG_AUTOTUNE,
                      obs_every=obs_every, obs_capacity=cap_rows) as sim:
        steps = 0
        t_done = np.full(events, -1)
        while steps < step_cap:
            n = min(check_every, step_cap - steps)
            sim.step(n, hydro=hydro)
            steps += n
            t_done = np.array([sim.transloc(r)["t_done"] for r in range(events)])
            if steps % (10 * check_every) == 0:
                log(f"    N={n_beads} step {steps}: {int(np.sum(t_done >= 0))}/{events} completed")
            if np.all(t_done >= 0):
                break
        err, _ = sim.status()
        records = [sim.observables(r)[0] for r in range(events)]
    dt = time.perf_counter() - t0
    log(f"  N={n_beads} {'coupled' if hydro else 'no solvent'}: {int(np.sum(t_done >= 0))}/{events} "
        f"completed in {steps} steps ({dt:.1f} s, error word {err:#x})")
    return {"t_done": t_done, "records": records, "steps": steps, "seconds": dt, "error_word": err}


def analyse_length(res: Dict[str, object], n_beads: int, gamma: float) -> Dict[str, object]:
    t_done = np.asarray(res["t_done"])
    done = t_done > 0
    times = t_done[done]
    out: Dict[str, object] = {"events": int(len(t_done)), "completed": int(done.sum())}
    if done.sum() >= 2:
        out["tau_most_probable"] = most_probable_time(times)
        out["tau_mean"] = float(times.mean())
        out["tau_median"] = float(np.median(times))
    recs = [r for r, d in zip(res["records"], done) if d]
    tds = [int(t) for t in times]
    out["retraction_rate"] = float(np.mean([retracted(r[:, N_T], n_beads) for r in res["records"]]))
    if recs:
        summ = [event_summary(r, t, gamma) for r, t in zip(recs, tds)]
        for key in summ[0]:
            vals = np.array([s[key] for s in summ])
            out[f"{key}_mean"] = float(np.nanmean(vals))
        prof = scaled_profile(zip(recs, tds), gamma, bins=10)
        out["profile"] = {k: [None if not np.isfinite(x) else round(float(x), 6) for x in v]
                          for k, v in prof.items()}
    return out


def main(argv: Optional[List[str]] = None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--lengths", default="20,40,60,80,100")
    ap.add_argument("--events", type=int, default=100)
    ap.add_argument("--box", default="80,40,40", help="nx,ny,nz of each replica's box")
    ap.add_argument("--step-cap", type=int, default=20000)
    ap.add_argument("--model", choices=["paper", "harmonic"], default="paper",
                    help="paper: rigid bonds, M = 5 (Sec. II-III); harmonic: k = 100, M = 20")
    ap.add_argument("--storage", default="f32", choices=["f64", "f32", "f16dev", "bf16dev"])
    ap.add_argument("--no-hydro", action="store_true", help="also run the no-solvent comparison")
    ap.add_argument("--seed", type=int, default=20550101)
    ap.add_argument("--obs-every", type=int, default=10)
    ap.add_argument("--fluid-kT", type=float, default=0.0,
                    help="temperature of the fluctuating-LB thermal source (0: none)")
    ap.add_argument("--out", default=None, help="write the JSON result here as well")
    args = ap.parse_args(argv)

    from workloads import configs as WC

    storage = {"f64": WC.STORE_F64, "f32": WC.STORE_F32, "f16dev": WC.STORE_F16, "bf16dev": WC.STORE_BF16}[args.storage]
    nx, ny, nz = (int(v) for v in args.box.split(","))
    import dataclasses

    box = dataclasses.replace(WC.pore_box(nx, ny, nz), fluid_kT=args.fluid_kT)
    md = WC.paper_polymer() if args.model == "paper" else WC.MDParams()
    lengths = [int(v) for v in args.lengths.split(",")]
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    result: Dict[str, object] = {"box": [nx, ny, nz], "model": args.model, "storage": args.storage,
                                 "fluid_kT": args.fluid_kT,
                                 "events_per_length": args.events, "step_cap": args.step_cap, "lengths": {}}
    modes = [True, False] if args.no_hydro else [True]
    for hydro in modes:
        key = "coupled" if hydro else "no_solvent"
        per: Dict[str, object] = {}
        for n in lengths:
            res = run_length(box, md, n, args.events, args.seed + 1000 * n, storage, args.step_cap,
                             hydro=hydro, obs_every=args.obs_every, log=log)
            per[str(n)] = analyse_length(res, n, md.gamma)
            per[str(n)]["seconds"] = round(res["seconds"], 2)
            per[str(n)]["error_word"] = int(res["error_word"])
        good = [n for n in lengths if "tau_most_probable" in per[str(n)]]
        if len(good) >= 2:
            a, se, A = scaling_exponent(good, [per[str(n)]["tau_most_probable"] for n in good])
            per["alpha"] = {"alpha": a, "stderr": se, "prefactor": A}
        result["lengths"][key] = per
    line = json.dumps(result)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(line + "\n")
    print(line, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
