"""Writes the oracle's ensemble of translocation times used by the distributional GPU test.

Every event is one replica of the 48^3 pore box of workloads.configs.ensemble48_n32 (the
translocation set-up of Sec. III at a reduced size): a 32-bead chain grown from the pore mouth
with its own seed, advanced by FP64 coupled oracle steps until every bead lies past the wall's
mid-plane (the completion step t_done) or the step cap is reached (t_done = -1, censored).
After every step the oracle's translocation observables are taken (Sec. III: S_H, S_E, K,
the radii of gyration of both sides); each event row also holds their means over the event
(steps 1..t_done), the ratio R_T(t_done) / R_U(1), and whether the chain retracted.
With --no-hydro the beads move alone in a fluid at rest (u = 0, no lattice, the no-solvent
comparison of Sec. III) and the sample goes to transloc_pore48_n32_nohydro.txt; with
--model paper the chain is the paper's own (rigid bonds, M = 5, eps = 2e-3) and the sample goes
to transloc_pore48_n32_rigid.txt.
Only oracle/ and the seeded input generators of workloads/ are called.

    python tests/golden/make_transloc_ensemble.py --events 256 --jobs 8
    python tests/golden/make_transloc_ensemble.py --events 512 --jobs 8 --no-hydro
    python tests/golden/make_transloc_ensemble.py --events 256 --jobs 8 --model paper
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HERE = os.path.dirname(os.path.abspath(__file__))
CHUNK = 50


def _model(name):
    from workloads import configs as WC

    return WC.paper_polymer() if name == "paper" else WC.MDParams()


def _event(args):
    k, hydro, model = args
    os.environ["OMP_NUM_THREADS"] = "1"
    import numpy as np

    from oracle import oracle as O
    from workloads import configs as WC
    from workloads import generate as G

    w = WC.ensemble48_n32(k + 1, WC.ENSEMBLE_SEED_ORACLE, md=_model(model))
    rep = w.replicas[k]
    beads = G.replica_beads(rep, w.md)
    f0 = O.equilibrium_populations(rep.box, np.full(rep.box.nodes, rep.box.rho0),
                                   np.zeros((3, rep.box.nodes)))
    sim = O.Sim(rep.box, w.md, rep.chain_len, f0, beads, None, seed=rep.seed)
    obs = []
    while sim.t_done < 0 and sim.step_no < WC.ENSEMBLE_STEP_CAP:
        sim.step(1, hydro=hydro)
        obs.append(sim.observables())
    obs = np.array(obs)
    n = rep.n_beads
    # retraction: N_T reached max(2, N/10) and fell back to 0 (the analysis module's rule)
    thr, seen, retr = max(2, n // 10), False, 0
    for v in obs[:, 0]:
        if v >= thr:
            seen = True
        elif seen and v == 0:
            retr = 1
            break
    if sim.t_done > 0:
        ev = obs[: sim.t_done]
        extra = (ev[:, 1].mean(), ev[:, 2].mean(), ev[:, 3].mean(), np.sqrt(ev[-1, 5] / ev[0, 4]))
    else:
        extra = (float("nan"),) * 4
    return (rep.seed, sim.t_done, sim.flags) + tuple(float(x) for x in extra) + (retr,)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--events", type=int, default=256)
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--no-hydro", action="store_true")
    ap.add_argument("--model", choices=["harmonic", "paper"], default="harmonic")
    args = ap.parse_args()
    hydro = not args.no_hydro
    if args.model == "paper":
        assert hydro, "the rigid-chain sample is the coupled one"
        out = os.path.join(HERE, "transloc_pore48_n32_rigid.txt")
    else:
        out = os.path.join(HERE, "transloc_pore48_n32.txt" if hydro else "transloc_pore48_n32_nohydro.txt")
    from multiprocessing import get_context

    from workloads import configs as WC

    t0 = time.time()
    rows = []
    with get_context("spawn").Pool(args.jobs) as pool:
        for i, row in enumerate(pool.imap(_event, [(k, hydro, args.model) for k in range(args.events)])):
            rows.append(row)
            print(f"event {i}: seed {row[0]} t_done {row[1]} flags {row[2]} S_H {row[3]:.3e} "
                  f"S_E {row[4]:.3e} K {row[5]:.3e} R_T/R_U {row[6]:.3f} retracted {row[7]} "
                  f"({time.time() - t0:.0f} s)", flush=True)
    md = _model(args.model)
    with open(out, "w") as fh:
        fh.write("# Translocation times of the FP64 oracle (coupled LB + bead steps, Sec. II-III).\n"
                 if hydro else
                 "# Translocation times of the FP64 oracle, beads alone in a fluid at rest (u = 0, "
                 "the no-solvent comparison of Sec. III).\n")
        fh.write("# Written by tests/golden/make_transloc_ensemble.py; inputs from workloads.configs."
                 "ensemble48_n32.\n")
        fh.write("# box 48^3, free-slip faces, tau=1, one wall x=22..24 with pore y,z=23..25; "
                 "one chain of 32 beads from the pore mouth\n")
        fh.write(f"# M={md.M} mass={md.mass} gamma={md.gamma} kT={md.kT} k_bond={md.k_bond} "
                 f"r0={md.r0} eps={md.eps} sigma={md.sigma} eps_w={md.eps_w} sigma_w={md.sigma_w} "
                 f"f_drive={md.f_drive} rigid={md.rigid} kappa_phi={md.kappa_phi}\n")
        fh.write(f"# seeds {WC.ENSEMBLE_SEED_ORACLE}+k; step cap {WC.ENSEMBLE_STEP_CAP}; "
                 "t_done = -1 marks a censored event\n")
        fh.write("# per event: means over steps 1..t_done of S_H = m gamma sum v.u, S_E = sum "
                 "F_drive.v, K = m/2 sum v^2; R_T(t_done)/R_U(1); retracted (0/1)\n")
        fh.write("# seed t_done flags S_H S_E K R_T_end_over_R_U_start retracted\n")
        for seed, t, fl, sh, se, ke, rr, retr in rows:
            fh.write(f"{seed} {t} {fl} {sh:.10e} {se:.10e} {ke:.10e} {rr:.10e} {retr}\n")
    print(f"wrote {out}: {len(rows)} events in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
