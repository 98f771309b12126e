"""Shared helpers for the GPU parity tests: build the same seeded case for the
oracle and for the HIP library, and compare."""
from __future__ import annotations

import sys

import numpy as np

from oracle import oracle as O
from workloads.configs import Replica


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def initial_f(box, rho=None, u=None):
    V = box.nodes
    rho = np.full(V, box.rho0) if rho is None else rho
    u = np.zeros((3, V)) if u is None else u
    return O.equilibrium_populations(box, rho, u)


def oracle_sim(rep: Replica, md, rho=None, u=None, beads=None, v=None, step0=0, pops=None):
    f0 = pops if pops is not None else initial_f(rep.box, rho, u)
    r0 = beads if beads is not None else np.zeros((0, 3))
    return O.Sim(rep.box, md, rep.chain_len, f0, r0, v, seed=rep.seed, step0=step0)


def gpu_sim(reps, md, storage, rho=None, u=None, beads=None, v=None, pops=None, step0=0, **kw):
    from paper_0710_1272_amd import lbmd as B

    init = {"step0": step0}
    if rho is not None:
        init["rho"] = rho
    if u is not None:
        init["u"] = u
    if pops is not None:
        init["pops"] = pops
    if beads is not None and len(beads):
        init["bead_r"] = beads
    if v is not None:
        init["bead_v"] = v
    return B.Simulation(reps, md, storage, init, **kw)


def max_rel(gpu: np.ndarray, ora: np.ndarray, fluid: np.ndarray) -> float:
    g, o = gpu[:, fluid], ora[:, fluid]
    return float(np.max(np.abs(g - o) / np.abs(o)))


def min_tie_distance(r: np.ndarray) -> float:
    """Distance of any coordinate of r + 1/2 from an integer (NGP decision margin)."""
    if len(r) == 0:
        return 1.0
    frac = (r + 0.5) - np.floor(r + 0.5)
    return float(np.min(np.minimum(frac, 1.0 - frac)))
