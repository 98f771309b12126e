"""Seeded synthetic inputs shared by the oracle and the GPU library.

Nothing here computes any part of the method: it only produces initial data
(bead positions of randomly grown chains, initial density/velocity fields).
Every generator takes an explicit seed and uses numpy's PCG64 stream.

Chain growth follows the set-up of arXiv:0710.1272, Sec. III: at t = 0 the whole
chain lies on one side of the wall (here the low-x "cis" side, pulled towards +x),
grown as a random walk of bond-length steps, each step redrawn when it comes
closer than the WCA range to an earlier non-bonded bead or closer than the wall
interaction range to a wall or outer face; bead 0 sits in the pore mouth so the
pulling force acts from the first step.  The paper's ensemble uses "different
realizations of the initial polymer configuration"; these are such realizations.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from .configs import FREESLIP, Box, MDParams, Replica, Workload

_WCA_RANGE = 2.0 ** (1.0 / 6.0)


def _unit_vectors(rng: np.random.Generator, k: int) -> np.ndarray:
    v = rng.normal(size=(k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _allowed_region(box: Box, md: MDParams, cis_only: bool):
    """Axis-aligned limits that keep a bead clear of faces and of wall 0's cis face."""
    margin = _WCA_RANGE * md.sigma_w * 1.05
    lo = np.array([-0.5 + margin] * 3)
    hi = np.array([box.nx - 0.5 - margin, box.ny - 0.5 - margin, box.nz - 0.5 - margin])
    for a, bc in enumerate(box.bc):
        if bc != FREESLIP:
            n = (box.nx, box.ny, box.nz)[a]
            lo[a], hi[a] = -0.5, n - 0.5
    if cis_only and box.walls:
        hi[0] = min(hi[0], box.walls[0][0] - 0.5 - margin)
    return lo, hi


def _clear_of_walls(box: Box, md: MDParams, p: np.ndarray) -> bool:
    margin = _WCA_RANGE * md.sigma_w * 1.05
    for (x0, x1, *_rest) in box.walls:
        if x0 - 0.5 - margin < p[0] < x1 + 0.5 + margin:
            return False
    return True


def grow_chain(box: Box, md: MDParams, n: int, rng: np.random.Generator,
               start: Optional[np.ndarray] = None, existing: Optional[np.ndarray] = None,
               cis_only: bool = True, max_restarts: int = 200) -> np.ndarray:
    """Random-walk chain of n beads, steps of length r0, redrawn on overlap."""
    excl = _WCA_RANGE * md.sigma
    lo, hi = _allowed_region(box, md, cis_only)
    others = existing if existing is not None else np.zeros((0, 3))
    for _ in range(max_restarts):
        if start is not None:
            p0 = np.asarray(start, dtype=np.float64)
        else:
            for _try in range(10000):
                p0 = lo + (hi - lo) * rng.random(3)
                if (_clear_of_walls(box, md, p0) and
                        (len(others) == 0 or np.min(np.linalg.norm(others - p0, axis=1)) >= excl)):
                    break
            else:
                raise RuntimeError("no free start position")
        pts = np.zeros((n, 3))
        pts[0] = p0
        ok = True
        for i in range(1, n):
            cand = pts[i - 1] + md.r0 * _unit_vectors(rng, 64)
            inside = np.all((cand > lo) & (cand < hi), axis=1)
            if box.walls and not cis_only:
                inside &= np.array([_clear_of_walls(box, md, c) for c in cand])
            good = inside
            if i >= 2:
                d = np.linalg.norm(cand[:, None, :] - pts[None, : i - 1, :], axis=2)
                good &= np.all(d >= excl, axis=1)
            if len(others):
                d = np.linalg.norm(cand[:, None, :] - others[None, :, :], axis=2)
                good &= np.all(d >= excl, axis=1)
            idx = np.flatnonzero(good)
            if len(idx) == 0:
                ok = False
                break
            pts[i] = cand[idx[0]]
        if ok:
            return pts
    raise RuntimeError(f"could not grow a chain of {n} beads")


def pore_mouth(box: Box) -> np.ndarray:
    """Just inside wall 0's pore, on its axis: 0.1 past the cis face plane x0 - 1/2,
    so the bead's nearest node is a pore node without sitting on a rounding tie."""
    x0, _x1, y0, y1, z0, z1 = box.walls[0]
    return np.array([x0 - 0.4, 0.5 * (y0 + y1), 0.5 * (z0 + z1)])


def replica_beads(rep: Replica, md: MDParams, seed: Optional[int] = None) -> np.ndarray:
    """Initial positions for all chains of a replica ([n_beads, 3] float64).

    Chain 0 starts in the pore mouth of wall 0 and lies on the cis side; further
    chains (crowders) start at random free positions anywhere clear of the walls.
    """
    rng = np.random.default_rng(rep.seed if seed is None else seed)
    box = rep.box
    out: List[np.ndarray] = []
    for c, n in enumerate(rep.chain_len):
        existing = np.concatenate(out) if out else None
        if c == 0 and box.walls:
            pts = grow_chain(box, md, n, rng, start=pore_mouth(box), existing=existing)
        else:
            pts = grow_chain(box, md, n, rng, existing=existing, cis_only=False)
        out.append(pts)
    if not out:
        return np.zeros((0, 3))
    return np.concatenate(out)


def workload_beads(w: Workload) -> List[np.ndarray]:
    return [replica_beads(r, w.md) for r in w.replicas]


def shear_wave_fields(box: Box, seed: int, amplitude: float = 0.01, noise: float = 1e-3):
    """rho = 1 + noise*(2U-1), u_y = amplitude*sin(2 pi x / nx), u_x = u_z = 0.

    Returns (rho [V], u [3, V]) in the node order x fastest, then y, then z.
    """
    rng = np.random.default_rng(seed)
    V = box.nodes
    rho = box.rho0 + noise * (2.0 * rng.random(V) - 1.0)
    x = np.arange(V) % box.nx
    u = np.zeros((3, V))
    u[1] = amplitude * np.sin(2.0 * np.pi * x / box.nx)
    return rho, u


def random_small_flow(box: Box, seed: int, du: float = 0.02, drho: float = 0.01):
    """A generic smooth-ish random state for parity tests: rho = rho0 + drho*(2U-1),
    u components uniform in [-du, du]."""
    rng = np.random.default_rng(seed)
    V = box.nodes
    rho = box.rho0 + drho * (2.0 * rng.random(V) - 1.0)
    u = du * (2.0 * rng.random((3, V)) - 1.0)
    return rho, u


def flatten_chains(chain_lens: Sequence[int]) -> np.ndarray:
    return np.asarray(list(chain_lens), dtype=np.int32)
