"""Workload descriptions: box, wall/pore geometry, bead-model parameters.

Plain data only.  The five named workloads follow the translocation set-up of
arXiv:0710.1272, Sec. III (a box split by a wall with a square pore at its centre,
a chain started on one side and pulled through by a force active inside the pore)
at the sizes and parameters the benchmark and the tests use.

Geometry rule (the paper puts the wall "at x = N_x/2" and gives the hole side
d = 3 without a wall thickness): a wall is the three node planes c-1, c, c+1 with
c = N_x/2 - 1, and the pore is the 3 x 3 block of nodes centred on (N_y/2, N_z/2)
(the even-size centre tie resolved upward).  A second wall, when present, sits at
c = 3 N_x/4 - 1 and the first one at c = N_x/4 - 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

PERIODIC = 0
FREESLIP = 1

STORE_F64 = 0
STORE_F32 = 1
STORE_F16 = 2  # FP16 deviation from w_p * rho0
STORE_BF16 = 3  # BF16 deviation from w_p * rho0
STORE_NAMES = {STORE_F64: "f64", STORE_F32: "f32", STORE_F16: "f16dev", STORE_BF16: "bf16dev"}


@dataclass
class Box:
    nx: int
    ny: int
    nz: int
    bc: Tuple[int, int, int] = (PERIODIC, PERIODIC, PERIODIC)
    # each wall: (x0, x1, y0, y1, z0, z1): solid planes x0..x1, open pore y0..y1 x z0..z1
    walls: Tuple[Tuple[int, int, int, int, int, int], ...] = ()
    tau: float = 1.0
    rho0: float = 1.0
    fluid_kT: float = 0.0  # temperature of the fluctuating-LB thermal source (0: none)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    def fluid_nodes(self) -> int:
        solid = 0
        for (x0, x1, y0, y1, z0, z1) in self.walls:
            pore = (y1 - y0 + 1) * (z1 - z0 + 1) if (y0 <= y1 and z0 <= z1) else 0
            solid += (x1 - x0 + 1) * (self.ny * self.nz - pore)
        return self.nodes - solid


@dataclass
class MDParams:
    M: int = 20
    mass: float = 1.0
    gamma: float = 0.1
    kT: float = 1e-4
    k_bond: float = 100.0
    r0: float = 1.2
    eps: float = 1.0
    sigma: float = 1.8
    eps_w: float = 1.0
    sigma_w: float = 0.9
    f_drive: float = 0.02
    drive_sign: int = 1
    rigid: int = 0             # 1: rigid bonds of length r0 (SHAKE/RATTLE), k_bond unused
    kappa_phi: float = 0.0     # angular term between consecutive bonds
    shake_tol: float = 1e-12   # rigid bonds: |s^2 - r0^2| <= shake_tol r0^2
    shake_iter: int = 30       # rigid bonds: most Newton iterations per substep
    stencil: int = 0           # coupling stencil: 0 nearest node, 1 trilinear (8 surrounding nodes)


def paper_polymer(**kw) -> MDParams:
    """The bead model of Sec. II-III itself: rigid bonds b = 1.2 (SHAKE/RATTLE), M = 5,
    eps = 2e-3, sigma = 1.8, gamma = 0.1, kT = 1/beta = 1e-4, F_drive = 0.02.  The paper
    gives no kappa_phi: 0 unless set."""
    base = dict(M=5, rigid=1, eps=2e-3, eps_w=2e-3, kappa_phi=0.0)
    base.update(kw)
    return MDParams(**base)


@dataclass
class Replica:
    box: Box
    chain_len: List[int] = field(default_factory=list)
    seed: int = 0

    @property
    def n_beads(self) -> int:
        return int(sum(self.chain_len))


@dataclass
class Workload:
    name: str
    replicas: List[Replica]
    md: MDParams
    storage: int
    steps: int
    description: str = ""

    @property
    def nodes(self) -> int:
        return sum(r.box.nodes for r in self.replicas)

    @property
    def fluid_nodes(self) -> int:
        return sum(r.box.fluid_nodes() for r in self.replicas)


def centre_wall(nx: int, ny: int, nz: int, c: Optional[int] = None):
    """Three solid planes c-1..c+1 with a 3 x 3 pore at the cross-section centre."""
    if c is None:
        c = nx // 2 - 1
    cy, cz = ny // 2, nz // 2
    return (c - 1, c + 1, cy - 1, cy + 1, cz - 1, cz + 1)


def pore_box(nx: int, ny: int, nz: int, n_walls: int = 1, tau: float = 1.0) -> Box:
    if n_walls == 1:
        walls = (centre_wall(nx, ny, nz),)
    else:
        walls = (centre_wall(nx, ny, nz, nx // 4 - 1), centre_wall(nx, ny, nz, 3 * nx // 4 - 1))
    return Box(nx, ny, nz, (FREESLIP, FREESLIP, FREESLIP), walls, tau, 1.0)


BASE_SEED = 20250101


def c1_shear_box() -> Workload:
    """Plain periodic 32^3 FP64 box, no polymer (shear-wave / conservation case)."""
    box = Box(32, 32, 32, (PERIODIC, PERIODIC, PERIODIC), (), 1.0, 1.0)
    return Workload("shear32_f64", [Replica(box, [], BASE_SEED)], MDParams(), STORE_F64, 100,
                    "periodic 32^3, tau=1, shear wave u_y=0.01 sin(2 pi x/32), rho=1+U(-1e-3,1e-3)")


def c2_translocation(storage: int = STORE_F32) -> Workload:
    """128 x 64 x 64 box, one wall with a 3 x 3 pore, one N=100 chain."""
    box = pore_box(128, 64, 64)
    return Workload("pore128x64x64_n100", [Replica(box, [100], BASE_SEED)], MDParams(), storage,
                    20000, "128x64x64 D3Q19 BGK tau=1, 3x3 pore wall, N=100 chain, M=20")


def c2_paper_polymer(storage: int = STORE_F32) -> Workload:
    """The 128 x 64 x 64 / N=100 set-up with the paper's own bead model: rigid bonds,
    M = 5 substeps, eps = eps_w = 2e-3."""
    box = pore_box(128, 64, 64)
    return Workload("pore128x64x64_n100_rigid", [Replica(box, [100], BASE_SEED)], paper_polymer(), storage,
                    20000, "128x64x64 D3Q19 BGK tau=1, 3x3 pore wall, N=100 rigid chain (SHAKE/RATTLE), M=5")


def c3_translocation(storage: int = STORE_F16) -> Workload:
    box = pore_box(256, 128, 128)
    return Workload("pore256x128x128_n400", [Replica(box, [400], BASE_SEED)], MDParams(), storage,
                    20000, "256x128x128 D3Q19 BGK tau=1, 3x3 pore wall, N=400 chain, M=20")


def c4_batched(n_replicas: int = 256, storage: int = STORE_F16, seed: int = BASE_SEED) -> Workload:
    """Independent replicas, cubic boxes 48..96 (multiples of 16), N in [20, 400]."""
    import numpy as np

    rng = np.random.default_rng(seed)
    sides = rng.choice([48, 64, 80, 96], size=n_replicas)
    ns = rng.integers(20, 401, size=n_replicas)
    reps = [Replica(pore_box(int(L), int(L), int(L)), [int(n)], seed + r)
            for r, (L, n) in enumerate(zip(sides, ns))]
    return Workload(f"batched{n_replicas}_48to96", reps, MDParams(), storage, 1000,
                    f"{n_replicas} replicas, cubic 48..96, 3x3 pore wall each, N in [20,400]")


def c5_large(storage: int = STORE_F32) -> Workload:
    box = pore_box(512, 512, 512, n_walls=2)
    return Workload("large512_two_walls", [Replica(box, [800] + [25] * 64, BASE_SEED)], MDParams(),
                    storage, 100, "512^3, two pore walls, N=800 chain + 64 crowder chains of 25")


def with_storage(w: Workload, storage: int) -> Workload:
    return replace(w, storage=storage)


# Translocation-time ensembles: independent 48^3 pore boxes, one 32-bead chain each.  The
# oracle's ensemble and the GPU's ensemble draw from disjoint seed ranges, so the two samples
# of completion times are independent draws of one distribution.
ENSEMBLE_SEED_ORACLE = BASE_SEED + 100_000
ENSEMBLE_SEED_GPU = BASE_SEED + 200_000
ENSEMBLE_STEP_CAP = 4000


def ensemble48_n32(n_replicas: int, seed0: int, storage: int = STORE_F32,
                   md: Optional[MDParams] = None) -> Workload:
    """n independent 48^3 boxes with one pore wall (x = 22..24) and a 32-bead chain started in
    the pore mouth; replica k has seed seed0 + k (its chain and its random forces).  md:
    the bead model (harmonic chain by default; paper_polymer() for the rigid one)."""
    box = pore_box(48, 48, 48)
    reps = [Replica(box, [32], seed0 + k) for k in range(n_replicas)]
    return Workload(f"ensemble48_n32x{n_replicas}", reps, md or MDParams(), storage, ENSEMBLE_STEP_CAP,
                    "48^3 boxes, 3x3 pore wall, N=32 chain each, run to completion")
