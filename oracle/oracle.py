"""ctypes wrapper of the FP64 CPU oracle (lbmd_oracle.c).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It never imports the GPU library.

Arrays follow the lattice data format: populations f[19, V] with node index
x + nx*(y + ny*z); bead arrays are [n, 3] float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbmd_oracle.c")
_LIB = os.path.join(_HERE, "liblbmd_oracle.so")

Q = 19
ERR_CONSTRAINT = 32  # rigid bonds: SHAKE did not converge within shake_iter iterations


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, OpenMP over z-planes of the LB loop)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Box(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("bc", C.c_int * 3),
                ("n_walls", C.c_int), ("wall", (C.c_int * 6) * 2), ("tau", C.c_double),
                ("rho0", C.c_double), ("kT", C.c_double)]


class _MD(C.Structure):
    _fields_ = [("M", C.c_int), ("mass", C.c_double), ("gamma", C.c_double), ("kT", C.c_double),
                ("k_bond", C.c_double), ("r0", C.c_double), ("eps", C.c_double),
                ("sigma", C.c_double), ("eps_w", C.c_double), ("sigma_w", C.c_double),
                ("f_drive", C.c_double), ("drive_sign", C.c_int), ("rigid", C.c_int),
                ("kappa_phi", C.c_double), ("shake_tol", C.c_double), ("shake_iter", C.c_int),
                ("stencil", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        lp = C.POINTER(C.c_long)
        up = C.POINTER(C.c_uint32)
        bp = C.POINTER(_Box)
        mp = C.POINTER(_MD)
        L.ora_is_solid.argtypes = [bp, C.c_int, C.c_int, C.c_int]
        L.ora_is_pore.argtypes = [bp, C.c_int, C.c_int, C.c_int]
        L.ora_push_target.argtypes = [bp, C.c_int, C.c_int, C.c_int, C.c_int, ip]
        L.ora_feq.argtypes = [C.c_double, dp, dp]
        L.ora_lb_step.argtypes = [bp, dp, dp, dp, C.c_uint32, C.c_uint64]
        L.ora_lb_step.restype = C.c_long
        L.ora_add_streamed_source.argtypes = [bp, dp, dp]
        L.ora_fields.argtypes = [bp, dp, dp, dp]
        L.ora_conserved.argtypes = [bp, dp, dp]
        L.ora_philox.argtypes = [up, up, up]
        L.ora_interp.argtypes = [bp, dp, C.c_int, dp, dp, lp]
        L.ora_spread.argtypes = [bp, C.c_int, lp, dp, dp]
        L.ora_interp_trilinear.argtypes = [bp, dp, C.c_int, dp, dp]
        L.ora_spread_trilinear.argtypes = [bp, C.c_int, dp, dp, dp]
        L.ora_wall_distance.argtypes = [bp, dp, dp]
        L.ora_wall_distance.restype = C.c_double
        L.ora_conservative_forces.argtypes = [bp, mp, C.c_int, C.c_int, ip, dp, dp]
        L.ora_potential_energy.argtypes = [bp, mp, C.c_int, C.c_int, ip, dp]
        L.ora_potential_energy.restype = C.c_double
        L.ora_md_substeps.argtypes = [bp, mp, C.c_int, C.c_int, ip, dp, dp, dp, dp, C.c_uint32,
                                      C.c_uint64]
        L.ora_transloc.argtypes = [bp, C.c_int, dp, dp]
        L.ora_shake_rattle.argtypes = [bp, mp, C.c_int, C.c_int, ip, dp, dp, dp, C.c_double]
        L.ora_coupled_step.argtypes = [bp, mp, C.c_int, C.c_int, ip, dp, dp, dp, dp, dp, dp, dp,
                                       lp, C.c_uint32, C.c_uint64]
        L.ora_observables.argtypes = [bp, mp, C.c_int, dp, dp, dp, dp]
        L.ora_lattice.argtypes = [ip, dp, ip]
        L.ora_cs2.restype = C.c_double
        L.ora_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _lp(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_long))


def make_box(box) -> _Box:
    b = _Box()
    b.nx, b.ny, b.nz = box.nx, box.ny, box.nz
    for a in range(3):
        b.bc[a] = int(box.bc[a])
    b.n_walls = len(box.walls)
    for k, w in enumerate(box.walls):
        for m in range(6):
            b.wall[k][m] = int(w[m])
    b.tau = float(box.tau)
    b.rho0 = float(box.rho0)
    b.kT = float(getattr(box, "fluid_kT", 0.0))
    return b


def make_md(md) -> _MD:
    m = _MD()
    for name, _t in _MD._fields_:
        setattr(m, name, getattr(md, name))
    return m


def lattice():
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    opp = np.zeros(Q, dtype=np.int32)
    lib().ora_lattice(_ip(c), _dp(w), _ip(opp))
    return c, w, opp


def threads() -> int:
    return lib().ora_threads()


def cs2() -> float:
    return lib().ora_cs2()


def feq(rho: float, u: Sequence[float]) -> np.ndarray:
    out = np.zeros(Q)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    lib().ora_feq(float(rho), _dp(uu), _dp(out))
    return out


def philox(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    up = C.POINTER(C.c_uint32)
    lib().ora_philox(c.ctypes.data_as(up), k.ctypes.data_as(up), o.ctypes.data_as(up))
    return o


def push_target(box, x: int, y: int, z: int, q: int):
    out = np.zeros(4, dtype=np.int32)
    b = make_box(box)
    lib().ora_push_target(C.byref(b), x, y, z, q, _ip(out))
    return tuple(int(v) for v in out)


def is_solid(box, x, y, z) -> bool:
    b = make_box(box)
    return bool(lib().ora_is_solid(C.byref(b), x, y, z))


def equilibrium_populations(box, rho: np.ndarray, u: np.ndarray) -> np.ndarray:
    """f = f_eq(rho(x), u(x)) on fluid nodes, zero on solid nodes ([19, V])."""
    V = box.nodes
    f = np.zeros((Q, V))
    c, w, _ = lattice()
    cu = c.astype(np.float64) @ u  # [19, V]
    uu = np.sum(u * u, axis=0)
    s = cs2()
    f[:] = w[:, None] * rho[None, :] * (1.0 + cu / s + (cu * cu - s * uu[None, :]) / (2 * s * s))
    solid = solid_mask(box)
    f[:, solid] = 0.0
    return f


def solid_mask(box) -> np.ndarray:
    V = box.nodes
    x = np.arange(V) % box.nx
    y = (np.arange(V) // box.nx) % box.ny
    z = np.arange(V) // (box.nx * box.ny)
    solid = np.zeros(V, dtype=bool)
    for (x0, x1, y0, y1, z0, z1) in box.walls:
        inslab = (x >= x0) & (x <= x1)
        if y0 <= y1 and z0 <= z1:
            inpore = (y >= y0) & (y <= y1) & (z >= z0) & (z <= z1)
        else:
            inpore = np.zeros(V, dtype=bool)
        solid |= inslab & ~inpore
    return solid


def lb_step(box, f: np.ndarray, S: Optional[np.ndarray] = None, work: Optional[np.ndarray] = None,
            step: int = 0, seed: int = 0):
    """One LB step in place on f; the thermal source (box.fluid_kT > 0) draws its random
    numbers for LB step `step` with key `seed`."""
    b = make_box(box)
    if work is None:
        work = np.empty_like(f)
    bad = lib().ora_lb_step(C.byref(b), _dp(f), _dp(work), _dp(S) if S is not None else None,
                            step & 0xFFFFFFFF, seed)
    return bad


def add_streamed_source(box, f: np.ndarray, S: np.ndarray):
    b = make_box(box)
    lib().ora_add_streamed_source(C.byref(b), _dp(f), _dp(S))


def fields(box, f: np.ndarray):
    V = box.nodes
    rho = np.zeros(V)
    u = np.zeros((3, V))
    b = make_box(box)
    lib().ora_fields(C.byref(b), _dp(f), _dp(rho), _dp(u))
    return rho, u


def conserved(box, f: np.ndarray) -> np.ndarray:
    out = np.zeros(4)
    b = make_box(box)
    lib().ora_conserved(C.byref(b), _dp(f), _dp(out))
    return out


def interp(box, f: np.ndarray, r: np.ndarray):
    n = len(r)
    u = np.zeros((n, 3))
    node = np.zeros(n, dtype=np.int64)
    b = make_box(box)
    lib().ora_interp(C.byref(b), _dp(f), n, _dp(np.ascontiguousarray(r)), _dp(u), _lp(node))
    return u, node


def interp_trilinear(box, f: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Fluid velocity at the beads from the 8 surrounding nodes (trilinear weights)."""
    n = len(r)
    u = np.zeros((n, 3))
    lib().ora_interp_trilinear(C.byref(make_box(box)), _dp(f), n, _dp(np.ascontiguousarray(r, dtype=np.float64)),
                               _dp(u))
    return u


def spread_trilinear(box, r: np.ndarray, fbar: np.ndarray, S: Optional[np.ndarray] = None) -> np.ndarray:
    """Reaction sources S_p on the 8 nodes around each start-of-step position r."""
    if S is None:
        S = np.zeros((Q, box.nodes))
    lib().ora_spread_trilinear(C.byref(make_box(box)), len(r), _dp(np.ascontiguousarray(r, dtype=np.float64)),
                               _dp(np.ascontiguousarray(fbar, dtype=np.float64)), _dp(S))
    return S


def spread(box, node: np.ndarray, fbar: np.ndarray, S: Optional[np.ndarray] = None) -> np.ndarray:
    if S is None:
        S = np.zeros((Q, box.nodes))
    b = make_box(box)
    lib().ora_spread(C.byref(b), len(node), _lp(np.ascontiguousarray(node, dtype=np.int64)),
                     _dp(np.ascontiguousarray(fbar)), _dp(S))
    return S


def wall_distance(box, r: Sequence[float]):
    dv = np.zeros(3)
    b = make_box(box)
    d = lib().ora_wall_distance(C.byref(b), _dp(np.ascontiguousarray(r, dtype=np.float64)), _dp(dv))
    return d, dv


def conservative_forces(box, md, chain_len, r: np.ndarray):
    n = len(r)
    F = np.zeros((n, 3))
    cl = np.ascontiguousarray(chain_len, dtype=np.int32)
    b, m = make_box(box), make_md(md)
    flags = lib().ora_conservative_forces(C.byref(b), C.byref(m), n, len(cl), _ip(cl),
                                          _dp(np.ascontiguousarray(r)), _dp(F))
    return F, flags


def potential_energy(box, md, chain_len, r: np.ndarray) -> float:
    cl = np.ascontiguousarray(chain_len, dtype=np.int32)
    b, m = make_box(box), make_md(md)
    return lib().ora_potential_energy(C.byref(b), C.byref(m), len(r), len(cl), _ip(cl),
                                      _dp(np.ascontiguousarray(r)))


def md_substeps(box, md, chain_len, r, v, u, step: int, seed: int):
    """M substeps in place on r, v; returns (fbar, flags)."""
    n = len(r)
    fbar = np.zeros((n, 3))
    cl = np.ascontiguousarray(chain_len, dtype=np.int32)
    b, m = make_box(box), make_md(md)
    flags = lib().ora_md_substeps(C.byref(b), C.byref(m), n, len(cl), _ip(cl), _dp(r), _dp(v),
                                  _dp(np.ascontiguousarray(u)), _dp(fbar), step & 0xFFFFFFFF, seed)
    return fbar, flags


def shake_rattle(box, md, chain_len, r_old, u, h: float):
    """Rigid-bond projection of one substep: (r', v, flags) from the start-of-substep
    positions r_old and the unconstrained positions u."""
    cl = np.ascontiguousarray(chain_len, dtype=np.int32)
    r_new = np.ascontiguousarray(u, dtype=np.float64).copy()
    v = np.zeros_like(r_new)
    b, m = make_box(box), make_md(md)
    fl = lib().ora_shake_rattle(C.byref(b), C.byref(m), len(r_new), len(cl), _ip(cl),
                                _dp(np.ascontiguousarray(r_old, dtype=np.float64)), _dp(r_new), _dp(v), h)
    return r_new, v, fl


def transloc(box, r: np.ndarray):
    com = np.zeros(3)
    b = make_box(box)
    nt = lib().ora_transloc(C.byref(b), len(r), _dp(np.ascontiguousarray(r)), _dp(com))
    return nt, com


OBSERVABLES = ("N_T", "S_H", "S_E", "K", "R_U2", "R_T2", "x_com")


def observables(box, md, r: np.ndarray, v: np.ndarray, u: np.ndarray) -> np.ndarray:
    """The translocation observables of Sec. III for one state (names in OBSERVABLES):
    N_T, S_H = m gamma sum v.u, S_E = sum F_drive.v, K, squared radii of gyration of the
    untranslocated and translocated parts, x of the centre of mass."""
    out = np.zeros(7)
    n = len(r)
    lib().ora_observables(C.byref(make_box(box)), C.byref(make_md(md)), n,
                          _dp(np.ascontiguousarray(r, dtype=np.float64)),
                          _dp(np.ascontiguousarray(v, dtype=np.float64)),
                          _dp(np.ascontiguousarray(u, dtype=np.float64)), _dp(out))
    return out


class Sim:
    """One replica advanced by the oracle: populations, beads, step counter."""

    def __init__(self, box, md, chain_len, f0: np.ndarray, r0: np.ndarray,
                 v0: Optional[np.ndarray] = None, seed: int = 0, step0: int = 0):
        self.box, self.md = box, md
        self.chain_len = np.ascontiguousarray(chain_len, dtype=np.int32)
        self.f = np.ascontiguousarray(f0, dtype=np.float64).copy()
        n = len(r0)
        self.r = np.ascontiguousarray(r0, dtype=np.float64).copy().reshape(n, 3)
        self.v = np.zeros((n, 3)) if v0 is None else np.ascontiguousarray(v0, dtype=np.float64).copy()
        self.u = np.zeros((n, 3))
        self.fbar = np.zeros((n, 3))
        self.node = np.zeros(n, dtype=np.int64)
        self.S = np.zeros_like(self.f)
        self.work = np.zeros_like(self.f)
        self.seed = int(seed)
        self.step_no = int(step0)
        self.flags = 0
        self.t_done = -1
        self._b, self._m = make_box(box), make_md(md)

    @property
    def n(self) -> int:
        return len(self.r)

    def observables(self) -> np.ndarray:
        """Translocation observables of the current state with this step's interpolated
        fluid velocity (zero after lattice-only or no-solvent steps)."""
        return observables(self.box, self.md, self.r, self.v, self.u)

    def step(self, n_steps: int = 1, coupled: bool = True, hydro: bool = True):
        """n LB steps: coupled (Sec. II), lattice only, or, with hydro=False, the beads
        alone in a fluid at rest (u = 0; the no-solvent comparison of Sec. III): the
        populations are left as they are."""
        L = lib()
        for _ in range(n_steps):
            if not hydro:
                if self.n > 0:
                    self.u[:] = 0.0
                    fbar, fl = md_substeps(self.box, self.md, self.chain_len, self.r, self.v,
                                           self.u, self.step_no, self.seed)
                    self.fbar[:] = fbar
                    self.flags |= fl
            elif coupled and self.n > 0:
                self.flags |= L.ora_coupled_step(
                    C.byref(self._b), C.byref(self._m), self.n, len(self.chain_len),
                    _ip(self.chain_len), _dp(self.f), _dp(self.S), _dp(self.work), _dp(self.r),
                    _dp(self.v), _dp(self.u), _dp(self.fbar), _lp(self.node),
                    self.step_no & 0xFFFFFFFF, self.seed)
            else:
                if L.ora_lb_step(C.byref(self._b), _dp(self.f), _dp(self.work), None,
                                 self.step_no & 0xFFFFFFFF, self.seed) > 0:
                    self.flags |= 16
            self.step_no += 1
            if self.n > 0 and self.t_done < 0:
                nt, _ = transloc(self.box, self.r)
                if nt == self.n:
                    self.t_done = self.step_no
