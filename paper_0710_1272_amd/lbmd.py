"""Python binding of the C ABI in include/lbmd.h (liblbmd.so, gfx950).

Argument marshalling only: every step of the coupled lattice-Boltzmann / bead
dynamics path runs in the HIP kernels of the shared library.  PyTorch provides
the device memory (caller-owned buffers) and the HIP stream.  If the library has
not been built, loading fails with an error; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "liblbmd.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_EUNSTABLE, LB_ESTATE, LB_ESIZE = 0, -1, -2, -3, -4, -5, -6
LB_BC_PERIODIC, LB_BC_FREESLIP = 0, 1
LB_STORE_F64, LB_STORE_F32, LB_STORE_F16DEV, LB_STORE_BF16DEV = 0, 1, 2, 3
LB_MAX_WALLS = 2
LB_CFG_NO_GRAPH, LB_CFG_AUTOTUNE, LB_CFG_DETERMINISTIC = 1, 2, 4
LB_MAP_AUTO, LB_MAP_FLAT, LB_MAP_ROWS, LB_MAP_SHIFTED, LB_MAP_FLAT2 = 0, 1, 2, 3, 4
LB_XCD_AUTO, LB_XCD_HARDWARE, LB_XCD_CONTIGUOUS = 0, -1, -2
LB_BUF_POPS, LB_BUF_BEADS, LB_BUF_WORK = 0, 1, 2
LB_STEP_COUPLED, LB_STEP_NO_HYDRO = 1, 2
LB_COUPLE_INTERP, LB_COUPLE_SPREAD = 1, 2
(LB_MOM_CONSERVED, LB_MOM_FIELDS, LB_MOM_POPULATIONS, LB_MOM_BEADS, LB_MOM_TRANSLOC,
 LB_MOM_COUPLING, LB_MOM_STATUS, LB_MOM_OBSERVABLES) = 1, 2, 3, 4, 5, 6, 7, 8
# columns of an LB_MOM_OBSERVABLES row
OBS_COLUMNS = ("step", "N_T", "S_H", "S_E", "K", "R_U2", "R_T2", "x_com")
LB_ERR_BEAD_IN_SOLID, LB_ERR_BEAD_OUTSIDE, LB_ERR_NONFINITE, LB_ERR_BOND_STRETCH, LB_ERR_DENSITY = (
    1, 2, 4, 8, 16)
LB_ERR_CONSTRAINT = 32
LB_STENCIL_NGP, LB_STENCIL_TRILINEAR = 0, 1

EXPORTED = ["lb_required_bytes", "lb_validate_config", "lb_init", "lb_step", "lb_graph_prepare", "lb_couple", "md_step",
            "lb_moments", "lb_moments_bytes", "lb_moments_range", "lb_block_size", "lb_launch_shape", "lb_md_lanes", "lb_destroy",
            "lb_strerror", "lb_last_error_message", "lb_conserved_noalloc", "lb_pattern_copy", "lb_plane_stride"]


class lbmd_wall(C.Structure):
    _fields_ = [("x0", C.c_int), ("x1", C.c_int), ("y0", C.c_int), ("y1", C.c_int), ("z0", C.c_int),
                ("z1", C.c_int)]


class lbmd_replica(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("bc", C.c_int * 3),
                ("n_walls", C.c_int), ("wall", lbmd_wall * LB_MAX_WALLS), ("tau", C.c_double),
                ("rho0", C.c_double), ("fluid_kT", C.c_double), ("n_chains", C.c_int),
                ("chain_len", C.POINTER(C.c_int)),
                ("seed", C.c_uint64)]


class lbmd_md_params(C.Structure):
    _fields_ = [("M", C.c_int), ("mass", C.c_double), ("gamma", C.c_double), ("kT", C.c_double),
                ("k_bond", C.c_double), ("r0", C.c_double), ("eps", C.c_double),
                ("sigma", C.c_double), ("eps_w", C.c_double), ("sigma_w", C.c_double),
                ("f_drive", C.c_double), ("drive_sign", C.c_int), ("rigid", C.c_int),
                ("kappa_phi", C.c_double), ("shake_tol", C.c_double), ("shake_iter", C.c_int),
                ("stencil", C.c_int)]


class lbmd_initial_state(C.Structure):
    _fields_ = [("rho", C.POINTER(C.c_double)), ("u", C.POINTER(C.c_double)),
                ("pops", C.POINTER(C.c_double)), ("bead_r", C.POINTER(C.c_double)),
                ("bead_v", C.POINTER(C.c_double)), ("step0", C.c_int64)]


class lbmd_config(C.Structure):
    _fields_ = [("n_replicas", C.c_int), ("replicas", C.POINTER(lbmd_replica)), ("storage", C.c_int),
                ("md", lbmd_md_params), ("init", C.POINTER(lbmd_initial_state)),
                ("block_size", C.c_int), ("lattice_mapping", C.c_int), ("xcd_order", C.c_int),
                ("md_lanes", C.c_int), ("flags", C.c_uint), ("obs_every", C.c_int),
                ("obs_capacity", C.c_int)]


class lbmd_buffers(C.Structure):
    _fields_ = [("pops", C.c_void_p * 2), ("beads", C.c_void_p), ("work", C.c_void_p)]


_lib = None


def lib():
    """Loads liblbmd.so (raises if it has not been built).  torch is imported first: the
    library then binds to the HIP runtime torch has loaded (its device buffers and streams come
    from torch), rather than loading a second copy of the runtime, which does not see the
    device that torch opened."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        import torch  # noqa: F401  (loads torch's HIP runtime before the library's dependency)

        L = C.CDLL(LIB_PATH)
        cp = C.POINTER(lbmd_config)
        L.lb_required_bytes.argtypes = [cp, C.c_int]
        L.lb_required_bytes.restype = C.c_size_t
        L.lb_validate_config.argtypes = [cp]
        L.lb_init.argtypes = [cp, C.POINTER(lbmd_buffers), C.c_void_p, C.POINTER(C.c_void_p)]
        L.lb_step.argtypes = [C.c_void_p, C.c_int, C.c_uint]
        L.lb_graph_prepare.argtypes = [C.c_void_p, C.c_int, C.c_uint]
        L.lb_couple.argtypes = [C.c_void_p, C.c_uint]
        L.md_step.argtypes = [C.c_void_p]
        L.lb_moments.argtypes = [C.c_void_p, C.c_int, C.c_uint, C.c_void_p, C.c_size_t]
        L.lb_moments_range.argtypes = [C.c_void_p, C.c_int, C.c_uint, C.c_longlong, C.c_int, C.c_void_p,
                                       C.c_size_t]
        L.lb_moments_bytes.argtypes = [C.c_void_p, C.c_int, C.c_uint]
        L.lb_moments_bytes.restype = C.c_size_t
        L.lb_block_size.argtypes = [C.c_void_p]
        L.lb_launch_shape.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                      C.POINTER(C.c_int)]
        L.lb_md_lanes.argtypes = [C.c_void_p]
        L.lb_pattern_copy.argtypes = [C.c_void_p, C.c_int]
        L.lb_conserved_noalloc.argtypes = [C.c_void_p, C.c_int, C.POINTER(lbmd_replica), C.c_void_p, C.c_void_p]
        L.lb_plane_stride.argtypes = [C.POINTER(lbmd_replica), C.c_int]
        L.lb_plane_stride.restype = C.c_longlong
        L.lb_destroy.argtypes = [C.c_void_p]
        L.lb_strerror.argtypes = [C.c_int]
        L.lb_strerror.restype = C.c_char_p
        L.lb_last_error_message.restype = C.c_char_p
        _lib = L
    return _lib


class LBError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = lib()
        super().__init__(f"{where}: {L.lb_strerror(code).decode()} ({code}): "
                         f"{L.lb_last_error_message().decode()}")
        self.code = code


def _check(code: int, where: str):
    if code != LB_OK:
        raise LBError(code, where)


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Config:
    """Builds and owns the ctypes structures (and the arrays they point to)."""

    def __init__(self, replicas, md, storage: int, init: Optional[dict] = None,
                 block_size: int = 0, flags: int = 0, mapping: int = LB_MAP_AUTO,
                 xcd_order: int = LB_XCD_AUTO, md_lanes: int = 0, obs_every: int = 0,
                 obs_capacity: int = 0):
        self._keep: List[object] = []
        n = len(replicas)
        self.reps = (lbmd_replica * n)()
        for k, rep in enumerate(replicas):
            box = rep.box
            R = self.reps[k]
            R.nx, R.ny, R.nz = box.nx, box.ny, box.nz
            for a in range(3):
                R.bc[a] = int(box.bc[a])
            R.n_walls = len(box.walls)
            for m, w in enumerate(box.walls):
                R.wall[m] = lbmd_wall(*[int(t) for t in w])
            R.tau, R.rho0 = float(box.tau), float(box.rho0)
            R.fluid_kT = float(getattr(box, "fluid_kT", 0.0))
            cl = np.ascontiguousarray(rep.chain_len, dtype=np.int32)
            self._keep.append(cl)
            R.n_chains = len(cl)
            R.chain_len = cl.ctypes.data_as(C.POINTER(C.c_int)) if len(cl) else None
            R.seed = int(rep.seed) & 0xFFFFFFFFFFFFFFFF
        self.md = lbmd_md_params()
        for name, _t in lbmd_md_params._fields_:
            setattr(self.md, name, getattr(md, name))
        self.init = lbmd_initial_state()
        init = init or {}
        for key in ("rho", "u", "pops", "bead_r", "bead_v"):
            a = init.get(key)
            if a is not None:
                a = np.ascontiguousarray(a, dtype=np.float64)
                self._keep.append(a)
                setattr(self.init, key, _dptr(a))
        self.init.step0 = int(init.get("step0", 0))
        self.cfg = lbmd_config()
        self.cfg.n_replicas = n
        self.cfg.replicas = C.cast(self.reps, C.POINTER(lbmd_replica))
        self.cfg.storage = int(storage)
        self.cfg.md = self.md
        self.cfg.init = C.pointer(self.init)
        self.cfg.block_size = int(block_size)
        self.cfg.lattice_mapping = int(mapping)
        self.cfg.xcd_order = int(xcd_order)
        self.cfg.md_lanes = int(md_lanes)
        self.cfg.flags = int(flags)
        self.cfg.obs_every = int(obs_every)
        self.cfg.obs_capacity = int(obs_capacity)

    def validate(self) -> int:
        return lib().lb_validate_config(C.byref(self.cfg))

    def required_bytes(self, which: int) -> int:
        return lib().lb_required_bytes(C.byref(self.cfg), which)


class Simulation:
    """A context of the library: replicas, their populations and beads on one GPU."""

    def __init__(self, replicas, md, storage: int, init: Optional[dict] = None,
                 block_size: int = 0, flags: int = 0, device_buffers: bool = True,
                 mapping: int = LB_MAP_AUTO, xcd_order: int = LB_XCD_AUTO, md_lanes: int = 0,
                 obs_every: int = 0, obs_capacity: int = 0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lbmd library runs on an MI355X (gfx950) only")
        self.replicas = list(replicas)
        self.storage = storage
        self._cfg = Config(self.replicas, md, storage, init, block_size, flags, mapping, xcd_order, md_lanes,
                           obs_every, obs_capacity)
        L = lib()
        self._bufs = None
        self._tensors = []
        bufs_p = None
        if device_buffers:
            sizes = [self._cfg.required_bytes(w) for w in (LB_BUF_POPS, LB_BUF_BEADS, LB_BUF_WORK)]
            if 0 in sizes:
                _check(self._cfg.validate(), "lb_validate_config")
            t = [torch.empty(sizes[0], dtype=torch.uint8, device="cuda"),
                 torch.empty(sizes[0], dtype=torch.uint8, device="cuda"),
                 torch.empty(sizes[1], dtype=torch.uint8, device="cuda"),
                 torch.empty(sizes[2], dtype=torch.uint8, device="cuda")]
            self._tensors = t
            self._bufs = lbmd_buffers()
            self._bufs.pops[0], self._bufs.pops[1] = t[0].data_ptr(), t[1].data_ptr()
            self._bufs.beads, self._bufs.work = t[2].data_ptr(), t[3].data_ptr()
            bufs_p = C.byref(self._bufs)
        self.stream = torch.cuda.current_stream()
        ctx = C.c_void_p()
        _check(L.lb_init(C.byref(self._cfg.cfg), bufs_p, C.c_void_p(self.stream.cuda_stream),
                         C.byref(ctx)), "lb_init")
        self.ctx = ctx

    # -- stepping -------------------------------------------------------------------------
    def step(self, n: int = 1, coupled: bool = True, hydro: bool = True):
        """n LB steps: coupled (default), lattice only (coupled=False), or beads only in a
        fluid at rest (hydro=False)."""
        flags = (LB_STEP_COUPLED if coupled else 0) if hydro else LB_STEP_NO_HYDRO
        _check(lib().lb_step(self.ctx, int(n), flags), "lb_step")

    def prepare(self, n: int, coupled: bool = True, hydro: bool = True):
        """Captures the HIP graphs that step(n, coupled, hydro) launches, for either buffer
        parity, without running them."""
        flags = (LB_STEP_COUPLED if coupled else 0) if hydro else LB_STEP_NO_HYDRO
        _check(lib().lb_graph_prepare(self.ctx, int(n), flags), "lb_graph_prepare")

    def couple(self, direction: int):
        _check(lib().lb_couple(self.ctx, int(direction)), "lb_couple")

    def md_step(self):
        _check(lib().md_step(self.ctx), "md_step")

    @property
    def block_size(self) -> int:
        return lib().lb_block_size(self.ctx)

    def plane_stride(self, replica: int = 0) -> int:
        """Elements between population planes in the replica's [19][S] block of a buffer."""
        s = lib().lb_plane_stride(C.byref(self._cfg.reps[replica]), self.storage)
        if s < 0:
            raise LBError(LB_EINVAL, "lb_plane_stride")
        return s

    def launch_shape(self):
        b, m, x, nt = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        _check(lib().lb_launch_shape(self.ctx, C.byref(b), C.byref(m), C.byref(x), C.byref(nt)),
               "lb_launch_shape")
        names = {LB_MAP_FLAT: "flat", LB_MAP_ROWS: "rows", LB_MAP_SHIFTED: "shifted", LB_MAP_FLAT2: "flat2"}
        return {"block": b.value, "mapping": names[m.value],
                "xcd_order": x.value, "nt_stores": bool(nt.value), "md_lanes": self.md_lanes}

    def pattern_copy(self, alternate: bool = False):
        """One same-pattern reference launch of the lattice kernel (lb_pattern_copy); with
        alternate, the copy becomes the current state (the populations lose their meaning)."""
        _check(lib().lb_pattern_copy(self.ctx, 1 if alternate else 0), "lb_pattern_copy")

    @property
    def md_lanes(self) -> int:
        """Lanes per bead of the bead kernel (0 without beads)."""
        v = lib().lb_md_lanes(self.ctx)
        if v < 0:
            _check(v, "lb_md_lanes")
        return v

    # -- observables ----------------------------------------------------------------------
    def _moments(self, replica: int, what: int, allow_unstable: bool = False) -> np.ndarray:
        L = lib()
        nbytes = L.lb_moments_bytes(self.ctx, replica, what)
        if nbytes == 0:
            raise ValueError("invalid replica or observable")
        out = np.zeros(nbytes // 8, dtype=np.float64)
        rc = L.lb_moments(self.ctx, replica, what, out.ctypes.data_as(C.c_void_p), nbytes)
        if rc == LB_EUNSTABLE and allow_unstable:
            return out
        _check(rc, "lb_moments")
        return out

    def conserved(self, replica: int = 0, allow_unstable: bool = False) -> np.ndarray:
        return self._moments(replica, LB_MOM_CONSERVED, allow_unstable)

    def populations(self, replica: int = 0, allow_unstable: bool = False) -> np.ndarray:
        return self._moments(replica, LB_MOM_POPULATIONS, allow_unstable).reshape(19, -1)

    def fields(self, replica: int = 0, allow_unstable: bool = False):
        a = self._moments(replica, LB_MOM_FIELDS, allow_unstable).reshape(4, -1)
        return a[0], a[1:4]

    def _range(self, replica: int, what: int, node0: int, count: int, ncomp: int,
               allow_unstable: bool) -> np.ndarray:
        out = np.zeros((ncomp, count), dtype=np.float64)
        rc = lib().lb_moments_range(self.ctx, replica, what, int(node0), int(count),
                                    out.ctypes.data_as(C.c_void_p), out.nbytes)
        if not (rc == LB_EUNSTABLE and allow_unstable):
            _check(rc, "lb_moments_range")
        return out

    def populations_range(self, node0: int, count: int, replica: int = 0,
                          allow_unstable: bool = False) -> np.ndarray:
        """[19][count] populations of nodes node0 .. node0 + count - 1."""
        return self._range(replica, LB_MOM_POPULATIONS, node0, count, 19, allow_unstable)

    def fields_range(self, node0: int, count: int, replica: int = 0, allow_unstable: bool = False):
        """(rho [count], u [3][count]) of nodes node0 .. node0 + count - 1."""
        a = self._range(replica, LB_MOM_FIELDS, node0, count, 4, allow_unstable)
        return a[0], a[1:4]

    def beads(self, replica: int = 0, allow_unstable: bool = False):
        a = self._moments(replica, LB_MOM_BEADS, allow_unstable)
        n = len(a) // 6
        return a[: 3 * n].reshape(n, 3), a[3 * n:].reshape(n, 3)

    def coupling(self, replica: int = 0, allow_unstable: bool = False):
        a = self._moments(replica, LB_MOM_COUPLING, allow_unstable)
        n = len(a) // 7
        return a[: 3 * n].reshape(n, 3), a[3 * n: 6 * n].reshape(n, 3), a[6 * n:].astype(np.int64)

    def transloc(self, replica: int = 0, allow_unstable: bool = False) -> dict:
        a = self._moments(replica, LB_MOM_TRANSLOC, allow_unstable)
        return {"n_t": int(a[0]), "t_done": int(a[1]), "com": a[2:5].copy(), "step": int(a[5])}

    def observables(self, replica: int = 0, allow_unstable: bool = False):
        """The recorded observable rows of a replica ([rows][8], columns OBS_COLUMNS) and the
        number of rows the kernel counted (larger than rows when the record overflowed)."""
        a = self._moments(replica, LB_MOM_OBSERVABLES, allow_unstable).reshape(-1, 8)
        counted = int(a[0, 0])
        kept = min(counted, len(a) - 1)
        return a[1:1 + kept].copy(), counted

    def status(self):
        a = self._moments(0, LB_MOM_STATUS, allow_unstable=True)
        return int(a[0]), int(a[1])

    def close(self):
        if getattr(self, "ctx", None):
            lib().lb_destroy(self.ctx)
            self.ctx = None
        self._tensors = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
