"""The C-ABI library loads, exports what include/lbmd.h declares, and validates
configurations on the host (no device call is made by these functions)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_0710_1272_amd import lbmd as B
from workloads import configs as WC
from workloads.configs import FREESLIP, PERIODIC, Box, MDParams, Replica

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "lbmd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:(?:const|long|unsigned)\s+)*\w+\**\s+\**(lb_\w+|md_\w+)\s*\(", text,
                                 flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = _declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(B.EXPORTED)


def test_strerror():
    L = B.lib()
    assert L.lb_strerror(0) == b"success"
    assert b"invalid" in L.lb_strerror(B.LB_EINVAL)
    assert L.lb_strerror(-99) == b"unknown error code"


def _cfg(replicas, md=None, storage=B.LB_STORE_F32, with_beads=True, **kw):
    n = sum(r.n_beads for r in replicas)
    init = {"bead_r": np.zeros((n, 3))} if (with_beads and n) else None
    return B.Config(replicas, md or MDParams(), storage, init, **kw)


@pytest.mark.parametrize("w", [WC.c1_shear_box(), WC.c2_translocation(), WC.c3_translocation(),
                               WC.c4_batched(8), WC.c5_large()], ids=lambda w: w.name)
def test_named_workloads_are_valid(w):
    c = _cfg(w.replicas, w.md, w.storage)
    assert c.validate() == B.LB_OK, B.lib().lb_last_error_message()
    pops = c.required_bytes(B.LB_BUF_POPS)
    elem = {0: 8, 1: 4, 2: 2, 3: 2}[w.storage]
    strides = [B.lib().lb_plane_stride(C.byref(c.reps[k]), w.storage) for k in range(len(w.replicas))]
    assert pops == 19 * sum(strides) * elem
    assert c.required_bytes(B.LB_BUF_WORK) > 0 and c.required_bytes(B.LB_BUF_BEADS) > 0


@pytest.mark.parametrize("storage", [B.LB_STORE_F64, B.LB_STORE_F32, B.LB_STORE_F16DEV, B.LB_STORE_BF16DEV])
@pytest.mark.parametrize("dims", [(512, 512, 512), (256, 128, 128), (48, 48, 48), (10, 10, 10), (1, 1, 1),
                                  (2, 64, 1)])
def test_plane_stride(storage, dims):
    """Planes start on 256-byte boundaries, an odd number of 256-byte units apart, and the
    smallest such stride at least 12032 bytes beyond the plane's nodes."""
    L = B.lib()
    rep = B.lbmd_replica()
    rep.nx, rep.ny, rep.nz = dims
    elem = {0: 8, 1: 4, 2: 2, 3: 2}[storage]
    V = dims[0] * dims[1] * dims[2]
    S = L.lb_plane_stride(C.byref(rep), storage)
    assert (S * elem) % 256 == 0 and ((S * elem) // 256) % 2 == 1
    assert S * elem >= V * elem + 12032
    assert S * elem - 512 < V * elem + 12032


def test_plane_stride_rejects_bad_input():
    L = B.lib()
    rep = B.lbmd_replica()
    rep.nx, rep.ny, rep.nz = 8, 8, 8
    assert L.lb_plane_stride(C.byref(rep), 9) == -1
    assert b"storage" in L.lb_last_error_message()
    assert L.lb_plane_stride(None, B.LB_STORE_F32) == -1
    rep.nz = 0
    assert L.lb_plane_stride(C.byref(rep), B.LB_STORE_F32) == -1


def _rep(**kw):
    box = Box(**{**dict(nx=32, ny=16, nz=16, bc=(FREESLIP,) * 3, walls=((14, 16, 7, 9, 7, 9),)), **kw})
    return Replica(box, [10], 1)


@pytest.mark.parametrize("bad", [
    dict(tau=0.5), dict(tau=float("nan")), dict(rho0=0.0), dict(nx=1),
    dict(walls=((1, 3, 7, 9, 7, 9),)), dict(walls=((14, 30, 7, 9, 7, 9),)),
    dict(walls=((14, 16, 7, 16, 7, 9),)), dict(walls=((14, 16, 7, 9, 7, 9), (17, 18, 7, 9, 7, 9))),
    dict(bc=(2, 0, 0)), dict(fluid_kT=-1e-4), dict(fluid_kT=float("inf")),
])
def test_invalid_boxes_rejected(bad):
    c = _cfg([_rep(**bad)])
    assert c.validate() == B.LB_EINVAL
    assert c.required_bytes(B.LB_BUF_POPS) == 0
    assert len(B.lib().lb_last_error_message()) > 0


@pytest.mark.parametrize("bad", [dict(M=5), dict(M=0), dict(mass=0.0), dict(drive_sign=0),
                                 dict(sigma=-1.0), dict(stencil=2), dict(stencil=-1)])
def test_invalid_md_rejected(bad):
    md = MDParams(**bad)
    assert _cfg([_rep()], md).validate() == B.LB_EINVAL


def test_kick_drift_stability_limit():
    # 2 sqrt(k/m)/M < 2: k = 100, m = 1 needs M > 10
    assert _cfg([_rep()], MDParams(M=10)).validate() == B.LB_EINVAL
    assert _cfg([_rep()], MDParams(M=11)).validate() == B.LB_OK


def test_other_invalid_configs():
    assert _cfg([_rep()], storage=7).validate() == B.LB_EINVAL
    assert _cfg([_rep()], with_beads=False).validate() == B.LB_EINVAL  # beads need positions
    assert _cfg([_rep()], block_size=96).validate() == B.LB_EINVAL
    assert _cfg([_rep()], mapping=B.LB_MAP_SHIFTED).validate() == B.LB_OK
    assert _cfg([_rep()], mapping=B.LB_MAP_FLAT2).validate() == B.LB_OK
    assert _cfg([_rep()], mapping=B.LB_MAP_FLAT2, block_size=64).validate() == B.LB_EINVAL
    assert _cfg([_rep()], mapping=B.LB_MAP_FLAT2 + 1).validate() == B.LB_EINVAL
    # one population of a replica is addressed with 32-bit byte offsets: at most 4 GiB
    big = [Replica(Box(1024, 1024, 512, (PERIODIC,) * 3), [], 1)]  # 2^29 nodes
    assert _cfg(big, storage=B.LB_STORE_F64, with_beads=False).validate() == B.LB_OK
    bigger = [Replica(Box(1024, 1024, 513, (PERIODIC,) * 3), [], 1)]
    assert _cfg(bigger, storage=B.LB_STORE_F64, with_beads=False).validate() == B.LB_EINVAL
    assert _cfg(bigger, storage=B.LB_STORE_F32, with_beads=False).validate() == B.LB_OK
    assert _cfg([_rep()], mapping=-1).validate() == B.LB_EINVAL
    box = Box(8, 8, 8, (PERIODIC,) * 3)
    assert _cfg([Replica(box, [], 0)], with_beads=False).validate() == B.LB_OK
    assert _cfg([Replica(box, [5000], 0)]).validate() == B.LB_EINVAL
    # the bead kernel holds a replica's positions in one compute unit's LDS: 53 bytes a bead
    # within 158 KB allows 3008 (rounded down to 64)
    assert _cfg([Replica(box, [3008], 0)]).validate() == B.LB_OK
    assert _cfg([Replica(box, [3009], 0)]).validate() == B.LB_EINVAL
    assert "LDS" in B.lib().lb_last_error_message().decode()


def test_no_gpu_needed_for_host_calls():
    # these calls must not touch the device: they work in a CPU-only process
    c = _cfg([_rep()])
    assert c.validate() == B.LB_OK
    # 8192 nodes x 4 bytes = 128 units of 256 bytes per plane, + 47 (odd): 175 units a plane
    assert c.required_bytes(B.LB_BUF_POPS) == 19 * 175 * 256


def test_md_lanes_validation():
    # lanes x beads of the largest replica <= 512 for grouped lanes; one lane up to 4096 beads
    one = [_rep()]  # 10 beads
    for lanes, ok in ((0, True), (1, True), (2, True), (4, True), (8, True), (16, True), (3, False),
                      (32, False), (-1, False)):
        assert (_cfg(one, md_lanes=lanes).validate() == B.LB_OK) == ok, lanes
    big = [Replica(_rep().box, [100], 1)]
    assert _cfg(big, md_lanes=4).validate() == B.LB_OK
    assert _cfg(big, md_lanes=8).validate() == B.LB_EINVAL
    assert _cfg(big, md_lanes=1).validate() == B.LB_OK
    # two lanes per bead up to 512 beads (the 1024-thread bound above 256)
    mid = [Replica(_rep().box, [300], 1)]
    assert _cfg(mid, md_lanes=2).validate() == B.LB_OK
    assert _cfg(mid, md_lanes=4).validate() == B.LB_EINVAL
    assert _cfg([Replica(_rep().box, [513], 1)], md_lanes=2).validate() == B.LB_EINVAL


def test_trilinear_node_table_in_bead_buffer():
    # the deterministic trilinear spread keeps a node table of at least 16 slots a bead
    # (8-byte key, 4-byte stride, 18 8-byte sums) in the bead buffer
    reps = [_rep()]
    ngp = _cfg(reps, MDParams(stencil=0), flags=B.LB_CFG_DETERMINISTIC)
    tri = _cfg(reps, MDParams(stencil=1), flags=B.LB_CFG_DETERMINISTIC)
    assert ngp.validate() == B.LB_OK and tri.validate() == B.LB_OK
    extra = tri.required_bytes(B.LB_BUF_BEADS) - ngp.required_bytes(B.LB_BUF_BEADS)
    assert extra >= 16 * 10 * (8 + 4 + 18 * 8)
