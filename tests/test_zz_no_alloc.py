"""lb_conserved_noalloc: the FP64 conserved sums of one replica's populations with no context
and no allocation (partial sums in the library's static device array), against lb_moments'
LB_MOM_CONSERVED of the same state; two calls in a row, the second on a smaller replica; and
the host-side rejections (no device call is made before them)."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from paper_0710_1272_amd import lbmd as B
from tests.common import gpu_sim, log
from workloads import configs as WC
from workloads import generate as G
from workloads.configs import MDParams, Replica

ELEM = {WC.STORE_F64: 8, WC.STORE_F32: 4, WC.STORE_F16: 2, WC.STORE_BF16: 2}


def _rep_struct(box):
    return B.Config([Replica(box, [], 1)], MDParams(), WC.STORE_F32).reps[0]


def test_rejections_on_the_host():
    L = B.lib()
    box = WC.pore_box(64, 32, 32)
    r = _rep_struct(box)
    assert L.lb_conserved_noalloc(None, WC.STORE_F32, C.byref(r), C.c_void_p(256), None) == B.LB_EINVAL
    assert L.lb_conserved_noalloc(C.c_void_p(256), 9, C.byref(r), C.c_void_p(256), None) == B.LB_EINVAL
    assert L.lb_conserved_noalloc(C.c_void_p(258), WC.STORE_F32, C.byref(r), C.c_void_p(256), None) == B.LB_EINVAL
    bad = _rep_struct(WC.Box(1, 8, 8))
    assert L.lb_conserved_noalloc(C.c_void_p(256), WC.STORE_F32, C.byref(bad), C.c_void_p(256), None) == B.LB_EINVAL
    # 2^27 nodes fit the static array's 32768 blocks of partial sums; 2^27 + 1024 do not
    ok = _rep_struct(WC.Box(512, 512, 512))
    big = _rep_struct(WC.Box(514, 512, 512))
    assert L.lb_conserved_noalloc(C.c_void_p(256), WC.STORE_F32, C.byref(big), C.c_void_p(256), None) == B.LB_ESIZE
    assert "2^27" in L.lb_last_error_message().decode()
    del ok


@pytest.mark.gpu
@pytest.mark.parametrize("storage", [WC.STORE_F64, WC.STORE_F32, WC.STORE_F16], ids=["f64", "f32", "f16dev"])
def test_matches_lb_moments_twice(storage):
    import torch

    L = B.lib()
    reps = [Replica(WC.pore_box(96, 48, 48), [30], 61), Replica(WC.pore_box(48, 24, 24), [10], 62)]
    md = MDParams()
    flows = [G.random_small_flow(r.box, 90 + k, du=0.01) for k, r in enumerate(reps)]
    rho = np.concatenate([f[0] for f in flows])
    u = np.concatenate([f[1].ravel() for f in flows])
    beads = np.concatenate([G.replica_beads(r, md) for r in reps])
    with gpu_sim(reps, md, storage, rho, u, beads=beads) as sim:
        sim.step(4)  # an even number of lattice updates: the current state is in buffer 0
        expect = [sim.conserved(k) for k in range(2)]
        out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        base = sim._tensors[0].data_ptr()
        offset = 0
        for k, rep in enumerate(reps):  # the second call takes the smaller replica
            log(f"  call {k + 1}: {rep.box.nx}x{rep.box.ny}x{rep.box.nz} {WC.STORE_NAMES[storage]}")
            rc = L.lb_conserved_noalloc(C.c_void_p(base + offset), storage, C.byref(sim._cfg.reps[k]),
                                        C.c_void_p(out.data_ptr()), C.c_void_p(stream))
            assert rc == B.LB_OK, L.lb_last_error_message()
            got = out.cpu().numpy()
            e = expect[k]
            log(f"    mass {got[0]:.15e} vs {e[0]:.15e}; momentum {got[1:]} vs {e[1:]}")
            assert abs(got[0] - e[0]) <= 1e-12 * e[0]
            assert np.max(np.abs(got[1:] - e[1:])) <= 1e-12 * e[0]
            offset += 19 * sim.plane_stride(k) * ELEM[storage]
