"""Run-to-run reproducibility (LB_CFG_DETERMINISTIC) and the parity of the fixed-point
trilinear spread it selects.

* Bitwise: two contexts of one configuration (autotuned, graph-launched, 20 coupled steps of
  a dense chain with crowders on a pore box, where many stencils and nodes are shared) give
  identical populations, positions, velocities and Fbar, for the nearest-node and trilinear
  stencils in FP32, FP16 and BF16 storage; two more contexts with other lattice launch shapes
  (block size and thread mapping: row segments, two nodes per lane) give the same bits too.
* Parity: the fixed-point spread (each contribution rounded once to a multiple of 2^-48,
  sums exact) against the oracle's FP64 spread, over 15 coupled steps (FP64, FP32) and
  10 steps in 16-bit storage, at the tolerances of the floating-point spread; and fluid +
  bead momentum kept in FP64 over 25 steps.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from tests.common import gpu_sim, log, max_rel, oracle_sim
from workloads import configs as WC
from workloads import generate as G
from workloads.configs import PERIODIC, Box, MDParams, Replica

pytestmark = pytest.mark.gpu

F64, F32, F16, BF16 = WC.STORE_F64, WC.STORE_F32, WC.STORE_F16, WC.STORE_BF16


def _flags(autotune=True):
    from paper_0710_1272_amd import lbmd as B
    return B.LB_CFG_DETERMINISTIC | (B.LB_CFG_AUTOTUNE if autotune else 0)


def _dense_case(stencil):
    """A 48x32x32 pore box with a 60-bead chain at the pore mouth and six 10-bead crowders
    packed around it (exclusion slightly inside the WCA range)."""
    box = WC.pore_box(48, 32, 32)
    md = MDParams(stencil=stencil)
    gen = dataclasses.replace(md, sigma=1.75)
    rng = np.random.default_rng(41)
    beads = [G.grow_chain(box, gen, 60, rng, start=G.pore_mouth(box))]
    for _ in range(6):
        beads.append(G.grow_chain(box, gen, 10, rng, existing=np.concatenate(beads), cis_only=False))
    return Replica(box, [60] + [10] * 6, 55), md, np.concatenate(beads)


def _run(rep, md, storage, beads, rho, u, steps, **kw):
    with gpu_sim([rep], md, storage, rho, u, beads=beads, **kw) as sim:
        sim.step(steps)
        out = dict(f=sim.populations(), rv=sim.beads(), cp=sim.coupling(), st=sim.status(),
                   shape=sim.launch_shape())
    return out


@pytest.mark.parametrize("storage", [F32, F16, BF16], ids=["f32", "f16dev", "bf16dev"])
@pytest.mark.parametrize("stencil", [0, 1], ids=["ngp", "trilinear"])
def test_two_runs_bitwise_equal(stencil, storage):
    rep, md, beads = _dense_case(stencil)
    rho, u = G.random_small_flow(rep.box, 21, du=0.01)
    a = _run(rep, md, storage, beads, rho, u, 20, flags=_flags())
    b = _run(rep, md, storage, beads, rho, u, 20, flags=_flags())
    # other lattice launch shapes (row segments; two nodes per lane): per-node results do not
    # depend on them
    c = _run(rep, md, storage, beads, rho, u, 20, flags=_flags(False), block_size=128, mapping=2)
    d = _run(rep, md, storage, beads, rho, u, 20, flags=_flags(False), block_size=256, mapping=4)
    log(f"  {['ngp', 'trilinear'][stencil]} {WC.STORE_NAMES[storage]}: shapes {a['shape']} / {c['shape']} / "
        f"{d['shape']}")
    for x in (a, b, c, d):
        assert x["st"][0] == 0
    for other in (b, c, d):
        assert np.array_equal(a["f"], other["f"])
        for k in range(2):
            assert np.array_equal(a["rv"][k], other["rv"][k])
        for k in range(3):
            assert np.array_equal(a["cp"][k], other["cp"][k])
    # the runs did move the fluid and the beads
    assert np.max(np.abs(a["rv"][0] - beads)) > 1e-2


@pytest.mark.parametrize("storage,pop_tol,pos_tol", [(F64, 1e-11, 1e-10), (F32, 1e-5, 1e-4)],
                         ids=["f64", "f32"])
def test_fixed_point_spread_coupled_steps(storage, pop_tol, pos_tol):
    rep, md, beads = _dense_case(1)
    ora = oracle_sim(rep, md, beads=beads)
    ora.step(15)
    with gpu_sim([rep], md, storage, beads=beads, flags=_flags(False)) as sim:
        sim.step(15)
        f = sim.populations()
        r, v = sim.beads()
        err_word, _ = sim.status()
    e = max_rel(f, ora.f, ~O.solid_mask(rep.box))
    dr = float(np.max(np.abs(r - ora.r)))
    log(f"  fixed-point trilinear spread {WC.STORE_NAMES[storage]}: populations {e:.2e}, |dr| {dr:.2e}")
    assert err_word == 0 and ora.flags == 0
    assert e < pop_tol and dr < pos_tol
    assert np.max(np.abs(v - ora.v)) < 100 * pos_tol


@pytest.mark.parametrize("storage,tol", [(F16, 1e-3), (BF16, 1e-2)], ids=["f16dev", "bf16dev"])
def test_fixed_point_spread_16bit(storage, tol):
    rep, md, beads = _dense_case(1)
    rho, u = G.random_small_flow(rep.box, 13, du=0.01)
    ora = oracle_sim(rep, md, rho, u, beads=beads)
    ora.step(10)
    with gpu_sim([rep], md, storage, rho, u, beads=beads, flags=_flags(False)) as sim:
        sim.step(10)
        _, ug = sim.fields()
        r, _ = sim.beads()
    fl = ~O.solid_mask(rep.box)
    _, uo = O.fields(rep.box, ora.f)
    e = float(np.max(np.abs(ug[:, fl] - uo[:, fl])) / np.max(np.abs(uo[:, fl])))
    log(f"  fixed-point trilinear {WC.STORE_NAMES[storage]}: velocity error / max|u| {e:.2e}, "
        f"|dr| {np.max(np.abs(r - ora.r)):.2e}")
    assert e < tol and np.max(np.abs(r - ora.r)) < 1e-3


def test_fixed_point_spread_momentum_fp64():
    box = Box(16, 16, 16, (PERIODIC,) * 3, (), 0.9)
    md = MDParams(stencil=1, f_drive=0.0, gamma=0.2)
    rng = np.random.default_rng(5)
    r0 = G.grow_chain(box, md, 12, rng, cis_only=False) + np.array([7.0, 0.0, 0.0])
    rho, u = G.random_small_flow(box, 9, du=0.01)
    v0 = 0.01 * rng.standard_normal(r0.shape)
    rep = Replica(box, [12], 77)
    with gpu_sim([rep], md, F64, rho, u, beads=r0, v=v0, flags=_flags(False)) as sim:
        c0 = sim.conserved()
        _, v = sim.beads()
        p0 = c0[1:] + md.mass * v.sum(axis=0)
        sim.step(25)
        c1 = sim.conserved()
        _, v = sim.beads()
        p1 = c1[1:] + md.mass * v.sum(axis=0)
    log(f"  fixed-point spread momentum drift {np.max(np.abs(p1 - p0)):.1e}")
    assert abs(c1[0] - c0[0]) < 1e-12 * c0[0]
    # each contribution is rounded to 2^-48 (3.6e-15): 25 steps of 12 beads x 8 nodes x 18
    # populations stay far inside 1e-10
    assert np.max(np.abs(p1 - p0)) < 1e-10
