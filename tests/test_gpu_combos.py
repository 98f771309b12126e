"""The optional parts of the method together: the paper's rigid chain with the angular term,
the trilinear coupling stencil, the thermal source of the fluid and the observable record, in
coupled steps against the oracle (each part alone has its own tests)."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from tests.common import gpu_sim, log, max_rel, oracle_sim
from workloads import configs as WC
from workloads import generate as G
from workloads.configs import Replica

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage,pop_tol,pos_tol", [(WC.STORE_F64, 1e-11, 1e-10), (WC.STORE_F32, 1e-5, 1e-4)],
                         ids=["f64", "f32"])
@pytest.mark.parametrize("stencil", [0, 1], ids=["ngp", "trilinear"])
def test_rigid_chain_in_a_thermal_fluid(stencil, storage, pop_tol, pos_tol):
    md = WC.paper_polymer(kappa_phi=0.05, stencil=stencil)
    box = dataclasses.replace(WC.pore_box(48, 24, 24), fluid_kT=1e-4, tau=0.8)
    rep = Replica(box, [24, 5], 4711)
    beads = G.replica_beads(rep, md)
    ora = oracle_sim(rep, md, beads=beads, step0=2)
    rows_o = []
    for _ in range(20):
        ora.step(1)
        rows_o.append(ora.observables())
    with gpu_sim([rep], md, storage, beads=beads, step0=2, obs_every=1, obs_capacity=32) as sim:
        sim.step(20)
        f = sim.populations()
        r, v = sim.beads()
        rows, counted = sim.observables()
        err_word, step = sim.status()
    e = max_rel(f, ora.f, ~O.solid_mask(box))
    dr = float(np.max(np.abs(r - ora.r)))
    rows_o = np.array(rows_o)
    eo = float(np.max(np.abs(rows[:, 2] - rows_o[:, 1])) / np.max(np.abs(rows_o[:, 1])))
    log(f"  rigid + kappa + thermal, stencil {stencil}, {WC.STORE_NAMES[storage]}: populations {e:.2e}, "
        f"|dr| {dr:.2e}, S_H rel {eo:.2e}")
    assert err_word == 0 and ora.flags == 0 and step == 22 and counted == 20
    assert e < pop_tol and dr < pos_tol
    assert np.max(np.abs(v - ora.v)) < 100 * pos_tol
    assert np.array_equal(rows[:, 1], rows_o[:, 0])
    assert eo < (1e-8 if storage == WC.STORE_F64 else 1e-2)
    s = r[:23] - r[1:24]  # bonds of the 24-bead chain
    assert np.max(np.abs(np.linalg.norm(s, axis=1) - md.r0)) < 1e-10
