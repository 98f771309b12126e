"""Node leaders of the nearest-node spread when the WCA cutoff is shorter than a node cell's
diagonal (sigma = 1: rc = 2^(1/6) < sqrt(3)).

Two unbonded beads start 2.14 apart, outside the Verlet-list radius rc + skin = 2.12, and
move 0.47 towards each other in the first LB step, which ends with both on node (10, 10, 10).
The second step keeps the list built in the first (no bead has moved half the skin), so the
list does not name the pair, yet the reaction of both beads must reach that node once each
(the S_p equation summed over the beads of the node): populations and beads after two coupled
steps against the oracle, in FP32 and 16-bit storage.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from tests.common import gpu_sim, log, max_rel, oracle_sim
from workloads import configs as WC
from workloads.configs import PERIODIC, Box, MDParams, Replica

F32, F16 = WC.STORE_F32, WC.STORE_F16


def _case():
    box = Box(20, 20, 20, (PERIODIC,) * 3, (), 1.0)
    md = MDParams(sigma=1.0, f_drive=0.0)
    a1, b1 = np.array([9.55, 9.6, 10.0]), np.array([10.45, 10.4, 10.0])
    e = (b1 - a1) / np.linalg.norm(b1 - a1)
    d = 0.47
    beads = np.array([a1 - d * e, b1 + d * e])
    # one LB step of drag alone moves a bead v0 h (1 - gamma h)(1 - (1 - gamma h)^M) / (gamma h)
    gh = md.gamma / md.M
    v0 = d / ((1 - gh) * (1 - (1 - gh) ** md.M) / md.gamma)
    vel = np.array([v0 * e, -v0 * e])
    return Replica(box, [1, 1], 23), md, beads, vel


def test_case_preconditions():
    """On the oracle: the pair is outside the list radius at the first step, shares a node
    at the second, and neither bead has moved half the skin (1.0) in between."""
    rep, md, beads, vel = _case()
    rl = 2 ** (1 / 6) * md.sigma + 1.0 + 1e-3
    assert np.linalg.norm(beads[1] - beads[0]) > rl + 0.01
    ora = oracle_sim(rep, md, beads=beads, v=vel)
    ora.step(1)
    g = np.floor(ora.r + 0.5).astype(int)
    assert np.array_equal(g[0], g[1]) and np.array_equal(g[0], [10, 10, 10])
    assert np.max(np.linalg.norm(ora.r - beads, axis=1)) < 0.49
    ora.step(1)
    assert np.all(ora.node[0] == ora.node[1])


@pytest.mark.gpu
@pytest.mark.parametrize("storage", [F32, F16], ids=["f32", "f16dev"])
def test_unlisted_pair_on_one_node(storage):
    rep, md, beads, vel = _case()
    box = rep.box
    ora = oracle_sim(rep, md, beads=beads, v=vel)
    ora.step(2)
    with gpu_sim([rep], md, storage, beads=beads, v=vel) as sim:
        sim.step(2)
        r, _ = sim.beads()
        _, _, node = sim.coupling()
        word, _ = sim.status()
        if storage == F32:
            f = sim.populations()
        else:
            _, ug = sim.fields()
    fluid = ~O.solid_mask(box)
    assert word == 0
    assert node[0] == node[1] == 10 + 20 * (10 + 20 * 10)
    drift = float(np.max(np.abs(r - ora.r)))
    if storage == F32:
        err = max_rel(f, ora.f, fluid)
        log(f"  f32: populations max rel {err:.2e}; |dr| {drift:.2e}")
        assert err < 1e-5 and drift < 1e-4
    else:
        _, uo = O.fields(box, ora.f)
        e = float(np.max(np.abs(ug - uo)) / np.max(np.abs(uo)))
        log(f"  f16dev: velocity error / max|u| {e:.2e}; |dr| {drift:.2e}")
        assert e < 1e-3 and drift < 1e-3
