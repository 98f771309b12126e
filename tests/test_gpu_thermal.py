"""GPU parity of the thermal source F_p (fluctuating LB; Sec. II takes it from Adhikari et
al.): the same Philox draws on both sides, so populations agree with the oracle pointwise,
lattice-only and coupled, in every storage format; and the GPU fluid heats up to
equipartition, <u_a^2> = kT / rho and <(rho - rho0)^2> = rho kT / c_s^2, on boxes far
larger than the oracle's."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from tests.common import gpu_sim, log, max_rel, oracle_sim
from workloads import configs as WC
from workloads import generate as G
from workloads.configs import FREESLIP, PERIODIC, Box, MDParams, Replica

pytestmark = pytest.mark.gpu

F64, F32, F16, BF16 = WC.STORE_F64, WC.STORE_F32, WC.STORE_F16, WC.STORE_BF16
KT = 1e-4

BOXES = {
    "periodic": Box(20, 16, 12, (PERIODIC,) * 3, (), 0.8, 1.0, KT),
    "pore": Box(32, 20, 20, (FREESLIP, PERIODIC, FREESLIP), ((14, 16, 8, 10, 8, 10),), 1.0, 1.0, KT),
    "two_walls": Box(40, 16, 16, (PERIODIC, FREESLIP, FREESLIP),
                     ((8, 10, 6, 8, 6, 8), (28, 30, 7, 9, 7, 9)), 1.7, 1.0, KT),
}


def _fluid(box):
    return ~O.solid_mask(box)


@pytest.mark.parametrize("storage,tol", [(F64, 1e-11), (F32, 1e-5)], ids=["f64", "f32"])
@pytest.mark.parametrize("name", list(BOXES))
@pytest.mark.parametrize("mapping", [1, 4], ids=["flat", "flat2"])  # LB_MAP_FLAT, LB_MAP_FLAT2
def test_lattice_steps_with_thermal_source(mapping, name, storage, tol):
    box = BOXES[name]
    rep = Replica(box, [], 0x1234_5678_9ABC)
    rho, u = G.random_small_flow(box, 8, du=0.01)
    ora = oracle_sim(rep, MDParams(), rho, u, step0=3)
    ora.step(12, coupled=False)
    with gpu_sim([rep], MDParams(), storage, rho, u, step0=3, block_size=128, mapping=mapping) as sim:
        sim.step(12, coupled=False)
        f = sim.populations()
        err_word, step = sim.status()
    fl = _fluid(box)
    e = max_rel(f, ora.f, fl)
    dev = float(np.max(np.abs(ora.f[:, fl] - O.equilibrium_populations(box, *O.fields(box, ora.f))[:, fl])))
    log(f"  thermal {name} tau {box.tau} {WC.STORE_NAMES[storage]}: populations max rel {e:.2e} "
        f"(non-equilibrium part up to {dev:.1e})")
    assert err_word == 0 and step == 15
    assert dev > 1e-3, "the noise must be visible in the populations"
    assert e < tol


@pytest.mark.parametrize("storage,pop_tol,pos_tol", [(F64, 1e-11, 1e-10), (F32, 1e-5, 1e-4)],
                         ids=["f64", "f32"])
def test_coupled_steps_with_thermal_fluid(storage, pop_tol, pos_tol):
    box = dataclasses.replace(WC.pore_box(48, 24, 24), fluid_kT=KT)
    md = MDParams()
    rep = Replica(box, [16], 77)
    beads = G.replica_beads(rep, md)
    ora = oracle_sim(rep, md, beads=beads)
    ora.step(15)
    with gpu_sim([rep], md, storage, beads=beads) as sim:
        sim.step(15)
        f = sim.populations()
        r, v = sim.beads()
        err_word, _ = sim.status()
    e = max_rel(f, ora.f, _fluid(box))
    log(f"  coupled thermal {WC.STORE_NAMES[storage]}: populations max rel {e:.2e}, "
        f"|dr| {np.max(np.abs(r - ora.r)):.2e}")
    assert err_word == 0 and ora.flags == 0
    assert e < pop_tol
    assert np.max(np.abs(r - ora.r)) < pos_tol
    assert np.max(np.abs(v - ora.v)) < 100 * pos_tol


# FP16 at the 1e-3 bar of the precision requirement (measured 2.5e-4); BF16, whose 8-bit
# significand cannot reach that bar, at 1e-2 (measured 2.2e-3)
@pytest.mark.parametrize("storage,tol", [(F16, 1e-3), (BF16, 1e-2)], ids=["f16dev", "bf16dev"])
def test_thermal_source_in_16bit_storage(storage, tol):
    box = BOXES["pore"]
    rep = Replica(box, [], 99)
    ora = oracle_sim(rep, MDParams())
    ora.step(10, coupled=False)
    with gpu_sim([rep], MDParams(), storage) as sim:
        sim.step(10, coupled=False)
        rho_g, u_g = sim.fields()
    rho_o, u_o = O.fields(box, ora.f)
    fl = _fluid(box)
    eu = float(np.max(np.abs(u_g[:, fl] - u_o[:, fl])) / np.max(np.abs(u_o[:, fl])))
    er = float(np.max(np.abs(rho_g[fl] - rho_o[fl])) / np.max(np.abs(rho_o[fl] - box.rho0)))
    log(f"  {WC.STORE_NAMES[storage]}: velocity error / max|u| {eu:.2e}, density error / max|drho| {er:.2e}")
    assert eu < tol and er < tol


def test_graph_and_direct_launches_equal_with_thermal_source():
    """The thermal sweep reads the step counter, which then moves in a launch of its own:
    graph replays, plain launches and lattice-only or coupled steps all draw the same
    numbers for the same step."""
    from paper_0710_1272_amd import lbmd as B
    box = dataclasses.replace(WC.pore_box(48, 24, 24), fluid_kT=KT)
    md = MDParams()
    rep = Replica(box, [12], 5)
    beads = G.replica_beads(rep, md)
    out = []
    for flags in (0, B.LB_CFG_NO_GRAPH):
        with gpu_sim([rep], md, F32, beads=beads, flags=flags) as sim:
            sim.step(7, coupled=False)
            sim.step(19)
            out.append((sim.populations(), sim.beads()[0], sim.status()[1]))
    assert out[0][2] == out[1][2] == 26
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("storage,tau", [(F32, 0.8), (F32, 1.0), (F16, 1.0), (F64, 1.6)],
                         ids=["f32-tau0.8", "f32-tau1", "f16dev-tau1", "f64-tau1.6"])
def test_equipartition_on_a_large_box(storage, tau):
    """A 64^3 periodic fluid heated from rest: after 1500 steps the per-node velocity and
    density variances reach kT / rho0 and rho0 kT / c_s^2 (1 % with 2.6e5 nodes and 20
    samples; total mass and momentum are fixed, which removes one mode of V)."""
    box = Box(64, 64, 64, (PERIODIC,) * 3, (), tau, 1.0, KT)
    rep = Replica(box, [], 4242)
    V = box.nodes
    u2, dr2 = [], []
    with gpu_sim([rep], MDParams(), storage) as sim:
        sim.step(1500, coupled=False)
        for _ in range(20):
            sim.step(50, coupled=False)
            rho, u = sim.fields()
            u2.append(np.mean(u * u, axis=1))
            dr2.append(np.mean((rho - box.rho0) ** 2))
        err_word, _ = sim.status()
    want_u2 = KT / box.rho0 * (1 - 1 / V)
    want_dr2 = box.rho0 * KT * 3.0 * (1 - 1 / V)
    u2 = np.array(u2)
    log(f"  64^3 tau {tau} {WC.STORE_NAMES[storage]}: <u^2>/(kT/rho) per axis "
        f"{np.round(u2.mean(axis=0) / want_u2, 4)}, <drho^2>/(rho kT/cs2) {np.mean(dr2) / want_dr2:.4f}")
    assert err_word == 0
    assert abs(u2.mean() / want_u2 - 1) < 0.01
    assert np.all(np.abs(u2.mean(axis=0) / want_u2 - 1) < 0.02)
    assert abs(np.mean(dr2) / want_dr2 - 1) < 0.01


def test_c2_full_size_thermal_fluid():
    """The 128x64x64 / N=100 benchmark set-up with a thermal fluid, autotuned and
    graph-launched: 10 coupled steps against the oracle."""
    from paper_0710_1272_amd import lbmd as B
    w = WC.c2_translocation(F32)
    rep = dataclasses.replace(w.replicas[0], box=dataclasses.replace(w.replicas[0].box, fluid_kT=KT))
    beads = G.replica_beads(rep, w.md)
    ora = oracle_sim(rep, w.md, beads=beads)
    ora.step(10)
    with gpu_sim([rep], w.md, F32, beads=beads, flags=B.LB_CFG_AUTOTUNE) as sim:
        sim.step(10)
        f = sim.populations()
        r, _ = sim.beads()
        err_word, _ = sim.status()
    e = max_rel(f, ora.f, _fluid(rep.box))
    log(f"  c2 thermal: populations max rel {e:.2e}, |dr| {np.max(np.abs(r - ora.r)):.2e}")
    assert err_word == 0
    assert e < 1e-5 and np.max(np.abs(r - ora.r)) < 1e-4
