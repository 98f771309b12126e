"""GPU parity for the paper's own polymer model (Sec. II): rigid bonds held by SHAKE
(positions) and RATTLE (velocities) inside every substep, and the angular term between
consecutive bonds, against the oracle's substeps and coupled steps."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from tests.common import gpu_sim, log, max_rel, min_tie_distance, oracle_sim
from workloads import configs as WC
from workloads import generate as G
from workloads.configs import FREESLIP, PERIODIC, Box, MDParams, Replica

pytestmark = pytest.mark.gpu

F64, F32 = WC.STORE_F64, WC.STORE_F32

MODELS = {
    # rigid bonds and the angular term, contacts switched on (eps = 1) so that the
    # constraint solve works against real forces
    "rigid_angle": dict(rigid=1, kappa_phi=0.05, eps=1.0, eps_w=1.0),
    "rigid": dict(rigid=1, kappa_phi=0.0, eps=1.0, eps_w=1.0),
    # harmonic bonds (k = 100) need the shorter substep of M = 20 to stay stable
    "harmonic_angle": dict(rigid=0, M=20, kappa_phi=0.05, eps=1.0, eps_w=1.0),
}


def _dense_chain(box, n, seed):
    import dataclasses
    md_gen = dataclasses.replace(MDParams(), sigma=1.75)
    return G.grow_chain(box, md_gen, n, np.random.default_rng(seed), cis_only=False)


def _bond_checks(r, v, chains, b):
    """Largest | |s| - b | and |(v_i - v_{i+1}) . s| over the bonds of the chains."""
    worst_len, worst_rel, i0 = 0.0, 0.0, 0
    for n in chains:
        s = r[i0:i0 + n - 1] - r[i0 + 1:i0 + n]
        dv = v[i0:i0 + n - 1] - v[i0 + 1:i0 + n]
        if n > 1:
            worst_len = max(worst_len, float(np.max(np.abs(np.linalg.norm(s, axis=1) - b))))
            worst_rel = max(worst_rel, float(np.max(np.abs(np.sum(dv * s, axis=1)))))
        i0 += n
    return worst_len, worst_rel


@pytest.mark.parametrize("storage,tol", [(F64, 1e-11), (F32, 2e-4)], ids=["f64", "f32"])
@pytest.mark.parametrize("periodic", [False, True], ids=["pore", "periodic"])
@pytest.mark.parametrize("lanes", [0, 1, 2, 4, 8], ids=lambda g: f"lanes{g}")
@pytest.mark.parametrize("model", list(MODELS))
def test_md_step_polymer_model(model, lanes, periodic, storage, tol):
    """One INTERP + md_step (M = 5 substeps) of a dense chain and a short one, with the
    wall, pore and faces (or periodic images), for each lanes-per-bead choice."""
    if periodic:
        box = Box(20, 16, 16, (PERIODIC,) * 3, (), 1.0)
        chains = [40, 8]
    else:
        box = Box(40, 24, 24, (FREESLIP,) * 3, ((18, 20, 10, 12, 10, 12),), 1.0)
        chains = [60, 8]
    md = WC.paper_polymer(**MODELS[model])
    a = _dense_chain(box, chains[0], 1)
    b = G.grow_chain(box, md, chains[1], np.random.default_rng(2), existing=a, cis_only=False)
    if periodic:
        a = a + np.array([12.0, 0.0, 0.0])  # the chain crosses the periodic x boundary
    beads = np.concatenate([a, b])
    if lanes * len(beads) > 512:
        pytest.skip(f"{lanes} lanes per bead need at most {512 // lanes} beads")
    rep = Replica(box, chains, 41)
    rho, u = G.random_small_flow(box, 6, du=0.01)
    from paper_0710_1272_amd import lbmd as B
    ora = oracle_sim(rep, md, rho, u, beads=beads, step0=9)
    u_o, node_o = O.interp(box, ora.f, ora.r)
    r_o, v_o = ora.r.copy(), ora.v.copy()
    fbar_o, flags_o = O.md_substeps(box, md, chains, r_o, v_o, u_o, 9, rep.seed)
    with gpu_sim([rep], md, storage, rho, u, beads=beads, step0=9, md_lanes=lanes) as sim:
        log(f"  {model}: lanes per bead {sim.md_lanes}")
        sim.couple(B.LB_COUPLE_INTERP)
        sim.md_step()
        r_g, v_g = sim.beads()
        u_g, fb_g, node_g = sim.coupling()
        word, _ = sim.status()
    scale_v = max(1.0, np.max(np.abs(v_o)))
    log(f"  {model} ({'periodic' if periodic else 'pore'}, storage {storage}): "
        f"|dr| {np.max(np.abs(r_g - r_o)):.2e} |dv| {np.max(np.abs(v_g - v_o)):.2e} "
        f"|dFbar| {np.max(np.abs(fb_g - fbar_o)):.2e} max|v| {np.max(np.abs(v_o)):.2e}")
    assert word == flags_o == 0
    assert np.array_equal(node_g, node_o)
    assert np.max(np.abs(r_g - r_o)) < tol
    assert np.max(np.abs(v_g - v_o)) < tol * scale_v
    assert np.max(np.abs(fb_g - fbar_o)) < tol * scale_v
    if md.rigid:
        dl, rel = _bond_checks(r_g, v_g, chains, md.r0)
        log(f"  bonds: max | |s| - b | {dl:.1e}, max |dv . s| {rel:.1e}")
        assert dl < 1e-10
        assert rel < (1e-12 if storage == F64 else 1e-6) * scale_v


@pytest.mark.parametrize("storage,pop_tol,pos_tol", [(F64, 1e-11, 1e-10), (F32, 1e-5, 1e-4)],
                         ids=["f64", "f32"])
def test_c2_paper_polymer_coupled_pointwise(storage, pop_tol, pos_tol):
    """30 coupled LB steps of the 128x64x64 / N=100 set-up with the rigid chain: every
    population, bead position and velocity against the oracle."""
    w = WC.c2_paper_polymer(storage)
    rep = w.replicas[0]
    beads = G.replica_beads(rep, w.md)
    ora = oracle_sim(rep, w.md, beads=beads)
    sim = gpu_sim([rep], w.md, storage, beads=beads)
    worst = np.inf
    with sim:
        for _ in range(30):
            ora.step(1)
            sim.step(1)
            r, _ = sim.beads()
            drift = float(np.max(np.abs(r - ora.r)))
            worst = min(worst, min_tie_distance(ora.r) / max(drift, 1e-15))
        f = sim.populations()
        r, v = sim.beads()
        err_word, step = sim.status()
    err = max_rel(f, ora.f, ~O.solid_mask(rep.box))
    log(f"  rigid c2 {WC.STORE_NAMES[storage]}: populations max rel {err:.2e}; "
        f"|dr| {np.max(np.abs(r - ora.r)):.2e} |dv| {np.max(np.abs(v - ora.v)):.2e}; "
        f"NGP margin / drift {worst:.1e}; oracle flags {ora.flags}")
    assert err_word == 0 and step == 30 and ora.flags == 0
    assert worst > 10.0
    assert err < pop_tol
    assert np.max(np.abs(r - ora.r)) < pos_tol
    assert np.max(np.abs(v - ora.v)) < 100 * pos_tol
    dl, rel = _bond_checks(r, v, [100], w.md.r0)
    assert dl < 1e-10 and rel < 1e-6


def test_rigid_chain_constraints_hold_over_long_run():
    """2000 coupled steps (10^4 substeps) of the rigid chain in FP32 storage, the graph
    launches of the benchmark: bond lengths stay at b to the SHAKE tolerance, relative
    velocities stay orthogonal to the bonds, and no error flag is raised."""
    w = WC.c2_paper_polymer(F32)
    rep = w.replicas[0]
    beads = G.replica_beads(rep, w.md)
    from paper_0710_1272_amd import lbmd as B
    with gpu_sim([rep], w.md, F32, beads=beads, flags=B.LB_CFG_AUTOTUNE) as sim:
        sim.step(2000)
        r, v = sim.beads()
        err_word, step = sim.status()
    dl, rel = _bond_checks(r, v, [100], w.md.r0)
    vmax = float(np.max(np.abs(v)))
    log(f"  after 2000 steps: max | |s| - b | {dl:.1e}, max |dv . s| {rel:.1e}, max|v| {vmax:.1e}")
    assert err_word == 0 and step == 2000
    assert dl < 1e-10
    assert rel < 1e-6 * max(vmax, 1e-3)


def test_shake_iteration_limit_sets_constraint_flag():
    """With one Newton iteration allowed and a tolerance no first iterate meets, the
    substep reports LB_ERR_CONSTRAINT (the oracle reports the same)."""
    box = Box(20, 16, 16, (PERIODIC,) * 3, (), 1.0)
    md = WC.paper_polymer(eps=1.0, shake_iter=1, shake_tol=1e-15)
    beads = _dense_chain(box, 20, 3) + 2.0
    rep = Replica(box, [20], 5)
    v0 = 0.05 * (2 * np.random.default_rng(1).random(beads.shape) - 1)
    ora = oracle_sim(rep, md, beads=beads, v=v0)
    r_o, vv = ora.r.copy(), ora.v.copy()
    _, flags_o = O.md_substeps(box, md, [20], r_o, vv, np.zeros_like(r_o), 0, rep.seed)
    from paper_0710_1272_amd import lbmd as B
    with gpu_sim([rep], md, F64, beads=beads, v=v0) as sim:
        sim.couple(B.LB_COUPLE_INTERP)
        sim.md_step()
        word, _ = sim.status()
    assert flags_o & O.ERR_CONSTRAINT
    assert word & B.LB_ERR_CONSTRAINT
