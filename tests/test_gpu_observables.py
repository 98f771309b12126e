"""GPU parity of the translocation observables (Sec. III) that the bead kernel records:
N_T, S_H (eq. Shydro), S_E (eq. Selec), K, the radii of gyration of both sides of the wall
and the centre of mass, step by step against the oracle's observables of the same states;
recording stride and capacity; batched replicas record independently."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from tests.common import gpu_sim, log, oracle_sim
from workloads import configs as WC
from workloads import generate as G
from workloads.configs import MDParams, Replica

pytestmark = pytest.mark.gpu

F64, F32 = WC.STORE_F64, WC.STORE_F32


def _threaded_chain(n, b):
    """A chain threading the pore of the 48x24x24 box along its axis (y = z = 12), zig-zagging
    by about 0.1 across it with bonds of length b, half of it on each side of the wall, so
    that both blobs and the drive act from the first step."""
    off = [np.array([0.12 * (-1) ** k, 0.08 * ((k % 3) - 1)]) for k in range(n)]
    x = [23.0 - b * (n // 2) + 0.3]
    for k in range(1, n):
        x.append(x[-1] + np.sqrt(b * b - np.sum((off[k] - off[k - 1]) ** 2)))
    return np.array([[x[k], 12.0 + off[k][0], 12.0 + off[k][1]] for k in range(n)])


def _compare(rows, ora_obs, steps, tol_abs, tol_rel):
    """rows: GPU record [k][8]; ora_obs: oracle observables [k][7] of the same steps."""
    assert np.array_equal(rows[:, 0], steps)
    g = rows[:, 1:]
    assert np.array_equal(g[:, 0], ora_obs[:, 0])           # N_T exactly
    for c in range(1, 7):
        scale = max(np.max(np.abs(ora_obs[:, c])), 1e-30)
        err = np.max(np.abs(g[:, c] - ora_obs[:, c]))
        assert err < tol_abs + tol_rel * scale, (O.OBSERVABLES[c], err, scale)


@pytest.mark.parametrize("model", ["harmonic", "rigid"])
@pytest.mark.parametrize("storage,tol_rel", [(F64, 1e-9), (F32, 2e-3)], ids=["f64", "f32"])
def test_observables_follow_the_oracle(model, storage, tol_rel):
    md = MDParams() if model == "harmonic" else WC.paper_polymer(eps=1.0, eps_w=1.0)
    box = WC.pore_box(48, 24, 24)
    rep = Replica(box, [16], 515)
    beads = _threaded_chain(16, md.r0)
    ora = oracle_sim(rep, md, beads=beads)
    steps = 25
    expect = []
    for _ in range(steps):
        ora.step(1)
        expect.append(ora.observables())
    for _ in range(5):
        ora.step(1, hydro=False)
        expect.append(ora.observables())
    expect = np.array(expect)
    with gpu_sim([rep], md, storage, beads=beads, obs_every=1, obs_capacity=64) as sim:
        sim.step(steps)
        sim.step(5, hydro=False)
        rows, counted = sim.observables()
        err_word, _ = sim.status()
    log(f"  {model} {WC.STORE_NAMES[storage]}: N_T {rows[[0, -1], 2 - 1]}; "
        f"S_H {rows[-6, 2]:.3e} S_E {rows[:, 3].max():.3e} R_U^2 {rows[0, 5]:.2f} R_T^2 {rows[-1, 6]:.2f}")
    assert err_word == 0 and ora.flags == 0 and counted == steps + 5
    assert np.any(expect[:, 0] > 0) and np.any(expect[:, 2] != 0), "drive and both blobs must be exercised"
    assert np.all(expect[steps:, 1] == 0.0)
    _compare(rows, expect, np.arange(1, steps + 6), 1e-14, tol_rel)


def test_record_stride_and_capacity():
    md = MDParams()
    box = WC.pore_box(48, 24, 24)
    rep = Replica(box, [12], 3)
    beads = G.replica_beads(rep, md)
    ora = oracle_sim(rep, md, beads=beads, step0=4)
    expect = []
    for _ in range(20):
        ora.step(1)
        if ora.step_no % 3 == 0:
            expect.append(ora.observables())
    with gpu_sim([rep], md, F64, beads=beads, step0=4, obs_every=3, obs_capacity=4) as sim:
        sim.step(20)
        rows, counted = sim.observables()
    # step counts 5..24 reached: rows at 6, 9, ..., 24 counted (seven), the first four kept
    assert counted == 7 and len(rows) == 4
    _compare(rows, np.array(expect[:4]), np.array([6, 9, 12, 15]), 1e-14, 1e-9)


def test_batched_replicas_record_independently():
    md = MDParams()
    reps = [Replica(WC.pore_box(48, 24, 24), [10], 11), Replica(WC.pore_box(64, 32, 32), [25], 12)]
    beads = [G.replica_beads(r, md) for r in reps]
    with gpu_sim(reps, md, F32, beads=np.concatenate(beads), obs_every=2, obs_capacity=10) as sim:
        sim.step(12)
        both = [sim.observables(k)[0] for k in range(2)]
        lanes = sim.md_lanes  # the lanes per bead set the order of a bead's force sums
    for k, rep in enumerate(reps):
        with gpu_sim([rep], md, F32, beads=beads[k], obs_every=2, obs_capacity=10, md_lanes=lanes) as one:
            one.step(12)
            assert np.array_equal(one.observables()[0], both[k])
