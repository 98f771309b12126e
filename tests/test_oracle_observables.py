"""Pins of the oracle's translocation observables (Sec. III: N_T, the work rates S_H of eq.
Shydro and S_E of eq. Selec, the kinetic energy, the radii of gyration of the two blobs),
against closed forms and identities that do not go through the oracle's own sums."""
import numpy as np

from oracle import oracle as O
from workloads import configs as WC
from workloads.configs import MDParams

BOX = WC.pore_box(48, 24, 24)   # wall x = 22..24, pore y, z = 11..13, mid-plane x = 23
XMID = 23.0


def test_straight_chains_give_the_closed_form_radius():
    """n collinear beads b apart: R_g^2 = b^2 (n^2 - 1) / 12."""
    md = MDParams()
    b = 1.2
    for n_u, n_t in [(7, 0), (5, 3), (0, 4), (1, 6)]:
        cis = [[XMID - 2.0 - b * k, 5.0, 6.0] for k in range(n_u)]
        trans = [[XMID + 3.0, 4.0 + b * k, 17.0] for k in range(n_t)]
        r = np.array(cis + trans).reshape(-1, 3)
        o = O.observables(BOX, md, r, np.zeros_like(r), np.zeros_like(r))
        assert o[0] == n_t
        assert abs(o[4] - b * b * (n_u * n_u - 1) / 12 * (n_u > 0)) < 1e-12
        assert abs(o[5] - b * b * (n_t * n_t - 1) / 12 * (n_t > 0)) < 1e-12


def test_radius_of_gyration_equals_the_pair_form():
    """R_g^2 = (1 / 2n^2) sum_ij |r_i - r_j|^2 over each blob."""
    rng = np.random.default_rng(3)
    r = np.concatenate([np.array([XMID - 8, 12, 12]) + 3 * rng.standard_normal((9, 3)),
                        np.array([XMID + 9, 12, 12]) + 2 * rng.standard_normal((6, 3))])
    o = O.observables(BOX, MDParams(), r, np.zeros_like(r), np.zeros_like(r))
    for part, k in ((r[r[:, 0] <= XMID], 4), (r[r[:, 0] > XMID], 5)):
        d = part[:, None, :] - part[None, :, :]
        pair = np.sum(d * d) / (2 * len(part) ** 2)
        assert abs(o[k] - pair) < 1e-10 * pair


def test_work_rates_and_kinetic_energy():
    md = MDParams(mass=1.7, gamma=0.3, f_drive=0.05, drive_sign=-1)
    rng = np.random.default_rng(5)
    r = np.array([[XMID, 12.2, 11.8],     # nearest node (23, 12, 12): a pore node
                  [XMID + 0.3, 13.4, 12.6],  # (23, 13, 13): pore
                  [XMID, 14.6, 12.0],      # (23, 15, 12): solid wall node, not pore
                  [30.0, 12.0, 12.0]])     # open fluid
    u = rng.standard_normal((4, 3)) * 0.01
    # velocities along u give S_H = m gamma |u|^2 ...
    o = O.observables(BOX, md, r, 2.0 * u, u)
    assert abs(o[1] - md.mass * md.gamma * 2.0 * np.sum(u * u)) < 1e-15
    # ... and orthogonal ones none
    w = np.cross(u, rng.standard_normal((4, 3)))
    o = O.observables(BOX, md, r, w, u)
    assert abs(o[1]) < 1e-16
    # S_E: only the x velocity of pore beads, with the drive's sign
    v = np.array([[0.3, 0.1, 0.0], [-0.2, 0.0, 0.4], [0.7, 0.0, 0.0], [0.9, 0.0, 0.0]])
    o = O.observables(BOX, md, r, v, np.zeros_like(v))
    assert abs(o[2] - (-1) * md.f_drive * (0.3 - 0.2)) < 1e-15
    assert abs(o[3] - 0.5 * md.mass * np.sum(v * v)) < 1e-15
    assert abs(o[6] - r[:, 0].mean()) < 1e-15


def test_observables_of_a_simulated_state():
    """After coupled steps, S_H uses the interpolated fluid velocity of the last step."""
    md = MDParams()
    rep = WC.Replica(BOX, [12], 7)
    from workloads import generate as G
    beads = G.replica_beads(rep, md)
    f0 = O.equilibrium_populations(BOX, np.ones(BOX.nodes), np.zeros((3, BOX.nodes)))
    sim = O.Sim(BOX, md, rep.chain_len, f0, beads, seed=rep.seed)
    sim.step(20)
    o = sim.observables()
    assert abs(o[1] - md.mass * md.gamma * np.sum(sim.v * sim.u)) < 1e-15
    assert o[1] != 0.0
    sim.step(1, hydro=False)
    assert sim.observables()[1] == 0.0
