"""Oracle pins for the paper's own polymer model (Sec. II): the angular term between
consecutive bonds and rigid bonds enforced by SHAKE (positions) and RATTLE
(velocities).  Each is checked against something other than the oracle's own
formula: finite differences of the energy, a closed form, an independent nonlinear
solve of the constraint equations, and conservation laws."""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import configs as WC
from workloads import generate as G
from workloads.configs import PERIODIC, Box, MDParams


def _periodic_box(L=24):
    return Box(L, L, L, (PERIODIC,) * 3, (), 1.0)


def _chain(box, n, seed, md=None):
    md = md or MDParams()
    return G.grow_chain(box, md, n, np.random.default_rng(seed), cis_only=False)


def test_angular_force_is_minus_energy_gradient():
    box = _periodic_box()
    md = MDParams(kappa_phi=0.05, eps=1e-3)
    r = _chain(box, 8, 3)
    F, _ = O.conservative_forces(box, md, [8], r)
    h = 1e-6
    for i in range(8):
        for a in range(3):
            rp, rm = r.copy(), r.copy()
            rp[i, a] += h
            rm[i, a] -= h
            fd = -(O.potential_energy(box, md, [8], rp) - O.potential_energy(box, md, [8], rm)) / (2 * h)
            assert abs(F[i, a] - fd) < 1e-6 * max(1.0, abs(fd)), (i, a, F[i, a], fd)


def test_angular_term_right_angle_closed_form():
    """Three beads with a right angle at the middle one: V = kappa (pi/2)^2 / 2, and each
    end bead is pushed with kappa (pi/2) / b, perpendicular to its own bond, towards the
    straight chain."""
    box = _periodic_box()
    kappa, b = 0.3, 1.2
    md = MDParams(kappa_phi=kappa, eps=0.0, k_bond=0.0)
    r = np.array([[10.0, 10.0, 10.0], [10.0 + b, 10.0, 10.0], [10.0 + b, 10.0 + b, 10.0]])
    E = O.potential_energy(box, md, [3], r)
    assert abs(E - 0.5 * kappa * (np.pi / 2) ** 2) < 1e-14
    F, _ = O.conservative_forces(box, md, [3], r)
    # d1 = +x, d2 = +y: straightening moves bead 0 along -y and bead 2 along +x
    assert np.allclose(F[0], [0.0, -kappa * np.pi / (2 * b), 0.0], atol=1e-14)
    assert np.allclose(F[2], [kappa * np.pi / (2 * b), 0.0, 0.0], atol=1e-14)
    assert np.allclose(F.sum(axis=0), 0.0, atol=1e-14)


def test_straight_chain_has_no_angular_force():
    box = _periodic_box()
    md = MDParams(kappa_phi=0.5, eps=0.0, k_bond=0.0)
    r = np.array([[5.0 + 1.2 * k, 7.0, 7.0] for k in range(5)])
    F, _ = O.conservative_forces(box, md, [5], r)
    assert np.max(np.abs(F)) < 1e-15
    assert O.potential_energy(box, md, [5], r) == 0.0


def _perturbed(r, seed, scale):
    rng = np.random.default_rng(seed)
    return r + scale * (2 * rng.random(r.shape) - 1)


@pytest.mark.parametrize("chains", [[6], [3, 4]], ids=["one_chain", "two_chains"])
def test_shake_matches_an_independent_nonlinear_solve(chains):
    """The SHAKE positions satisfy the constraint equations r'_i = u_i + (lam_k d_k -
    lam_{k-1} d_{k-1})/m, |r'_k - r'_{k+1}| = b, whose multipliers scipy finds here by a
    general root finder from the same starting point."""
    from scipy.optimize import fsolve

    box = _periodic_box()
    md = WC.paper_polymer(shake_tol=1e-14, shake_iter=50, mass=1.3)
    n = sum(chains)
    r_old = np.concatenate([_chain(box, c, 10 + k) + np.array([0.0, 8.0 * k, 0.0]) for k, c in enumerate(chains)])
    u = _perturbed(r_old, 4, 0.05)
    r_new, v, fl = O.shake_rattle(box, md, chains, r_old, u, 0.2)
    assert fl == 0
    bonds = [i for i in range(n - 1) if i + 1 < n and not (chains[0] == i + 1 and len(chains) > 1)]
    d = {k: r_old[k] - r_old[k + 1] for k in bonds}

    def positions(lam):
        x = u.copy()
        for j, k in enumerate(bonds):
            x[k] += lam[j] * d[k] / md.mass
            x[k + 1] -= lam[j] * d[k] / md.mass
        return x

    def g(lam):
        x = positions(lam)
        return [np.dot(x[k] - x[k + 1], x[k] - x[k + 1]) - md.r0 ** 2 for k in bonds]

    lam = fsolve(g, np.zeros(len(bonds)), xtol=1e-14)
    assert np.max(np.abs(g(lam))) < 1e-12
    assert np.max(np.abs(positions(lam) - r_new)) < 1e-10


def test_rattle_velocities_orthogonal_and_in_the_constraint_span():
    box = _periodic_box()
    md = WC.paper_polymer()
    r_old = _chain(box, 7, 21)
    u = _perturbed(r_old, 5, 0.03)
    h = 0.2
    r_new, v, fl = O.shake_rattle(box, md, [7], r_old, u, h)
    assert fl == 0
    s = r_new[:-1] - r_new[1:]
    assert np.max(np.abs(np.sum((v[:-1] - v[1:]) * s, axis=1))) < 1e-13
    # v - (r' - r)/h = (mu_k s_k - mu_{k-1} s_{k-1}) / m for some mu: least squares fits exactly
    dv = (v - (r_new - r_old) / h).ravel()
    Amat = np.zeros((21, 6))
    for k in range(6):
        Amat[3 * k:3 * k + 3, k] += s[k] / md.mass
        Amat[3 * (k + 1):3 * (k + 1) + 3, k] -= s[k] / md.mass
    mu, *_ = np.linalg.lstsq(Amat, dv, rcond=None)
    assert np.max(np.abs(Amat @ mu - dv)) < 1e-12


def test_rigid_bonds_hold_through_substeps_with_all_forces():
    box = WC.pore_box(48, 48, 48)
    md = WC.paper_polymer(kappa_phi=0.02)
    rep = WC.Replica(box, [24], 77)
    r = G.replica_beads(rep, md)
    v = np.zeros_like(r)
    u = 0.01 * np.ones_like(r)
    for step in range(20):
        fbar, fl = O.md_substeps(box, md, [24], r, v, u, step, rep.seed)
        assert fl == 0
        lens = np.linalg.norm(r[:-1] - r[1:], axis=1)
        assert np.max(np.abs(lens - md.r0)) < 1e-11
        assert np.max(np.abs(np.sum((v[:-1] - v[1:]) * (r[:-1] - r[1:]), axis=1))) < 1e-11


def test_rigid_chain_conserves_momentum_without_external_forces():
    """Constraint reactions, WCA and the angular term are internal: with no drag, noise,
    drive or walls the total momentum of a rigid chain does not change."""
    box = _periodic_box(32)
    md = WC.paper_polymer(gamma=0.0, kT=0.0, f_drive=0.0, kappa_phi=0.05, eps=0.5)
    r = _chain(box, 12, 8) + 8.0
    rng = np.random.default_rng(2)
    h = 1.0 / md.M
    # random velocities made consistent with the constraints by one projected substep
    r, v, fl = O.shake_rattle(box, md, [12], r, r + h * 0.05 * (2 * rng.random(r.shape) - 1), h)
    p0 = v.sum(axis=0)
    assert np.max(np.abs(p0)) > 0.01
    for step in range(10):
        _, fl = O.md_substeps(box, md, [12], r, v, np.zeros_like(r), step, 1)
        assert fl == 0
    assert np.max(np.abs(v.sum(axis=0) - p0)) < 1e-12


def test_free_rigid_dimer_rotates_at_constant_rate():
    """A dimer spun about its centre: the bond length stays b and the angular speed
    stays that of the start (kick-drift with SHAKE/RATTLE, no forces)."""
    box = _periodic_box(32)
    md = WC.paper_polymer(gamma=0.0, kT=0.0, f_drive=0.0, eps=0.0)
    b, w = md.r0, 0.2
    r = np.array([[16.0 - b / 2, 16.0, 16.0], [16.0 + b / 2, 16.0, 16.0]])
    v = np.array([[0.0, -w * b / 2, 0.0], [0.0, w * b / 2, 0.0]])
    for step in range(200):
        O.md_substeps(box, md, [2], r, v, np.zeros_like(r), step, 1)
    d = r[1] - r[0]
    assert abs(np.linalg.norm(d) - b) < 1e-12
    rel = v[1] - v[0]
    assert abs(np.linalg.norm(rel) / b - w) < 1e-3 * w
    assert abs(np.dot(rel, d)) < 1e-13
