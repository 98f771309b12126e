"""Pins of the oracle's lattice-Boltzmann step (Eq. lbe, Sec. II of arXiv:0710.1272).

What fixes the answer, with no implementation to compare against:
  * streaming "secures exact conservation of mass and momentum" (Sec. II): the
    push map must be a bijection of (fluid node, population) slots, mass is
    conserved with any boundary mix and momentum with periodic boxes;
  * BGK collision conserves rho and j at every node;
  * nu = cs^2 (1/omega - 1/2) (Sec. II): the shear-wave decay rate; the exact
    per-step decay factor of a linear shear wave is the eigenvalue of the
    single-mode 19x19 update matrix (brute force, von Neumann analysis);
  * Poiseuille flow between bounce-back walls has an exactly parabolic bulk
    profile with curvature -F/(rho nu);
  * specular free-slip faces leave a uniform tangential flow untouched, while
    bounce-back walls do not.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from workloads.configs import FREESLIP, PERIODIC, Box
from workloads.generate import random_small_flow, shear_wave_fields

TINY_BOXES = [
    Box(6, 5, 7, (FREESLIP, PERIODIC, FREESLIP), ((2, 3, 1, 2, 3, 4),)),
    Box(9, 6, 6, (FREESLIP, FREESLIP, FREESLIP), ((2, 2, 2, 3, 2, 3), (6, 7, 1, 1, 4, 4))),
    Box(5, 4, 3, (PERIODIC, PERIODIC, PERIODIC), ((1, 1, 0, 1, 1, 1),)),
    Box(4, 4, 4, (FREESLIP, FREESLIP, FREESLIP), ()),
    Box(7, 5, 5, (PERIODIC, FREESLIP, PERIODIC), ((3, 3, 5, 4, 0, -1),)),  # wall without pore
]


def _fluid_slots(box):
    solid = O.solid_mask(box)
    for z, y, x in itertools.product(range(box.nz), range(box.ny), range(box.nx)):
        i = x + box.nx * (y + box.ny * z)
        if not solid[i]:
            yield x, y, z


@pytest.mark.parametrize("box", TINY_BOXES)
def test_push_map_is_bijection(box):
    seen = {}
    for (x, y, z) in _fluid_slots(box):
        for q in range(19):
            t = O.push_target(box, x, y, z, q)
            assert not O.is_solid(box, *t[:3])
            assert t not in seen, f"slot {t} reached from {seen.get(t)} and {(x, y, z, q)}"
            seen[t] = (x, y, z, q)
    n_fluid = sum(1 for _ in _fluid_slots(box))
    assert len(seen) == 19 * n_fluid


def test_resolver_hand_cases():
    c, _, opp = O.lattice()
    idx = {tuple(v): p for p, v in enumerate(c)}
    box = Box(6, 5, 5, (FREESLIP, FREESLIP, PERIODIC), ((3, 3, 2, 2, 2, 2),))
    # interior link
    assert O.push_target(box, 1, 1, 1, idx[(1, 1, 0)]) == (2, 2, 1, idx[(1, 1, 0)])
    # leaving through the x=0 free-slip face: x kept, c_x flipped, y still advances
    assert O.push_target(box, 0, 1, 1, idx[(-1, 1, 0)]) == (0, 2, 1, idx[(1, 1, 0)])
    # corner of two free-slip faces: both components flipped, node kept
    assert O.push_target(box, 0, 0, 1, idx[(-1, -1, 0)]) == (0, 0, 1, idx[(1, 1, 0)])
    # periodic z wraps
    assert O.push_target(box, 1, 1, 4, idx[(0, 0, 1)]) == (1, 1, 0, idx[(0, 0, 1)])
    # into the solid wall at x=3 (outside the pore): half-way bounce-back
    assert O.push_target(box, 2, 1, 1, idx[(1, 0, 0)]) == (2, 1, 1, opp[idx[(1, 0, 0)]])
    # through the pore node (3,2,2)
    assert O.push_target(box, 2, 2, 2, idx[(1, 0, 0)]) == (3, 2, 2, idx[(1, 0, 0)])
    # diagonal from the pore into the wall: bounce-back
    assert O.push_target(box, 3, 2, 2, idx[(1, 1, 0)]) == (4, 3, 2, idx[(1, 1, 0)])
    assert O.push_target(box, 3, 2, 2, idx[(0, 1, 0)]) == (3, 2, 2, opp[idx[(0, 1, 0)]])


def _random_state(box, seed):
    rho, u = random_small_flow(box, seed)
    return O.equilibrium_populations(box, rho, u) + 1e-3 * np.random.default_rng(seed).random(
        (19, box.nodes)) * (~O.solid_mask(box))


@pytest.mark.parametrize("box", TINY_BOXES)
def test_mass_conserved_any_boundaries(box):
    f = _random_state(box, 3)
    m0 = O.conserved(box, f)[0]
    for _ in range(25):
        O.lb_step(box, f)
    assert abs(O.conserved(box, f)[0] - m0) <= 1e-13 * m0


def test_collision_conserves_node_moments():
    # a single-node periodic box: streaming maps every population onto itself,
    # so one step is a pure collision
    box = Box(1, 1, 1, (PERIODIC, PERIODIC, PERIODIC), (), 0.7)
    rng = np.random.default_rng(5)
    for _ in range(20):
        f = (O.feq(1.0, 0.05 * rng.random(3)) + 0.01 * rng.random(19)).reshape(19, 1).copy()
        before = O.conserved(box, f)
        O.lb_step(box, f)
        assert np.allclose(O.conserved(box, f), before, rtol=0, atol=1e-15)


def test_momentum_conserved_periodic():
    box = Box(8, 6, 5, (PERIODIC, PERIODIC, PERIODIC), (), 0.8)
    f = _random_state(box, 11)
    c0 = O.conserved(box, f)
    for _ in range(30):
        O.lb_step(box, f)
    c1 = O.conserved(box, f)
    assert abs(c1[0] - c0[0]) <= 1e-13 * c0[0]
    assert np.allclose(c1[1:], c0[1:], rtol=0, atol=1e-13 * c0[0])


def test_freeslip_keeps_uniform_tangential_flow():
    box = Box(6, 4, 4, (FREESLIP, PERIODIC, PERIODIC), (), 0.9)
    V = box.nodes
    u = np.zeros((3, V))
    u[1] = 0.03
    f = O.equilibrium_populations(box, np.ones(V), u)
    for _ in range(50):
        O.lb_step(box, f)
    rho, uu = O.fields(box, f)
    assert np.allclose(uu[1], 0.03, rtol=0, atol=1e-14)
    assert np.allclose(rho, 1.0, rtol=0, atol=1e-14)


def test_bounceback_wall_is_no_slip():
    box = Box(8, 4, 4, (PERIODIC, PERIODIC, PERIODIC), ((0, 0, 5, 4, 0, -1),), 0.9)
    V = box.nodes
    u = np.zeros((3, V))
    u[1] = 0.03
    f = O.equilibrium_populations(box, np.ones(V), u)
    for _ in range(200):
        O.lb_step(box, f)
    _, uu = O.fields(box, f)
    fluid = ~O.solid_mask(box)
    assert np.max(np.abs(uu[1][fluid])) < 0.03 * 0.5


def _shear_eigenvalue(tau, k):
    """Largest-|j_y| eigenvalue of the linear one-mode update L = D (I - w (I - E))."""
    c, w, _ = O.lattice()
    cs2 = O.cs2()
    c = c.astype(float)
    E = w[:, None] * (1.0 + (c @ c.T) / cs2)          # linearised equilibrium about rho=1, u=0
    D = np.diag(np.exp(-1j * k * c[:, 0]))             # push streaming of the mode exp(i k x)
    L = D @ (np.eye(19) - (1.0 / tau) * (np.eye(19) - E))
    vals, vecs = np.linalg.eig(L)
    jy = np.abs(c[:, 1] @ vecs)
    jy_total = np.abs(vecs.T @ np.ones(19)) + np.abs(c[:, 0] @ vecs) + np.abs(c[:, 2] @ vecs)
    pick = np.argmax(jy - jy_total)
    return vals[pick]


@pytest.mark.parametrize("tau", [1.0, 0.8, 0.6])
def test_shear_wave_decay_matches_linear_eigenvalue(tau):
    box = Box(32, 2, 2, (PERIODIC, PERIODIC, PERIODIC), (), tau)
    k = 2 * np.pi / 32
    lam = _shear_eigenvalue(tau, k)
    assert abs(lam.imag) < 1e-14
    if tau == 1.0:  # closed form of the same eigenvalue at omega = 1
        assert abs(lam.real - (2 + np.cos(k)) / 3) < 1e-14
    V = box.nodes
    x = np.arange(V) % box.nx
    u = np.zeros((3, V))
    u[1] = 1e-7 * np.sin(k * x)
    f = O.equilibrium_populations(box, np.ones(V), u)
    amps = []
    for _ in range(60):
        O.lb_step(box, f)
        _, uu = O.fields(box, f)
        amps.append(2.0 / V * np.sum(uu[1] * np.sin(k * x)))
    ratios = np.array(amps[31:]) / np.array(amps[30:-1])
    assert np.max(np.abs(ratios - lam.real)) < 1e-8


def test_shear_wave_viscosity_fit():
    """The C1 case: nu fitted over steps 20..100 within 1% of (tau - 1/2)/3."""
    box = Box(32, 32, 32, (PERIODIC, PERIODIC, PERIODIC), (), 1.0)
    rho, u = shear_wave_fields(box, seed=20250101)
    f = O.equilibrium_populations(box, rho, u)
    V = box.nodes
    x = np.arange(V) % box.nx
    k = 2 * np.pi / box.nx
    amps = {}
    for t in range(1, 101):
        O.lb_step(box, f)
        if t >= 20:
            _, uu = O.fields(box, f)
            amps[t] = 2.0 / V * np.sum(uu[1] * np.sin(k * x))
    ts = np.array(sorted(amps))
    slope = np.polyfit(ts, np.log([amps[t] for t in ts]), 1)[0]
    nu = -slope / k ** 2
    assert abs(nu - (1.0 - 0.5) / 3) < 0.01 * (1.0 / 6)
    assert abs(amps[100] / 0.01 - np.exp(-nu * k * k * 100)) < 2e-3


@pytest.mark.parametrize("tau", [1.0, 0.5 + np.sqrt(3.0) / 4.0, 0.7])
def test_poiseuille_bulk_curvature(tau):
    """Walls at x=0 and x=nx-1 (bounce-back), flow along periodic y driven by a
    uniform force entering as S_p = w_p F c_p / cs^2 (the source form of Sec. II).
    The steady bulk profile is parabolic with u'' = -F / (rho nu)."""
    nx = 14
    box = Box(nx, 2, 2, (PERIODIC, PERIODIC, PERIODIC),
              ((0, 0, 5, 4, 0, -1), (nx - 1, nx - 1, 5, 4, 0, -1)), tau)
    V = box.nodes
    c, w, _ = O.lattice()
    F = 1e-6
    S = (w[:, None] * F * c[:, 1:2].astype(float) / O.cs2()) * np.ones((1, V))
    S[:, O.solid_mask(box)] = 0.0
    f = O.equilibrium_populations(box, np.ones(V), np.zeros((3, V)))
    for _ in range(6000):
        O.lb_step(box, f, S)
    rho, u = O.fields(box, f)
    prof = u[1][: nx][1:-1]  # nodes x=1..nx-2 on the row y=z=0
    nu = (tau - 0.5) / 3.0
    curv = prof[2:] - 2 * prof[1:-1] + prof[:-2]
    assert np.allclose(curv, -F / nu, rtol=1e-7, atol=0)
