"""Pins of the oracle's bead dynamics (Eq. force, LJ potential, drag, Sec. II).

  * WCA: the LJ form 4 eps[(s/r)^12-(s/r)^6] truncated at 2^(1/6) s and shifted
    by eps: known values, zero force at the cutoff;
  * forces are minus the gradient of the potential energy written from the
    potentials themselves (central finite differences);
  * wall distance: the analytic slab-minus-pore decomposition against a brute
    force minimum over the solid unit cubes;
  * drag with frozen fluid velocity: v - u decays by exactly (1 - gamma h) per
    substep (kick-drift);
  * random force: the discrete Ornstein-Uhlenbeck stationary variance
    <v^2> = (kT/m) 2/(2 - gamma h), which fixes the noise amplitude;
  * harmonic bond + kick-drift: the relative coordinate obeys the three-term
    recurrence of the discrete oscillator, cos(theta) = 1 - (omega h)^2 / 2,
    omega^2 = 2k/m.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from workloads.configs import FREESLIP, PERIODIC, Box, MDParams

RC = 2 ** (1 / 6)


def _pair_energy(md, r):
    box = Box(64, 64, 64, (PERIODIC,) * 3)
    pts = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
    return O.potential_energy(box, md, [1, 1], pts)


def test_wca_values():
    md = MDParams(eps=1.0, sigma=1.8)
    assert abs(_pair_energy(md, 1.8) - 1.0) < 1e-14            # V(sigma) = eps after the shift
    assert abs(_pair_energy(md, RC * 1.8)) < 1e-14               # zero at the cutoff
    assert _pair_energy(md, RC * 1.8 + 1e-9) == 0.0
    r = 1.5
    lj = 4 * ((1.8 / r) ** 12 - (1.8 / r) ** 6) + 1.0
    assert abs(_pair_energy(md, r) - lj) < 1e-12 * lj
    # bonded neighbours do not feel WCA: one chain of two beads at r0 has zero energy
    box = Box(64, 64, 64, (PERIODIC,) * 3)
    pts = np.array([[10.0, 10.0, 10.0], [11.2, 10.0, 10.0]])
    assert O.potential_energy(box, md, [2], pts) < 1e-20  # only the (rounded) bond term


def _fd_check(box, md, chains, r, h=1e-6):
    F, _ = O.conservative_forces(box, md, chains, r)
    Ffd = np.zeros_like(r)
    for i, a in itertools.product(range(len(r)), range(3)):
        rp, rm = r.copy(), r.copy()
        rp[i, a] += h
        rm[i, a] -= h
        Ffd[i, a] = -(O.potential_energy(box, md, chains, rp) -
                      O.potential_energy(box, md, chains, rm)) / (2 * h)
    scale = max(1.0, np.max(np.abs(F)))
    assert np.max(np.abs(F - Ffd)) < 1e-5 * scale
    return F


def test_forces_are_minus_gradient_near_pore():
    box = Box(24, 16, 16, (FREESLIP,) * 3, ((10, 12, 7, 9, 7, 9),), 1.0)
    md = MDParams()
    rng = np.random.default_rng(7)
    # a chain threading the pore, one bead close to the pore edge, one crowder near a face
    r = np.array([[8.4, 8.0, 8.1], [9.6, 8.1, 8.0], [10.8, 7.3, 8.2], [12.0, 8.0, 8.6],
                  [13.1, 8.4, 8.0], [14.2, 9.0, 8.5], [0.3, 3.0, 14.1]])
    r += 1e-3 * rng.random(r.shape)
    F = _fd_check(box, md, [6, 1], r)
    assert np.max(np.abs(F)) > 1e-3  # the configuration actually exercises the forces


def test_forces_minus_gradient_overlapping_pairs_periodic():
    box = Box(10, 10, 10, (PERIODIC,) * 3)
    md = MDParams()
    # pairs across the periodic boundary (minimum image) and a stretched bond
    r = np.array([[0.2, 5.0, 5.0], [9.1, 5.3, 4.8], [1.0, 6.2, 5.0], [5.0, 5.0, 9.7],
                  [5.2, 5.4, 0.9]])
    F = _fd_check(box, md, [3, 2], r)
    assert np.max(np.abs(F)) > 1e-2
    assert np.allclose(F.sum(axis=0), 0.0, atol=1e-10)  # Newton's third law


def _brute_wall_distance(box, p):
    best = np.inf
    for (x0, x1, y0, y1, z0, z1) in box.walls:
        for x in range(x0, x1 + 1):
            for y in range(box.ny):
                for z in range(box.nz):
                    if y0 <= y1 and z0 <= z1 and y0 <= y <= y1 and z0 <= z <= z1:
                        continue
                    lo = np.array([x, y, z]) - 0.5
                    d = p - np.clip(p, lo, lo + 1.0)
                    best = min(best, np.linalg.norm(d))
    return best


def test_wall_distance_against_solid_cubes():
    box = Box(20, 12, 12, (FREESLIP,) * 3, ((8, 10, 5, 7, 5, 7), (15, 15, 2, 3, 8, 9)), 1.0)
    rng = np.random.default_rng(3)
    # points inside the box away from the faces (the wall boxes extend past the faces)
    pts = np.column_stack([rng.uniform(4, 19, 300), rng.uniform(0.6, 10.4, 300),
                           rng.uniform(0.6, 10.4, 300)])
    for p in pts:
        d, dv = O.wall_distance(box, p)
        bf = _brute_wall_distance(box, p)
        assert abs(d - bf) < 1e-12
        assert abs(np.linalg.norm(dv) - d) < 1e-12


def test_drag_relaxation_exact():
    box = Box(16, 16, 16, (PERIODIC,) * 3)
    md = MDParams(M=8, kT=0.0, gamma=0.3)
    r = np.array([[3.0, 4.0, 5.0]])
    v = np.array([[0.02, -0.01, 0.005]])
    u = np.array([[0.004, 0.001, -0.002]])
    v0 = v.copy()
    h = 1.0 / md.M
    for step in range(5):
        fbar, flags = O.md_substeps(box, md, [1], r, v, u, step, 99)
        assert flags == 0
    expect = u + (1 - md.gamma * h) ** (5 * md.M) * (v0 - u)
    assert np.allclose(v, expect, rtol=0, atol=1e-16)


def test_fluctuation_dissipation_discrete_ou():
    box = Box(40, 40, 40, (PERIODIC,) * 3)
    md = MDParams(M=2, gamma=0.5, kT=1e-4, eps=0.0)
    rng = np.random.default_rng(1)
    n = 64
    r = np.column_stack([rng.uniform(0, 40, n) for _ in range(3)])
    v = np.zeros((n, 3))
    u = np.zeros((n, 3))
    acc, cnt, mean = 0.0, 0, 0.0
    for step in range(12000):
        O.md_substeps(box, md, [1] * n, r, v, u, step, 12345)
        if step >= 100:
            acc += np.sum(v * v)
            mean += np.sum(v)
            cnt += v.size
    h = 1.0 / md.M
    expect = md.kT / md.mass * 2.0 / (2.0 - md.gamma * h)
    assert abs(acc / cnt / expect - 1.0) < 6e-3
    assert abs(mean / cnt) < 6.0 * np.sqrt(expect / cnt * 4)


def test_harmonic_dimer_discrete_frequency():
    box = Box(32, 32, 32, (PERIODIC,) * 3)
    md = MDParams(M=20, gamma=0.0, kT=0.0, k_bond=100.0, r0=1.2)
    r = np.array([[10.0, 10.0, 10.0], [11.23, 10.0, 10.0]])
    v = np.zeros((2, 3))
    u = np.zeros((2, 3))
    e = [r[1, 0] - r[0, 0] - md.r0]
    com0 = r.mean(axis=0)
    for step in range(200):
        O.md_substeps(box, md, [2], r, v, u, step, 1)
        e.append(r[1, 0] - r[0, 0] - md.r0)
    e = np.array(e)
    h = 1.0 / md.M
    omega = np.sqrt(2 * md.k_bond / md.mass)
    theta = np.arccos(1 - (omega * h) ** 2 / 2)
    two_cos = 2 * np.cos(md.M * theta)  # one LB step = M substeps of the linear map
    resid = e[2:] - two_cos * e[1:-1] + e[:-2]
    assert np.max(np.abs(resid)) < 1e-12
    assert np.allclose(r.mean(axis=0), com0, atol=1e-13)
    assert np.allclose(r[:, 1:], 10.0, atol=1e-14)


def test_drive_only_inside_pore():
    box = Box(24, 16, 16, (FREESLIP,) * 3, ((10, 12, 7, 9, 7, 9),), 1.0)
    md = MDParams(M=1, kT=0.0, gamma=0.0, eps_w=0.0, f_drive=0.02)
    inside = np.array([[11.2, 8.3, 7.6]])
    outside = np.array([[5.0, 8.0, 8.0]])
    for r, expect in ((inside, 0.02), (outside, 0.0)):
        v = np.zeros((1, 3))
        O.md_substeps(box, md, [1], r.copy(), v, np.zeros((1, 3)), 0, 0)
        assert np.allclose(v, [[expect, 0, 0]], atol=1e-17)


def test_random_force_uses_philox_stream():
    """F_r = A c with A = sqrt(24 m gamma kT / h) and c the centred top-24-bit uniform
    of Philox outputs for counter (bead, step, substep, 1) and key (seed lo, seed hi)."""
    box = Box(16, 16, 16, (PERIODIC,) * 3)
    md = MDParams(M=1, gamma=0.2, kT=1e-3, eps=0.0)
    seed = (7 << 32) | 99
    r = np.array([[3.0, 3.0, 3.0], [9.0, 9.0, 9.0]])
    v = np.zeros((2, 3))
    fbar, _ = O.md_substeps(box, md, [1, 1], r, v, np.zeros((2, 3)), 41, seed)
    A = np.sqrt(24 * md.mass * md.gamma * md.kT * md.M)
    for i in range(2):
        out = O.philox([i, 41, 0, 1], [99, 7])
        c = np.array([np.int32(np.uint32(o & 0xFFFFFF00).view(np.int32)) for o in out[:3]],
                     dtype=np.float64) / 2 ** 32
        assert np.allclose(fbar[i], A * c, rtol=1e-15, atol=0)
