"""Pins of the oracle's thermal source F_p (the fluctuating lattice Boltzmann equation
that Sec. II adopts from Adhikari et al. without writing it out).

What fixes the answer, independently of how the noise is drawn:
  * the collision conserves density and momentum at every node, noise included;
  * fluctuation-dissipation: populations fluctuating with the equilibrium covariance
    <df_p df_q> = mu rho w_p delta_pq (mu = kT / c_s^2, independent nodes) keep that
    covariance through one collision and streaming, for any relaxation time; the
    boundary rules (periodic wrap, specular faces, bounce-back) only permute populations
    of equal weight and keep it too;
  * equipartition: started from a fluid at rest, the fluid heats up to <u_a^2> = kT/rho
    per node and component and <(rho - rho0)^2> = rho kT / c_s^2, whatever the
    relaxation time.
A mistake in the amplitude (mu, the 1 - gamma^2 factor, the weights) or in the
projection that keeps the conserved moments out of the noise moves one of these.
"""
import numpy as np
import pytest

from oracle import oracle as O
from workloads.configs import FREESLIP, PERIODIC, Box

KT = 1e-4
CS2 = 1.0 / 3.0


def _box(n, tau, kT=KT, walls=(), bc=(PERIODIC,) * 3):
    return Box(n, n, n, bc, walls, tau, 1.0, kT)


def _rest(box):
    V = box.nodes
    return O.equilibrium_populations(box, np.full(V, box.rho0), np.zeros((3, V)))


def _equilibrium_fluctuations(box, seed):
    """Populations w_p rho0 + df_p with df Gaussian of covariance mu rho0 w_p delta_pq,
    independent at every fluid node (numpy's generator, not the oracle's)."""
    _, w, _ = O.lattice()
    rng = np.random.default_rng(seed)
    V = box.nodes
    mu = box.fluid_kT / CS2
    f = w[:, None] * box.rho0 + np.sqrt(mu * box.rho0 * w)[:, None] * rng.standard_normal((19, V))
    f[:, O.solid_mask(box)] = 0.0
    return f


def test_thermal_collision_conserves_mass_and_momentum():
    box = _box(10, 0.8)
    f = _equilibrium_fluctuations(box, 1)
    c, _, _ = O.lattice()
    m0 = f.sum()
    p0 = (c.T.astype(float) @ f).sum(axis=1)
    for step in range(5):
        O.lb_step(box, f, step=step, seed=7)
    assert abs(f.sum() - m0) < 1e-12 * m0
    assert np.max(np.abs((c.T.astype(float) @ f).sum(axis=1) - p0)) < 1e-13


def test_zero_temperature_is_the_deterministic_step():
    box_hot = _box(8, 0.9, kT=0.0)
    box_det = Box(8, 8, 8, (PERIODIC,) * 3, (), 0.9, 1.0)
    f1 = _equilibrium_fluctuations(_box(8, 0.9), 2)
    f2 = f1.copy()
    O.lb_step(box_hot, f1, step=3, seed=5)
    O.lb_step(box_det, f2)
    assert np.array_equal(f1, f2)


def test_noise_depends_on_step_and_seed_only_through_philox():
    box = _box(6, 1.0)
    f0 = _rest(box)
    a, b, c_ = f0.copy(), f0.copy(), f0.copy()
    O.lb_step(box, a, step=11, seed=3)
    O.lb_step(box, b, step=11, seed=3)
    O.lb_step(box, c_, step=12, seed=3)
    assert np.array_equal(a, b)
    assert not np.allclose(a, c_)


@pytest.mark.parametrize("tau", [1.0, 0.8, 2.0])
@pytest.mark.parametrize("walls", [False, True], ids=["periodic", "pore_wall"])
def test_one_step_keeps_the_equilibrium_covariance(tau, walls):
    if walls:
        box = Box(24, 24, 24, (FREESLIP,) * 3, ((10, 12, 10, 12, 10, 12),), tau, 1.0, KT)
    else:
        box = _box(24, tau)
    _, w, _ = O.lattice()
    fluid = ~O.solid_mask(box)
    f = _equilibrium_fluctuations(box, 11)
    O.lb_step(box, f, step=0, seed=21)
    d = f[:, fluid] - w[:, None] * box.rho0
    n = d.shape[1]
    cov = d @ d.T / n
    target = (KT / CS2) * box.rho0 * w
    se = np.sqrt(2.0 / n) * target  # standard error of a sample variance
    assert np.all(np.abs(np.diag(cov) - target) < 5 * se), np.diag(cov) / target
    off = cov - np.diag(np.diag(cov))
    scale = np.sqrt(np.outer(target, target) / n)
    assert np.all(np.abs(off) < 5 * scale)


@pytest.mark.parametrize("tau", [0.8, 1.0, 1.5])
def test_fluid_at_rest_heats_up_to_equipartition(tau):
    box = _box(16, tau)
    f = _rest(box)
    V = box.nodes
    burn, samples, every = 300, 24, 25
    for step in range(burn):
        O.lb_step(box, f, step=step, seed=99)
    u2, dr2 = [], []
    step = burn
    for _ in range(samples):
        for _k in range(every):
            O.lb_step(box, f, step=step, seed=99)
            step += 1
        rho, u = O.fields(box, f)
        u2.append(np.mean(u * u, axis=1))
        dr2.append(np.mean((rho - box.rho0) ** 2))
    u2 = np.array(u2)
    # total mass and momentum are fixed, which removes one of the V modes
    want_u2 = KT / box.rho0 * (1 - 1 / V)
    want_dr2 = box.rho0 * KT / CS2 * (1 - 1 / V)
    got_u2 = u2.mean()
    got_dr2 = np.mean(dr2)
    assert abs(got_u2 / want_u2 - 1) < 0.04, (got_u2, want_u2)
    assert np.all(np.abs(u2.mean(axis=0) / want_u2 - 1) < 0.06)
    assert abs(got_dr2 / want_dr2 - 1) < 0.04, (got_dr2, want_dr2)
