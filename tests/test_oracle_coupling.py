"""Pins of the oracle's LB <-> bead coupling (Sec. II, steps 1-4, S_p eq., Fig. 1).

  * S_p: sum_p S_p = 0 and sum_p S_p c_p = -Fbar (closed form; the fluid receives
    the reaction of the frictional + random force);
  * total momentum of fluid + beads is conserved by a coupled step in a periodic
    box without walls or drive (bonds and WCA obey Newton's third law, and the
    exchanged force is the same average on both sides);
  * nearest-grid-point interpolation picks floor(x + 1/2) and returns that node's
    velocity, zero on solid nodes;
  * the coupled step equals LB-only followed by the streamed source (linearity of
    Eq. lbe in S_p), which is how the GPU library exposes the two halves.
"""
import numpy as np
import pytest

from oracle import oracle as O
from workloads.configs import FREESLIP, PERIODIC, Box, MDParams
from workloads.generate import grow_chain, random_small_flow


def test_source_moments():
    box = Box(4, 4, 4, (PERIODIC,) * 3)
    c, _, _ = O.lattice()
    fbar = np.array([[0.013, -0.021, 0.007]])
    node = np.array([21])
    S = O.spread(box, node, fbar)
    col = S[:, 21]
    assert abs(col.sum()) < 1e-17
    assert np.allclose(col @ c.astype(float), -fbar[0], atol=1e-17)
    assert np.count_nonzero(S[:, np.arange(box.nodes) != 21]) == 0


def test_ngp_interpolation():
    box = Box(8, 8, 8, (FREESLIP, FREESLIP, PERIODIC), ((5, 5, 2, 3, 2, 3),))
    V = box.nodes
    rng = np.random.default_rng(0)
    u = 0.01 * rng.random((3, V))
    f = O.equilibrium_populations(box, np.ones(V), u)
    r = np.array([[2.5, 3.49, 4.51],     # -> (3, 3, 5): x tie rounds up
                  [0.1, 7.4, -0.4],      # -> (0, 7, 0): periodic z wraps -0.4 -> 0
                  [3.0, 3.0, 7.6],       # -> (3, 3, 0): 8 wraps to 0 on periodic z
                  [5.2, 0.9, 0.8],       # -> (5, 1, 1): solid node of the wall
                  [-3.0, 9.7, 2.0]])     # outside on free-slip axes: clamped to (0, 7, 2)
    ui, node = O.interp(box, f, r)
    expect_nodes = [(3, 3, 5), (0, 7, 0), (3, 3, 0), None, (0, 7, 2)]
    for i, g in enumerate(expect_nodes):
        if g is None:
            assert node[i] == -1 and np.all(ui[i] == 0)
            continue
        k = g[0] + 8 * (g[1] + 8 * g[2])
        assert node[i] == k
        assert np.allclose(ui[i], u[:, k], atol=1e-15)


@pytest.mark.parametrize("model", ["harmonic", "rigid"])
def test_total_momentum_conserved_by_coupled_step(model):
    """Fluid plus bead momentum is conserved by coupled steps, with harmonic bonds and
    with the paper's rigid bonds and angular term (constraint reactions are internal)."""
    box = Box(16, 16, 16, (PERIODIC,) * 3, (), 0.9)
    if model == "harmonic":
        md = MDParams(M=10, kT=1e-4, gamma=0.2, f_drive=0.0)
    else:
        md = MDParams(M=5, kT=1e-4, gamma=0.2, f_drive=0.0, rigid=1, kappa_phi=0.02, eps=2e-3)
    rng = np.random.default_rng(5)
    chain = grow_chain(box, md, 12, rng, cis_only=False)
    crowd = grow_chain(box, md, 3, rng, existing=chain, cis_only=False)
    r0 = np.concatenate([chain, crowd])
    rho, u = random_small_flow(box, 9, du=0.01)
    f0 = O.equilibrium_populations(box, rho, u)
    v0 = 0.01 * rng.standard_normal(r0.shape)
    if md.rigid:  # start with velocities that respect the constraints
        r0, v0, _ = O.shake_rattle(box, md, [12, 3], r0, r0 + v0 / md.M, 1.0 / md.M)
    sim = O.Sim(box, md, [12, 3], f0, r0, v0, seed=77)

    def total():
        c = O.conserved(box, sim.f)
        return c[1:] + md.mass * sim.v.sum(axis=0), c[0]

    p0, m0 = total()
    for _ in range(15):
        sim.step()
    p1, m1 = total()
    assert abs(m1 - m0) < 1e-13 * m0
    # rigid bonds rebuild velocities from positions, (r' - r)/h, which loses about
    # ulp(r)/h ~ 1e-14 per bead and substep; the sum stays at that rounding level
    assert np.allclose(p1, p0, rtol=0, atol=1e-13 if model == "harmonic" else 1e-12)
    assert np.max(np.abs(sim.fbar)) > 1e-5  # the exchange actually happened
    assert sim.flags == 0


def test_coupled_step_equals_lb_then_streamed_source():
    box = Box(12, 10, 10, (FREESLIP,) * 3, ((5, 6, 4, 6, 4, 6),), 1.0)
    md = MDParams(M=5)
    rng = np.random.default_rng(2)
    r = np.array([[4.2, 5.1, 5.0], [3.1, 5.6, 5.2], [2.4, 4.6, 4.4]])
    rho, u = random_small_flow(box, 4, du=0.01)
    f = O.equilibrium_populations(box, rho, u)
    sim = O.Sim(box, md, [3], f, r, seed=5, step0=17)
    sim.step()
    # same thing, halves separately
    r2, v2 = r.copy(), np.zeros((3, 3))
    f2 = f.copy()
    ui, node = O.interp(box, f2, r2)
    fbar, _ = O.md_substeps(box, md, [3], r2, v2, ui, 17, 5)
    O.lb_step(box, f2)
    O.add_streamed_source(box, f2, O.spread(box, node, fbar))
    assert np.allclose(f2, sim.f, rtol=0, atol=1e-15)
    assert np.allclose(r2, sim.r, atol=0) and np.allclose(v2, sim.v, atol=0)
    del rng


def test_translocation_count():
    box = Box(20, 8, 8, (FREESLIP,) * 3, ((8, 10, 3, 5, 3, 5),))
    r = np.array([[8.9, 4, 4], [9.0, 4, 4], [9.1, 4, 4], [15.0, 4, 4]])
    nt, com = O.transloc(box, r)
    assert nt == 2  # strictly past the wall's mid-plane x = 9
    assert np.allclose(com, r.mean(axis=0))
