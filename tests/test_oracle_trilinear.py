"""Pins of the oracle's trilinear coupling stencil (the flagged variant of steps 1 and 3 of
Sec. II: velocity interpolated from, and reaction spread back to, the 8 surrounding nodes).

  * a multilinear velocity field (a + b x + c y z + d x y z) is interpolated exactly;
  * a bead on a node sees that node alone, as the nearest-node stencil does;
  * the spread puts -Fbar on the lattice with its first moment at the bead: sum_x x m(x) =
    -Fbar r (trilinear weights reproduce linear functions), and sum_p S_p = 0 at every node;
  * interpolation and spreading are adjoint: for any node velocity field u(x),
    Fbar . u_interp(r) = -sum_x u(x) . m(x);
  * a coupled step conserves fluid + bead momentum in a periodic box, also where the stencil
    wraps; near a free-slip face the stencil folds onto the face node and still sums to one.
"""
import numpy as np

from oracle import oracle as O
from workloads.configs import FREESLIP, PERIODIC, Box, MDParams
from workloads.generate import grow_chain, random_small_flow

BOX = Box(16, 14, 12, (PERIODIC,) * 3, (), 1.0)


def _grid(box):
    V = box.nodes
    k = np.arange(V)
    return np.stack([k % box.nx, (k // box.nx) % box.ny, k // (box.nx * box.ny)]).astype(float)


def _momentum_density(box, S):
    c, _, _ = O.lattice()
    return S.T @ c.astype(float)  # [V][3]


def test_multilinear_field_is_interpolated_exactly():
    X = _grid(BOX)
    u = np.stack([1e-3 + 2e-4 * X[0] - 1e-5 * X[1] * X[2],
                  -5e-4 + 3e-6 * X[0] * X[1] * X[2],
                  2e-4 * X[2] - 1e-4 * X[1]])
    f = O.equilibrium_populations(BOX, np.ones(BOX.nodes), u)
    rng = np.random.default_rng(1)
    r = np.column_stack([rng.uniform(1, 13, 20), rng.uniform(1, 11, 20), rng.uniform(1, 9, 20)])
    ui = O.interp_trilinear(BOX, f, r)
    x, y, z = r.T
    exact = np.stack([1e-3 + 2e-4 * x - 1e-5 * y * z, -5e-4 + 3e-6 * x * y * z, 2e-4 * z - 1e-4 * y]).T
    assert np.max(np.abs(ui - exact)) < 1e-15


def test_bead_on_a_node_sees_that_node():
    rho, u = random_small_flow(BOX, 3, du=0.01)
    f = O.equilibrium_populations(BOX, rho, u)
    r = np.array([[3.0, 7.0, 5.0], [15.0, 0.0, 11.0]])
    ut = O.interp_trilinear(BOX, f, r)
    un, _ = O.interp(BOX, f, r)
    assert np.max(np.abs(ut - un)) < 1e-16


def test_spread_moments_and_first_moment():
    fbar = np.array([[0.013, -0.021, 0.007], [-0.002, 0.004, 0.011]])
    r = np.array([[4.3, 6.8, 2.25], [15.6, 13.2, 11.7]])   # the second wraps on every axis
    X = _grid(BOX)
    for i in range(2):
        S = O.spread_trilinear(BOX, r[i:i + 1], fbar[i:i + 1])
        assert np.max(np.abs(S.sum(axis=0))) < 1e-17
        m = _momentum_density(BOX, S)
        assert np.allclose(m.sum(axis=0), -fbar[i], atol=1e-17)
        assert np.count_nonzero(np.any(m != 0, axis=1)) == 8
        if i == 0:  # first moment (no wrap): sum_x x m_a(x) = -Fbar_a r
            assert np.allclose(X @ m, -np.outer(r[i], fbar[i]), atol=1e-15)


def test_interpolation_and_spreading_are_adjoint():
    box = Box(12, 10, 10, (FREESLIP, PERIODIC, FREESLIP), ((5, 6, 3, 5, 3, 6),), 1.0)
    rho, u = random_small_flow(box, 4, du=0.01)
    f = O.equilibrium_populations(box, rho, u)
    rho_n, u_n = O.fields(box, f)  # node velocities, 0 on solid nodes
    rng = np.random.default_rng(7)
    r = np.column_stack([rng.uniform(-0.5, 11.5, 30), rng.uniform(0, 10, 30), rng.uniform(-0.5, 9.5, 30)])
    fbar = 0.01 * rng.standard_normal((30, 3))
    ui = O.interp_trilinear(box, f, r)
    for i in range(30):
        m = _momentum_density(box, O.spread_trilinear(box, r[i:i + 1], fbar[i:i + 1]))
        lhs = fbar[i] @ ui[i]
        rhs = -np.sum(u_n.T * m)
        assert abs(lhs - rhs) < 1e-16, (i, lhs, rhs)


def test_stencil_folds_at_free_slip_faces():
    box = Box(10, 10, 10, (FREESLIP,) * 3, (), 1.0)
    fbar = np.array([[0.01, 0.02, -0.03]])
    r = np.array([[-0.3, 4.5, 9.4]])  # within half a node of the x = -1/2 and z = 9.5 faces
    m = _momentum_density(box, O.spread_trilinear(box, r, fbar))
    assert np.allclose(m.sum(axis=0), -fbar[0], atol=1e-17)
    X = _grid(box)
    touched = X[:, np.any(m != 0, axis=1)]
    assert set(touched[0]) == {0.0} and set(touched[2]) == {9.0}


def test_coupled_steps_conserve_momentum_with_the_trilinear_stencil():
    box = Box(16, 16, 16, (PERIODIC,) * 3, (), 0.9)
    md = MDParams(M=10, kT=1e-4, gamma=0.2, f_drive=0.0, stencil=1)
    rng = np.random.default_rng(5)
    r0 = grow_chain(box, md, 12, rng, cis_only=False) + np.array([7.0, 0.0, 0.0])  # crosses the x wrap
    rho, u = random_small_flow(box, 9, du=0.01)
    f0 = O.equilibrium_populations(box, rho, u)
    v0 = 0.01 * rng.standard_normal(r0.shape)
    sim = O.Sim(box, md, [12], f0, r0, v0, seed=77)

    def total():
        c = O.conserved(box, sim.f)
        return c[1:] + md.mass * sim.v.sum(axis=0), c[0]

    p0, m0 = total()
    for _ in range(15):
        sim.step()
    p1, m1 = total()
    assert abs(m1 - m0) < 1e-13 * m0
    assert np.allclose(p1, p0, rtol=0, atol=1e-13)
    assert np.max(np.abs(sim.fbar)) > 1e-5 and sim.flags == 0
    # and it differs from the nearest-node coupling
    sim_n = O.Sim(box, MDParams(M=10, kT=1e-4, gamma=0.2, f_drive=0.0), [12], f0, r0, v0, seed=77)
    sim_n.step(15)
    assert np.max(np.abs(sim_n.r - sim.r)) > 1e-6
