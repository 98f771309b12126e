"""Pins of the oracle's D3Q19 table, equilibrium and Philox against closed forms.

Sec. II of arXiv:0710.1272 uses the standard 19-speed lattice with weights
"normalized to unity" and the second-order equilibrium (f_eq eq.).  The table
identities below are those every D3Q19 model must satisfy for the equilibrium
moments to be the Euler ones; the equilibrium moments are checked against their
closed forms (Sec. II, Eqs. dens, vel, pre).
"""
import itertools
import os

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def test_table_identities():
    c, w, opp = O.lattice()
    cs2 = O.cs2()
    c = c.astype(float)
    assert len(w) == 19
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w @ c, 0.0, atol=1e-16)
    assert np.allclose(np.einsum("p,pa,pb->ab", w, c, c), cs2 * np.eye(3), atol=1e-15)
    assert np.allclose(np.einsum("p,pa,pb,pc->abc", w, c, c, c), 0.0, atol=1e-16)
    d = np.eye(3)
    iso4 = cs2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) +
                       np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("p,pa,pb,pc,pd->abcd", w, c, c, c, c), iso4, atol=1e-15)
    # every speed appears once, the rest speed first, |c|^2 <= 2
    assert len({tuple(v) for v in c.astype(int)}) == 19
    assert tuple(c[0]) == (0, 0, 0)
    assert all(np.sum(v * v) <= 2 for v in c)
    for p in range(19):
        assert np.array_equal(c[opp[p]], -c[p])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_moments_closed_form(seed):
    rng = np.random.default_rng(seed)
    c, _, _ = O.lattice()
    c = c.astype(float)
    cs2 = O.cs2()
    rho = 0.8 + 0.4 * rng.random()
    u = 0.1 * (2 * rng.random(3) - 1)
    f = O.feq(rho, u)
    assert abs(f.sum() - rho) < 1e-14
    assert np.allclose(f @ c, rho * u, atol=1e-15)
    P = np.einsum("p,pa,pb->ab", f, c, c)
    assert np.allclose(P, rho * cs2 * np.eye(3) + rho * np.outer(u, u), atol=1e-15)


def test_equilibrium_at_rest_is_weights():
    _, w, _ = O.lattice()
    assert np.allclose(O.feq(1.3, [0, 0, 0]), 1.3 * w, atol=1e-16)


def _kats():
    out = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            out.append((v[:4], v[4:6], v[6:]))
    return out


@pytest.mark.parametrize("ctr,key,expect", _kats())
def test_philox_known_answers(ctr, key, expect):
    assert list(O.philox(ctr, key)) == expect


def test_philox_counter_sensitivity():
    base = O.philox([5, 7, 3, 1], [11, 13])
    for i, j in itertools.product(range(4), range(0, 32, 7)):
        ctr = [5, 7, 3, 1]
        ctr[i] ^= 1 << j
        assert not np.array_equal(O.philox(ctr, [11, 13]), base)
