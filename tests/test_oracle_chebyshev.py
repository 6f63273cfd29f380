"""Pins for oracle/chebyshev.py against textbook facts about Chebyshev
interpolation (Section 5 uses Chebyshev interpolation for the nested bases)."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import chebyshev as cheb


@pytest.mark.parametrize("p", [2, 4, 6, 8])
def test_nodes_are_roots_of_T_p(p):
    t = cheb.nodes(p)
    coef = np.zeros(p + 1)
    coef[p] = 1.0
    assert np.max(np.abs(npcheb.chebval(t, coef))) < 1e-13
    assert len(np.unique(np.round(t, 12))) == p and np.all(np.abs(t) < 1)


@pytest.mark.parametrize("p", [3, 4, 6])
def test_lagrange_is_cardinal_and_partition_of_unity(p):
    t = cheb.nodes(p)
    assert np.allclose(cheb.lagrange(p, t), np.eye(p), atol=1e-13)
    s = np.linspace(-1, 1, 37)
    assert np.allclose(cheb.lagrange(p, s).sum(axis=1), 1.0, atol=1e-13)


@pytest.mark.parametrize("p", [3, 4, 6])
def test_interpolation_reproduces_polynomials_of_degree_below_p(p):
    rng = np.random.default_rng(p)
    C = rng.standard_normal((p, p))  # f(x,y) = sum C_ab x^a y^b, degree < p per variable

    def f(P):
        return sum(C[a, b] * P[:, 0] ** a * P[:, 1] ** b for a in range(p) for b in range(p))

    centre, half = (0.3, -0.2), 0.7
    nodes = cheb.box_nodes(p, centre, half)
    pts = np.column_stack([centre[0] + half * rng.uniform(-1, 1, 50),
                           centre[1] + half * rng.uniform(-1, 1, 50)])
    S = cheb.interp2d(p, centre, half, pts)
    assert np.allclose(S @ f(nodes), f(pts), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("p", [4, 6])
def test_nested_transfer_equals_direct_parent_interpolation(p):
    rng = np.random.default_rng(1)
    for c in range(4):
        dx = 0.5 if c & 1 else -0.5
        dy = 0.5 if c >> 1 else -0.5
        pts = np.column_stack([dx + 0.5 * rng.uniform(-1, 1, 40), dy + 0.5 * rng.uniform(-1, 1, 40)])
        direct = cheb.interp2d(p, (0.0, 0.0), 1.0, pts)
        nested = cheb.interp2d(p, (dx, dy), 0.5, pts) @ cheb.transfer(p, c)
        assert np.allclose(direct, nested, atol=1e-12)
