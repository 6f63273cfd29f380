"""Chebyshev interpolation operators (the low-rank bases of the FMM matrix).

Paper, Section 5: the nested low-rank form of well-separated blocks comes from
Chebyshev interpolation with a fixed number of nodes per dimension (8 in the
paper's runs; the order p is an input here).  The nodes and the Lagrange
basis are the textbook ones (first-kind nodes, product basis in 2D):

    t_m = cos((2m - 1) pi / (2p)),  m = 1..p
    l_m(s) = prod_{k != m} (s - t_k) / (t_m - t_k)
    2D basis index (mx, my) -> mx * p + my,  value l_mx(s_x) * l_my(s_y)

with box-local coordinates s = (x - centre) / half_width.
"""
from __future__ import annotations

import numpy as np


def nodes(p: int) -> np.ndarray:
    m = np.arange(1, p + 1)
    return np.cos((2 * m - 1) * np.pi / (2 * p))


def lagrange(p: int, s: np.ndarray) -> np.ndarray:
    """(len(s), p) matrix of l_m(s)."""
    t = nodes(p)
    s = np.asarray(s, dtype=np.float64)
    out = np.ones((s.shape[0], p))
    for m in range(p):
        for k in range(p):
            if k != m:
                out[:, m] *= (s - t[k]) / (t[m] - t[k])
    return out


def interp2d(p: int, centre, half: float, pts: np.ndarray) -> np.ndarray:
    """S[a, mx*p+my] = l_mx(sx_a) l_my(sy_a): potential at the points from the
    p x p node values of the box (L2P), and transposed, P2M."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 2)
    lx = lagrange(p, (pts[:, 0] - centre[0]) / half)
    ly = lagrange(p, (pts[:, 1] - centre[1]) / half)
    return (lx[:, :, None] * ly[:, None, :]).reshape(pts.shape[0], p * p)


def box_nodes(p: int, centre, half: float) -> np.ndarray:
    """(p*p, 2) node coordinates, index mx*p+my."""
    t = nodes(p)
    gx, gy = np.meshgrid(centre[0] + half * t, centre[1] + half * t, indexing="ij")
    return np.stack([gx.ravel(), gy.ravel()], axis=1)


def transfer(p: int, c: int) -> np.ndarray:
    """E_c: parent Lagrange basis evaluated at the nodes of child quadrant c
    (c & 1 = x half, c >> 1 = y half).  Rows: child nodes; columns: parent
    nodes.  The parent basis restricted to the child box equals S_child @ E_c
    exactly, which is what makes the bases nested (M2M = E_c^T, L2L = E_c)."""
    dx = 0.5 if (c & 1) else -0.5
    dy = 0.5 if (c >> 1) else -0.5
    child = box_nodes(p, (dx, dy), 0.5)
    return interp2d(p, (0.0, 0.0), 1.0, child)
