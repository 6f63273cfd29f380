"""The FMM matrix A~ that the IFMM factors, written out from its definition.

Paper, Section 2.2 (FMM / H^2 matrices with strong admissibility; the 1D
two-level example table and the 2D figure): blocks between neighbouring leaf
clusters are the exact kernel; every other block is U K~ V^T with nested
bases, taken at the unique level where the two ancestor clusters are well
separated while their parents are neighbours (i.e. where one lies in the
other's interaction list).  The bases are the Chebyshev ones of Section 5.

Diagonal (readings where the paper is silent):
* "rowsum": A_ii = c0 + sum_{j != i} A~_ij  (diagonally dominant 1/r systems;
  the sum runs over the FMM matrix so that oracle and solver factor the same
  matrix);
* "const":  A_ii = c0  (exp(-r/ell) + sigma^2 I: c0 = K(0) + sigma^2; the
  paper's benchmark equation of Section 5 has c0 = 1);
* "vector": A_ii = a given vector (tree order here).

Everything here is in tree order (the order of ``Tree.points``).
"""
from __future__ import annotations

import numpy as np

from . import chebyshev as cheb
from .geometry import Tree


def _chain(tree: Tree, p: int, leaf: int, k: int, cache: dict) -> np.ndarray:
    """C_leaf^(k): ancestor-at-level-k Chebyshev node values -> leaf points."""
    key = (leaf, k)
    if key in cache:
        return cache[key]
    if k == tree.kappa:
        c, h = tree.box(k, leaf)
        out = cheb.interp2d(p, c, h, tree.leaf_points(leaf))
    else:
        anc_child = leaf >> (2 * (tree.kappa - k - 1))
        out = _chain(tree, p, leaf, k + 1, cache) @ cheb.transfer(p, anc_child & 3)
    cache[key] = out
    return out


def m2l_cheb(tree: Tree, kernel, p: int, k: int, i: int, l: int) -> np.ndarray:
    """K~_il: kernel between the Chebyshev nodes of clusters i and l."""
    ci, hi = tree.box(k, i)
    cl, hl = tree.box(k, l)
    return kernel(cheb.box_nodes(p, ci, hi), cheb.box_nodes(p, cl, hl))


def separation_level(tree: Tree, a: int, b: int) -> int:
    """Level at which the ancestors of leaves a, b stop being neighbours."""
    for k in range(2, tree.kappa + 1):
        s = 2 * (tree.kappa - k)
        if not Tree.adjacent(a >> s, b >> s):
            return k
    return -1


def dense_offdiag(tree: Tree, kernel, p: int) -> np.ndarray:
    """A~ with a zero diagonal, dense (tree order).  O(N^2 p^2)."""
    N = tree.N
    A = np.zeros((N, N))
    nleaf = 4 ** tree.kappa
    cache: dict = {}
    st, en = tree.leaf_start, tree.leaf_end
    for a in range(nleaf):
        if en[a] == st[a]:
            continue
        for b in range(nleaf):
            if en[b] == st[b]:
                continue
            if Tree.adjacent(a, b):
                blk = kernel(tree.leaf_points(a), tree.leaf_points(b))
                if a == b:
                    np.fill_diagonal(blk, 0.0)
            else:
                k = separation_level(tree, a, b)
                s = 2 * (tree.kappa - k)
                blk = (_chain(tree, p, a, k, cache)
                       @ m2l_cheb(tree, kernel, p, k, a >> s, b >> s)
                       @ _chain(tree, p, b, k, cache).T)
            A[st[a]:en[a], st[b]:en[b]] = blk
    return A


def diagonal(offdiag_rowsum: np.ndarray, mode: str, c0: float, values=None) -> np.ndarray:
    if mode == "rowsum":
        return c0 + offdiag_rowsum
    if mode == "const":
        return np.full_like(offdiag_rowsum, c0)
    if mode == "vector":
        return np.array(values, dtype=np.float64, copy=True)
    raise ValueError(mode)


def dense_matrix(tree: Tree, kernel, p: int, mode: str, c0: float, values=None) -> np.ndarray:
    """values: the diagonal of mode "vector" in tree order."""
    A = dense_offdiag(tree, kernel, p)
    d = diagonal(A.sum(axis=1), mode, c0, values)
    A[np.diag_indices_from(A)] = d
    return A


def exact_offdiag(tree: Tree, kernel) -> np.ndarray:
    """The true kernel matrix A (zero diagonal), for reporting only."""
    A = kernel(tree.points, tree.points)
    np.fill_diagonal(A, 0.0)
    return A


def fmm_apply_offdiag(tree: Tree, kernel, p: int, x: np.ndarray) -> np.ndarray:
    """A~ (zero diagonal) times x by the FMM passes: P2M, M2M, M2L, L2L, L2P
    plus direct neighbour sums (Section 4.2, table of FMM operators)."""
    x = np.asarray(x, dtype=np.float64)
    squeeze = x.ndim == 1
    X = x.reshape(tree.N, -1)
    kap = tree.kappa
    E = [cheb.transfer(p, c) for c in range(4)]
    st, en = tree.leaf_start, tree.leaf_end
    S = {}
    w = {kap: {}}
    for m in range(4 ** kap):
        if en[m] > st[m]:
            c, h = tree.box(kap, m)
            S[m] = cheb.interp2d(p, c, h, tree.leaf_points(m))
            w[kap][m] = S[m].T @ X[st[m]:en[m]]
    for k in range(kap - 1, 1, -1):
        w[k] = {}
        for m in range(4 ** k):
            acc = None
            for c in range(4):
                ch = w[k + 1].get(4 * m + c)
                if ch is not None:
                    t = E[c].T @ ch
                    acc = t if acc is None else acc + t
            if acc is not None:
                w[k][m] = acc
    g = {}
    for k in range(2, kap + 1):
        g[k] = {}
        for m in range(4 ** k):
            acc = np.zeros((p * p, X.shape[1]))
            for l in tree.interaction_list(k, m):
                if l in w[k]:
                    acc += m2l_cheb(tree, kernel, p, k, m, l) @ w[k][l]
            if k > 2:
                acc += E[m & 3] @ g[k - 1][m >> 2]
            g[k][m] = acc
    Y = np.zeros_like(X)
    for m in range(4 ** kap):
        if en[m] == st[m]:
            continue
        acc = S[m] @ g[kap][m]
        for j in tree.neighbours(kap, m):
            if en[j] == st[j]:
                continue
            blk = kernel(tree.leaf_points(m), tree.leaf_points(j))
            if j == m:
                np.fill_diagonal(blk, 0.0)
            acc = acc + blk @ X[st[j]:en[j]]
        Y[st[m]:en[m]] = acc
    return Y.reshape(x.shape) if not squeeze else Y[:, 0]
