"""Pins for oracle/fmm_matrix.py: the FMM matrix A~ (Section 2.2) and its
matrix-vector product, against the exact kernel and exact identities."""
import numpy as np
import pytest

import workloads
from oracle import fmm_matrix as fm
from oracle.geometry import Tree
from oracle.kernels import Kernel


def _tree(n=1024, leaf=16, seed=3):
    return Tree(workloads.uniform(n, seed), leaf)


def test_polynomial_kernel_is_reproduced_exactly():
    # K(x, y) = (1 + x.y)^2 has degree 2 per coordinate in x and in y, so
    # p = 3 Chebyshev interpolation on both sides is exact: A~ == A.
    K = Kernel("callable", fn=lambda a, b: (1.0 + a @ b.T) ** 2)
    T = _tree()
    A = fm.dense_offdiag(T, K, 3)
    E = fm.exact_offdiag(T, K)
    assert np.max(np.abs(A - E)) < 1e-12 * np.max(np.abs(E))


def test_near_blocks_exact_and_far_blocks_converge_with_p():
    K = Kernel("inv_r")
    T = _tree(512, 8, 4)
    E = fm.exact_offdiag(T, K)
    errs = []
    for p in (3, 4, 6):
        A = fm.dense_offdiag(T, K, p)
        near = np.zeros_like(A, dtype=bool)
        st, en = T.leaf_start, T.leaf_end
        for a in range(4 ** T.kappa):
            for b in T.neighbours(T.kappa, a):
                near[st[a]:en[a], st[b]:en[b]] = True
        assert np.array_equal(A[near], E[near])
        errs.append(np.max(np.abs(A[~near] - E[~near]) / np.abs(E[~near])))
    # Chebyshev error decreases geometrically in p for well-separated boxes
    assert errs[0] < 5e-2 and errs[1] < errs[0] / 2 and errs[2] < errs[1] / 4


@pytest.mark.parametrize("kind", ["inv_r", "exp"])
def test_fmm_product_equals_dense_fmm_matrix(kind):
    K = Kernel(kind, 0.1)
    T = _tree(1500, 16, 7)
    A = fm.dense_offdiag(T, K, 4)
    x = np.random.default_rng(0).standard_normal((T.N, 2))
    y = fm.fmm_apply_offdiag(T, K, 4, x)
    assert np.max(np.abs(y - A @ x)) < 1e-12 * np.max(np.abs(A @ x))


def test_fmm_matrix_symmetric_for_symmetric_kernel():
    K = Kernel("exp", 0.2)
    T = _tree(700, 16, 9)
    A = fm.dense_offdiag(T, K, 4)
    assert np.max(np.abs(A - A.T)) < 1e-14 * np.max(np.abs(A))


def test_rowsum_diagonal_makes_the_matrix_diagonally_dominant():
    K = Kernel("inv_r")
    T = _tree(800, 16, 2)
    A = fm.dense_matrix(T, K, 4, "rowsum", 1.0)
    off = A - np.diag(np.diag(A))
    assert np.allclose(np.diag(A), 1.0 + off.sum(axis=1))
    assert np.all(np.diag(A) - np.abs(off).sum(axis=1) > 0.999)
    C = fm.dense_matrix(T, K, 4, "const", 2.5)
    assert np.all(np.diag(C) == 2.5)
