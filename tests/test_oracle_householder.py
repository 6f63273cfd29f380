"""Pins for oracle/householder.py against LAPACK (numpy) and against matrices
of known rank."""
import numpy as np
import pytest

from oracle import householder as hh


@pytest.mark.parametrize("shape", [(30, 12), (12, 30), (17, 17), (1, 5), (5, 1)])
def test_qr_matches_lapack_up_to_signs(shape):
    A = np.random.default_rng(sum(shape)).standard_normal(shape)
    Q, R = hh.qr(A)
    K = min(shape)
    assert Q.shape == (shape[0], K) and R.shape == (K, shape[1])
    assert np.allclose(Q.T @ Q, np.eye(K), atol=1e-13)
    assert np.allclose(Q @ R, A, atol=1e-13)
    assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)
    Q2, R2 = np.linalg.qr(A)
    s = np.sign(np.diag(R2))
    assert np.allclose(R, R2 * s[:, None], atol=1e-12)


def test_qr_of_rank_deficient_and_zero_columns():
    A = np.zeros((6, 4))
    A[:, 1] = 1.0
    Q, R = hh.qr(A)
    assert np.allclose(Q @ R, A, atol=1e-14) and np.allclose(Q.T @ Q, np.eye(4), atol=1e-14)


@pytest.mark.parametrize("rank", [1, 5, 11])
def test_pivoted_qr_finds_the_rank_and_spans_the_range(rank):
    rng = np.random.default_rng(rank)
    n, m = 40, 60
    A = rng.standard_normal((n, rank)) @ rng.standard_normal((rank, m))
    k, vs, al = hh.pivoted_qr(A, 1e-10, n)
    assert k == rank
    Q = hh.basis_from_reflectors(n, vs, al, k)
    assert np.allclose(Q.T @ Q, np.eye(k), atol=1e-13)
    Us = np.linalg.svd(A)[0][:, :rank]
    assert np.allclose(Q @ Q.T, Us @ Us.T, atol=1e-10)


def test_pivoted_qr_first_pivot_is_largest_column_and_threshold_is_relative():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((20, 8)) * np.array([1, 2, 3, 100, 5, 6, 7, 8.0])
    k, vs, al = hh.pivoted_qr(A, 0.0, 20)
    assert abs(abs(al[0]) - np.linalg.norm(A[:, 3])) < 1e-12 * np.linalg.norm(A[:, 3])
    # scaling the matrix does not change the rank decision
    B = rng.standard_normal((30, 4)) @ np.diag([1, 1e-3, 1e-7, 1e-12]) @ rng.standard_normal((4, 30))
    for s in (1e-8, 1.0, 1e8):
        assert hh.pivoted_qr(s * B, 1e-9, 30)[0] == 3

