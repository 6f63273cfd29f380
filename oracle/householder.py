"""Plain Householder QR, with and without column pivoting (FP64, numpy).

Conventions (shared as mathematics, not as code, with the GPU kernels):
* reflector of x: alpha = -sign(x_0) ||x|| (sign(0) = +1), v = x - alpha e_0,
  H = I - 2 v v^T / (v^T v), so H x = alpha e_0; a zero column gives H = I;
* Q and R are sign-normalised so that R_jj >= 0 (column j of Q flipped
  together with row j of R when alpha_j < 0);
* column pivoting (Businger-Golub): at step j take the remaining column of
  largest norm (first one on ties); the number of steps whose pivot norm is
  > eps * (first pivot norm) is the numerical rank at relative tolerance eps.
"""
from __future__ import annotations

import numpy as np


def _reflector(x: np.ndarray):
    nrm = np.linalg.norm(x)
    if nrm == 0.0:
        return None, 0.0
    alpha = -nrm if x[0] >= 0 else nrm
    v = x.copy()
    v[0] -= alpha
    v /= np.linalg.norm(v)
    return v, alpha


def qr(A: np.ndarray):
    """Thin QR: A (n x m) = Q (n x K) R (K x m), K = min(n, m), R_jj >= 0."""
    A = np.array(A, dtype=np.float64, copy=True)
    n, m = A.shape
    K = min(n, m)
    vs = []
    for j in range(K):
        v, alpha = _reflector(A[j:, j])
        vs.append(v)
        if v is not None:
            A[j:, j:] -= 2.0 * np.outer(v, v @ A[j:, j:])
    R = np.triu(A[:K, :])
    Q = np.eye(n, K)
    for j in range(K - 1, -1, -1):
        v = vs[j]
        if v is not None:
            Q[j:, :] -= 2.0 * np.outer(v, v @ Q[j:, :])
    sg = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * sg[None, :], R * sg[:, None]


def r_factor(A: np.ndarray) -> np.ndarray:
    """R of the thin QR of A (K x m, R_jj >= 0)."""
    return qr(A)[1]


def pivoted_qr(A: np.ndarray, eps: float, kmax: int):
    """Column-pivoted Householder QR run for kmax steps (capped at min(n, m)).

    Returns (rank, reflectors, alphas): rank = number of steps with pivot norm
    > eps * first pivot norm."""
    A = np.array(A, dtype=np.float64, copy=True)
    n, m = A.shape
    K = min(n, m, kmax)
    vs, alphas = [], []
    rank = 0
    first = None
    counting = True
    for j in range(K):
        norms = np.linalg.norm(A[j:, j:], axis=0)
        c = j + int(np.argmax(norms))
        piv = norms[c - j]
        if first is None:
            first = piv
        if counting and first > 0.0 and piv > eps * first:
            rank = j + 1
        else:
            counting = False
        if c != j:
            A[:, [j, c]] = A[:, [c, j]]
        v, alpha = _reflector(A[j:, j])
        vs.append(v)
        alphas.append(alpha)
        if v is not None:
            A[j:, j:] -= 2.0 * np.outer(v, v @ A[j:, j:])
    return rank, vs, alphas


def basis_from_reflectors(n: int, vs, alphas, r: int) -> np.ndarray:
    """First r columns of H_0 H_1 ... H_{K-1} (n x r), sign-normalised."""
    Q = np.eye(n, r)
    K = min(len(vs), r)
    for j in range(K - 1, -1, -1):
        v = vs[j]
        if v is not None:
            Q[j:, :] -= 2.0 * np.outer(v, v @ Q[j:, :])
    for j in range(K):
        if alphas[j] < 0:
            Q[:, j] = -Q[:, j]
    return Q

