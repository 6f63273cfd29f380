"""Pins for oracle/ifmm.py (Algorithms 1 and 2 with on-the-fly compression).

What fixes the scalar IFMM, independently of its own code:
* eps = 0 with no rank cap makes every compression lossless, so the solution
  must equal the dense LU solve of the FMM matrix A~ (brute force) to
  round-off -- this exercises every elimination, fill, basis change, level
  transition and the back substitution;
* the extended sparse system of Section 4.1 (multipoles and locals as extra
  unknowns), assembled densely from the oracle's operators and solved by
  LAPACK, has the same particle unknowns as the dense solve of A~;
* at eps > 0 the relative residual against A~ is below 10 eps, and FP64
  refinement with the FMM product converges to round-off;
* linearity / permutation invariances and the rank bound of the paper's
  numerical section (ranks independent of N);
* a mistake planted in the oracle (wrong Schur sign, a skipped basis change)
  breaks the eps = 0 pin, showing the pin is sensitive to it.
"""
import numpy as np
import pytest

import workloads
from oracle import fmm_matrix as fm
from oracle.ifmm import IFMM
from oracle.kernels import Kernel


def _dense_solution(o: IFMM, b):
    T = o.tree
    A = fm.dense_matrix(T, o.kernel, o.p, o.diag_mode, o.c0)
    xt = np.linalg.solve(A, b.reshape(T.N, -1)[T.perm])
    x = np.empty_like(xt)
    x[T.perm] = xt
    return x.reshape(b.shape), A


def _c1(n=2048, eps=1e-6, r_cap=None):
    pts = workloads.points_for("c1_invr_2k", n)
    return IFMM(pts, Kernel("inv_r"), eps, 32, 4, "rowsum", 1.0, r_cap=r_cap)


def test_eps0_equals_dense_solve_inv_r():
    o = _c1(eps=0.0, r_cap=10 ** 6).factor()
    b = workloads.rhs_for("c1_invr_2k")[:, 0]
    x = o.solve(b)
    xd, _ = _dense_solution(o, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-12


def test_eps0_equals_dense_solve_exp_uniform_three_levels():
    pts = workloads.uniform(1500, 77)
    o = IFMM(pts, Kernel("exp", 0.1), 0.0, 8, 4, "const", 1.01, r_cap=10 ** 6).factor()
    assert o.tree.kappa == 4
    b = workloads.rhs(1500, 2, 78)
    x = o.solve(b)
    xd, A = _dense_solution(o, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10 * np.linalg.cond(A) ** 0.5


def _extended_system(o: IFMM, b):
    """Dense extended system of Section 4.1 built from the assembled operators."""
    T, kap = o.tree, o.tree.kappa
    N = T.N
    off = N
    yid, zid = {}, {}
    for k in range(kap, 1, -1):
        for i in range(4 ** k):
            if o.r[k][i] > 0:
                yid[(k, i)] = off
                zid[(k, i)] = off + o.r[k][i]
                off += 2 * o.r[k][i]
    Mx = np.zeros((off, off))
    rhs = np.zeros(off)
    st, en = T.leaf_start, T.leaf_end
    bt = b[T.perm]
    row = 0
    for i in range(4 ** kap):  # P2P(i) at the leaves
        if o.n[kap][i] == 0:
            continue
        s = slice(st[i], en[i])
        for j in T.neighbours(kap, i):
            if o.n[kap][j]:
                Mx[s, st[j]:en[j]] = o.P[kap][(i, j)]
        z = zid[(kap, i)]
        Mx[s, z:z + o.r[kap][i]] = o.U[kap][i]
        rhs[s] = bt[s]
    row = N
    for k in range(kap, 1, -1):
        for i in range(4 ** k):
            r = o.r[k][i]
            if r == 0:
                continue
            y, z = yid[(k, i)], zid[(k, i)]
            # P2M(i): V_i^T x_i - y_i = 0 (non-leaf particles are children's multipoles)
            if k == kap:
                Mx[row:row + r, st[i]:en[i]] = o.V[k][i].T
            else:
                for c in range(4):
                    ch = 4 * i + c
                    if o.r[k + 1][ch]:
                        yc = yid[(k + 1, ch)]
                        Mx[row:row + r, yc:yc + o.r[k + 1][ch]] = o.VP[k + 1][ch].T
            Mx[row:row + r, y:y + r] = -np.eye(r)
            row += r
            # M2L(i): -z_i + sum M_il y_l + L2L from the parent = 0
            Mx[row:row + r, z:z + r] = -np.eye(r)
            for l in T.interaction_list(k, i):
                if o.r[k][l]:
                    yl = yid[(k, l)]
                    Mx[row:row + r, yl:yl + o.r[k][l]] = o.M[k][(i, l)]
            if k > 2 and o.r[k - 1][i >> 2]:
                zp = zid[(k - 1, i >> 2)]
                Mx[row:row + r, zp:zp + o.r[k - 1][i >> 2]] = o.UP[k][i]
            row += r
    assert row == off
    sol = np.linalg.solve(Mx, rhs)
    x = np.empty(N)
    x[T.perm] = sol[:N]
    return x, off


def test_extended_sparse_system_has_the_dense_solution():
    o = _c1(n=1024, eps=1e-6)
    b = workloads.rhs(1024, 1, 5)[:, 0]
    x, M = _extended_system(o, b)
    xd, _ = _dense_solution(o, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-12
    # M = N + 2 sum_i r_i (a multipole and a local per cluster); the paper's
    # M ~ 3N (Section 3) -- the ratio depends on leaf size against p^2
    assert M == 1024 + 2 * sum(int(o.r[k].sum()) for k in o.r)
    assert 2.0 * 1024 < M < 4.0 * 1024


def test_c1_residual_below_10_eps_and_refinement():
    o = _c1().factor()
    b = workloads.rhs_for("c1_invr_2k")[:, 0]
    x = o.solve(b)
    res = np.linalg.norm(b - o.apply(x)) / np.linalg.norm(b)
    assert res < 10 * 1e-6
    xr, hist = o.solve_refined(b, 1e-13)
    assert hist[-1] < 1e-13 and len(hist) <= 4
    xd, _ = _dense_solution(o, b)
    assert np.linalg.norm(xr - xd) / np.linalg.norm(xd) < 1e-12


def test_exp_kernel_residual_and_refinement():
    pts = workloads.uniform(2048, 1003)
    o = IFMM(pts, Kernel("exp", 0.1), 1e-8, 32, 4, "const", 1.01).factor()
    b = workloads.rhs(2048, 1, 2003)[:, 0]
    xr, hist = o.solve_refined(b, 1e-12)
    assert hist[0] < 1e-4 and hist[-1] < 1e-12


def test_linearity_multirhs_and_point_permutation():
    o = _c1().factor()
    rng = np.random.default_rng(9)
    B = rng.standard_normal((2048, 3))
    X = o.solve(B)
    for j in range(3):
        assert np.allclose(X[:, j], o.solve(B[:, j]), rtol=0, atol=1e-13 * np.abs(X).max())
    assert np.allclose(o.solve(2.5 * B), 2.5 * X, atol=1e-13 * np.abs(X).max())
    # permuting points and right-hand side permutes the solution
    pts = workloads.points_for("c1_invr_2k")
    perm = rng.permutation(2048)
    o2 = IFMM(pts[perm], Kernel("inv_r"), 1e-6, 32, 4, "rowsum", 1.0).factor()
    X2 = o2.solve(B[perm])
    assert np.linalg.norm(X2 - X[perm]) / np.linalg.norm(X) < 1e-6


def test_max_rank_bounded_as_n_grows():
    ranks = []
    for n in (1024, 4096):
        pts = workloads.jittered_grid(n, 3)
        o = IFMM(pts, Kernel("inv_r"), 1e-6, 16, 4, "rowsum", 1.0, r_cap=10 ** 6).factor()
        ranks.append(o.stats["max_rank"])
    assert ranks[1] <= ranks[0] + 8 and ranks[1] < 4 * 4 * 4


def test_planted_mistakes_break_the_eps0_pin(monkeypatch):
    b = workloads.rhs_for("c1_invr_2k", n=512)[:, 0]

    def err():
        pts = workloads.points_for("c1_invr_2k", 512)
        o = IFMM(pts, Kernel("inv_r"), 0.0, 8, 3, "rowsum", 1.0, r_cap=10 ** 6).factor()
        assert o.tree.kappa == 3
        x = o.solve(b)
        xd, _ = _dense_solution(o, b)
        return np.linalg.norm(x - xd) / np.linalg.norm(xd)

    assert err() < 1e-12
    orig_add = IFMM._add

    def wrong_sign(self, k, rk, a, ck, b_, upd, fills):
        return orig_add(self, k, rk, a, ck, b_, -upd if rk == "m2l" else upd, fills)

    monkeypatch.setattr(IFMM, "_add", wrong_sign)
    assert err() > 1e-6
    monkeypatch.setattr(IFMM, "_add", orig_add)

    orig_compress = IFMM._compress

    def skip_parent_update(self, k, fills):
        saved = {q: (self.UP[k][q].copy(), self.VP[k][q].copy()) for q in self.UP[k]}
        orig_compress(self, k, fills)
        for q, (u, v) in saved.items():  # undo the parent L2P/P2M update
            if self.UP[k][q].shape == u.shape:
                self.UP[k][q], self.VP[k][q] = u, v

    monkeypatch.setattr(IFMM, "_compress", skip_parent_update)
    assert err() > 1e-6


def test_symmetric_mode_agrees_with_two_sided_compression():
    # for a symmetric kernel the row and column compressions coincide, so the
    # one-sided (symmetric) variant must reproduce the general one
    pts = workloads.points_for("c1_invr_2k", 1024)
    b = workloads.rhs(1024, 1, 4)[:, 0]
    xs = IFMM(pts, Kernel("inv_r"), 1e-7, 16, 4, "rowsum", 1.0, symmetric=True).factor().solve(b)
    og = IFMM(pts, Kernel("inv_r"), 1e-7, 16, 4, "rowsum", 1.0, symmetric=False).factor()
    xg = og.solve(b)
    assert np.linalg.norm(xs - xg) / np.linalg.norm(xg) < 1e-7


def test_eps0_with_a_diagonal_vector_equals_dense_solve():
    # A_ii given per point (caller's order): the lossless factor solves the
    # dense FMM matrix with that diagonal
    pts = workloads.uniform(1500, 77)
    d = 1.01 + np.random.default_rng(79).uniform(size=1500)
    o = IFMM(pts, Kernel("exp", 0.1), 0.0, 8, 3, "vector", 0.0, r_cap=10 ** 6, diag_values=d).factor()
    A = fm.dense_matrix(o.tree, o.kernel, o.p, "vector", 0.0, d[o.tree.perm])
    assert np.array_equal(np.diag(A), d[o.tree.perm])
    b = workloads.rhs(1500, 1, 80)[:, 0]
    xt = np.linalg.solve(A, b[o.tree.perm])
    xd = np.empty_like(xt)
    xd[o.tree.perm] = xt
    x = o.solve(b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-11
