"""Scalar IFMM: factorisation (Algorithm 1) and solve (Algorithm 2), FP64.

Paper passages followed:
* Section 4.1 (extended sparsification): the dense FMM system is rewritten
  with multipoles y_i = V_i^T x_i and locals z_i as extra unknowns, and the
  equations are reordered so that each cluster's (x_i, z_i) pairs with its
  (P2P, P2M) equations and y_i with its M2L equation.
* Section 4.2 tables (cluster lists; variables x, y, z, r, E; FMM operators
  P2P, P2M, L2P, M2L; IFMM operators P2L, M2P), the equation stacking non-leaf
  particles as children's multipoles, the remark building non-leaf P2P from
  the children's M2L, and the remark listing what is zero initially.
* Section 4.2.2, equations P2P(i,k) and P2M(i,k), Algorithm 1 (elimination
  with compression of fill between well-separated clusters, updating the
  cluster's P2M/L2P, its M2L row and column, and its parent's P2M/L2P) and
  Algorithm 2 (back substitution in reverse order).

Block names used below (level k, clusters i, j):
  P[i,j]  P2P   (n_i x n_j)  j in N_i           row P2P(i), column x_j
  Qm[i,j] M2P   (n_i x r_j)  j in N_i           row P2P(i), column y_j
  L[i,j]  P2L   (r_i x n_j)  j in N_i           row M2L(i), column x_j
  M[i,j]  M2L   (r_i x r_j)  j in N_i u I_i     row M2L(i), column y_j
  U[i] = L2P (n_i x r_i)  column z_i in row P2P(i)
  V[i] = P2M^T (n_i x r_i) row P2M(i) is V_i^T x_i - y_i = 0
  UP[i], VP[i] (r_i x r_parent): the parent's L2P / P2M restricted to child i
  (row M2L(i) carries UP[i] z_parent; y_parent = sum_c VP[c]^T y_c).
Row M2L(i) reads  -z_i + sum_l M[i,l] y_l + sum_j L[i,j] x_j + UP[i] z_par = c_i.

Readings where the paper is silent:
* bases are Chebyshev interpolation orthonormalised exactly by Householder QR
  (A~ unchanged); non-leaf ranks start at min(n_i, p^2);
* elimination order: 9 colours, and inside a level each colour runs three
  phases: eliminate all clusters of the colour, then compute all new bases,
  then apply all basis changes and project the compressed fill;
* pivot block D_i = [[P_ii, U_i], [V_i^T, 0]] factored by LU with partial
  pivoting;
* compression of a non-eliminated cluster q that received fill towards a
  well-separated cluster: new bases from column-pivoted QR of
  [U_q Omega_q^T | row fill] and [V_q Omega'_q^T | column fill], truncated at
  relative tolerance eps, same rank r^ on both sides, r^ <= min(n_q, r_cap);
  Omega_q weights the existing far field: R factor of the QR of the
  transposed M2L row of q joined with the parent chain UP[q] Omega_parent^T
  (precomputed top-down from the assembled operators);
* symmetric kernels: the reordered extended system is symmetric (P2M is the
  transpose of L2P), so the column basis equals the row basis -- only the row
  side is compressed and V^ = U^;
* level transition re-orthonormalises the parent bases by Householder QR.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np
import scipy.linalg as sla

from . import chebyshev as cheb
from . import householder as hh
from .fmm_matrix import diagonal, fmm_apply_offdiag, m2l_cheb
from .geometry import Tree
from .kernels import Kernel


def _z(a, b):
    return np.zeros((a, b))


class IFMM:
    def __init__(self, points, kernel: Kernel, eps: float, leaf_size: int, p: int,
                 diag_mode: str = "rowsum", c0: float = 1.0, r_cap: int | None = None,
                 lo=(0.0, 0.0), size: float = 1.0, symmetric: bool | None = None,
                 diag_values=None):
        """diag_mode "rowsum" (A_ii = c0 + the FMM row sum), "const" (A_ii =
        c0) or "vector" (A_ii = diag_values[i], caller's point order)."""
        self.tree = Tree(points, leaf_size, lo, size)
        self.diag_values = None if diag_values is None else np.asarray(diag_values, dtype=np.float64)[self.tree.perm]
        self.symmetric = (kernel.kind != "callable") if symmetric is None else bool(symmetric)
        self.kernel = kernel
        self.eps = float(eps)
        self.p = int(p)
        self.diag_mode = diag_mode
        self.c0 = float(c0)
        self.r_cap = int(r_cap) if r_cap is not None else 2 * p * p
        self.stats = {"max_rank": 0, "ranks": {}}
        # counted FP64 flops of the factorisation by part (leading terms of the
        # dense primitives: LU (2/3) m^3, triangular solves 2 m^2 w, products
        # 2 m k n, Householder QR 2 m n^2 - (2/3) n^3, pivoted QR and basis
        # formation 4 m n k); counting only, no effect on the arithmetic
        self.work = {"elim": 0.0, "compress": 0.0, "transition": 0.0, "top": 0.0}
        self.assemble()

    # ------------------------------------------------------------------ assembly
    def assemble(self):
        """Orthonormal nested Chebyshev bases, M2L, near field, weights (t_a)."""
        T, p, kap = self.tree, self.p, self.tree.kappa
        pp = p * p
        E = [cheb.transfer(p, c) for c in range(4)]
        self.n = {k: np.zeros(4 ** k, dtype=int) for k in range(2, kap + 1)}
        self.r = {k: np.zeros(4 ** k, dtype=int) for k in range(2, kap + 1)}
        self.U, self.V, self.UP, self.VP = ({k: {} for k in range(2, kap + 1)} for _ in range(4))
        Ru, Rv = {k: {} for k in range(2, kap + 1)}, {k: {} for k in range(2, kap + 1)}
        st, en = T.leaf_start, T.leaf_end
        for m in range(4 ** kap):
            nm = int(en[m] - st[m])
            self.n[kap][m] = nm
            if nm == 0:
                continue
            c, h = T.box(kap, m)
            S = cheb.interp2d(p, c, h, T.leaf_points(m))
            Q, R = hh.qr(S)
            self.U[kap][m], Ru[kap][m] = Q, R
            self.V[kap][m], Rv[kap][m] = Q.copy(), R.copy()
            self.r[kap][m] = Q.shape[1]
        for k in range(kap - 1, 1, -1):
            for m in range(4 ** k):
                su, sv = [], []
                for c in range(4):
                    ch = 4 * m + c
                    if self.r[k + 1][ch] > 0:
                        su.append(Ru[k + 1][ch] @ E[c])
                        sv.append(Rv[k + 1][ch] @ E[c])
                if not su:
                    continue
                Qu, R1 = hh.qr(np.vstack(su))
                Qv, R2 = hh.qr(np.vstack(sv))
                self.n[k][m] = Qu.shape[0]
                self.r[k][m] = Qu.shape[1]
                Ru[k][m], Rv[k][m] = R1, R2
                self.U[k][m], self.V[k][m] = Qu, Qv
                off = 0
                for c in range(4):
                    ch = 4 * m + c
                    rc = self.r[k + 1][ch]
                    if rc > 0:
                        self.UP[k + 1][ch] = Qu[off:off + rc].copy()
                        self.VP[k + 1][ch] = Qv[off:off + rc].copy()
                        off += rc
        # M2L in orthonormal coordinates: M_il = R_i K~_il R'_l^T
        self.M = {k: {} for k in range(2, kap + 1)}
        for k in range(2, kap + 1):
            for i in range(4 ** k):
                if self.r[k][i] == 0:
                    continue
                for l in T.interaction_list(k, i):
                    if self.r[k][l] > 0:
                        self.M[k][(i, l)] = Ru[k][i] @ m2l_cheb(T, self.kernel, p, k, i, l) @ Rv[k][l].T
        # diagonal and leaf near field
        if self.diag_mode == "rowsum":
            rs = fmm_apply_offdiag(T, self.kernel, p, np.ones(T.N))
        else:
            rs = np.zeros(T.N)
        self.d = diagonal(rs, self.diag_mode, self.c0, self.diag_values)
        self.P = {k: {} for k in range(2, kap + 1)}
        for i in range(4 ** kap):
            if self.n[kap][i] == 0:
                continue
            for j in T.neighbours(kap, i):
                if self.n[kap][j] == 0:
                    continue
                blk = self.kernel(T.leaf_points(i), T.leaf_points(j))
                if i == j:
                    blk[np.diag_indices_from(blk)] = self.d[st[i]:en[i]]
                self.P[kap][(i, j)] = blk
        self.Qm = {k: {} for k in range(2, kap + 1)}
        self.L = {k: {} for k in range(2, kap + 1)}
        # far-field weights of parents, top-down
        self.Om, self.Omp = {k: {} for k in range(2, kap + 1)}, {k: {} for k in range(2, kap + 1)}
        for k in range(2, kap):
            for i in range(4 ** k):
                if self.r[k][i] > 0:
                    self.Om[k][i], self.Omp[k][i] = self._weights(k, i)

    def _weights(self, k, i):
        """Omega_i, Omega'_i: R factors of the far-field row / column of i."""
        T, r = self.tree, self.r[k]
        row, col = [], []
        for l in T.interaction_list(k, i):
            if r[l] > 0:
                row.append(self.M[k].get((i, l), _z(r[i], r[l])))
                col.append(self.M[k].get((l, i), _z(r[l], r[i])).T)
        par = i >> 2
        if k > 2 and self.r[k - 1][par] > 0:
            row.append(self.UP[k][i] @ self.Om[k - 1][par].T)
            col.append(self.VP[k][i] @ self.Omp[k - 1][par].T)
        if not row:
            return _z(0, r[i]), _z(0, r[i])
        return hh.r_factor(np.hstack(row).T), hh.r_factor(np.hstack(col).T)

    # ------------------------------------------------------------- factorisation
    def factor(self):
        """Algorithm 1: levels kappa..2, colour batches, then the top solve."""
        T, kap = self.tree, self.tree.kappa
        self.records = {k: [] for k in range(2, kap + 1)}
        self.elim = {k: np.zeros(4 ** k, dtype=bool) for k in range(2, kap + 1)}
        for k in range(kap, 1, -1):
            for batch in T.elimination_order(k):
                fills = []
                for i in batch:
                    if self.n[k][i] > 0:
                        self._eliminate(k, i, fills)
                    else:
                        self.elim[k][i] = True
                if fills:
                    self._compress(k, fills)
            for i in range(4 ** k):
                self.stats["max_rank"] = max(self.stats["max_rank"], int(self.r[k][i]))
            self.stats["ranks"][k] = self.r[k].copy()
            if k > 2:
                self._transition(k)
        # top: level-2 multipoles, dense system of the remaining M2L rows
        self.top_ids = [c for c in range(16) if self.r[2][c] > 0]
        offs = np.cumsum([0] + [self.r[2][c] for c in self.top_ids])
        Mt = np.zeros((offs[-1], offs[-1]))
        for a, ca in enumerate(self.top_ids):
            for b, cb in enumerate(self.top_ids):
                blk = self.M[2].get((ca, cb))
                if blk is not None:
                    Mt[offs[a]:offs[a + 1], offs[b]:offs[b + 1]] = blk
        self.top_offs = offs
        self.top_lu = sla.lu_factor(Mt) if offs[-1] > 0 else None
        self.work["top"] += 2.0 / 3.0 * float(offs[-1]) ** 3
        return self

    def _eliminate(self, k, i, fills):
        """Eliminate (x_i, z_i) with equations P2P(i,k), P2M(i,k)."""
        T = self.tree
        n, r, el = self.n[k], self.r[k], self.elim[k]
        P, Qm, L, M = self.P[k], self.Qm[k], self.L[k], self.M[k]
        ni, ri = int(n[i]), int(r[i])
        nb = [j for j in T.neighbours(k, i) if j != i]
        Qs = [q for q in nb if not el[q] and n[q] > 0]
        Es = [p for p in nb if el[p] and r[p] > 0]
        m = ni + ri
        D = np.zeros((m, m))
        D[:ni, :ni] = P[(i, i)]
        D[:ni, ni:] = self.U[k][i]
        D[ni:, :ni] = self.V[k][i].T
        cols = [("x", q, int(n[q])) for q in Qs] + [("y", p, int(r[p])) for p in Es] + [("y", i, ri)]
        w = sum(c[2] for c in cols)
        B = np.zeros((m, w))
        off = 0
        coloffs = []
        for kind, j, sz in cols:
            if kind == "x":
                B[:ni, off:off + sz] = P[(i, j)]
            elif j != i:
                B[:ni, off:off + sz] = Qm.get((i, j), _z(ni, sz))
            else:
                B[ni:, off:off + sz] = -np.eye(ri)
            coloffs.append(off)
            off += sz
        lu = sla.lu_factor(D)
        X = sla.lu_solve(lu, B)
        Xx, Xz = X[:ni], X[ni:]
        h = sum(int(n[q]) for q in Qs) + sum(int(r[p]) for p in Es)
        self.work["elim"] += 2.0 / 3.0 * m ** 3 + 2.0 * m * m * w + 2.0 * h * ni * w
        rows = [("p2p", q, P[(q, i)]) for q in Qs] + \
               [("m2l", p, L.get((p, i), _z(int(r[p]), ni))) for p in Es]
        for rk, a, Ca in rows:
            G = Ca @ Xx
            for (ck, b, sz), o in zip(cols, coloffs):
                self._add(k, rk, a, ck, b, -G[:, o:o + sz], fills)
        for (ck, b, sz), o in zip(cols, coloffs):
            self._add(k, "m2l", i, ck, b, Xz[:, o:o + sz], fills)
        self.records[k].append(dict(
            i=i, ni=ni, ri=ri, lu=lu, Q=Qs, E=Es,
            Piq=[P[(i, q)].copy() for q in Qs],
            Qip=[Qm.get((i, p), _z(ni, int(r[p]))).copy() for p in Es],
            Pqi=[P[(q, i)].copy() for q in Qs],
            Lpi=[L.get((p, i), _z(int(r[p]), ni)).copy() for p in Es]))
        el[i] = True

    def _add(self, k, rk, a, ck, b, upd, fills):
        """Schur update of block (row unit, column unit); fill between
        well-separated clusters is kept aside for compression."""
        adj = Tree.adjacent(a, b)
        if rk == "p2p" and ck == "x":
            store, tag = self.P[k], "P"
        elif rk == "p2p":
            store, tag = self.Qm[k], "Q"
        elif ck == "x":
            store, tag = self.L[k], "L"
        else:
            store, tag, adj = self.M[k], "M", True
        if adj:
            if (a, b) in store:
                store[(a, b)] = store[(a, b)] + upd
            else:
                store[(a, b)] = upd.copy()
        else:
            fills.append((tag, a, b, upd.copy()))

    def _compress(self, k, fills):
        """Compress fill towards well-separated clusters into new P2M/L2P
        bases and the M2L operators (Algorithm 1, the well-separated cases)."""
        n, r = self.n[k], self.r[k]
        rowf, colf = defaultdict(list), defaultdict(list)
        for tag, a, b, F in fills:
            if tag == "P":
                rowf[a].append(F)
                colf[b].append(F.T)
            elif tag == "Q":
                rowf[a].append(F)
            else:  # "L"
                colf[b].append(F.T)
        touched = sorted(set(rowf) | set(colf))
        Tq, Sq, new = {}, {}, {}
        for q in touched:
            Om, Omp = self._weights(k, q)
            AU = np.hstack([self.U[k][q] @ Om.T] + rowf[q])
            nq, rq = int(n[q]), int(r[q])
            rows_w = sum(int(r[l]) for l in self.tree.interaction_list(k, q)) + rq
            self.work["compress"] += (2.0 * rows_w * rq * rq + 2.0 * nq * rq * Om.shape[0]
                                      + 4.0 * nq * AU.shape[1] * min(nq, self.r_cap))
            kmax = min(int(n[q]), self.r_cap)
            kU, vU, aU = hh.pivoted_qr(AU, self.eps, kmax)
            if self.symmetric:
                rh = min(kU, int(n[q]), self.r_cap)
                Uh = hh.basis_from_reflectors(int(n[q]), vU, aU, rh)
                Vh = Uh
            else:
                AV = np.hstack([self.V[k][q] @ Omp.T] + colf[q])
                kV, vV, aV = hh.pivoted_qr(AV, self.eps, kmax)
                rh = min(max(kU, kV), int(n[q]), self.r_cap)
                Uh = hh.basis_from_reflectors(int(n[q]), vU, aU, rh)
                Vh = hh.basis_from_reflectors(int(n[q]), vV, aV, rh)
            Tq[q] = Uh.T @ self.U[k][q]
            Sq[q] = self.V[k][q].T @ Vh
            new[q] = (Uh, Vh, rh)
            self.work["compress"] += 4.0 * nq * rh * min(nq, self.r_cap) + 2.0 * rh * nq * rq
        M = self.M[k]
        for key in list(M.keys()):
            a, b = key
            if a in Tq or b in Sq:
                blk = M[key]
                if a in Tq:
                    self.work["compress"] += 2.0 * Tq[a].shape[0] * blk.shape[0] * blk.shape[1]
                    blk = Tq[a] @ blk
                if b in Sq:
                    self.work["compress"] += 2.0 * blk.shape[0] * blk.shape[1] * Sq[b].shape[1]
                    blk = blk @ Sq[b]
                M[key] = blk
        for q in touched:
            if q in self.UP[k]:
                self.UP[k][q] = Tq[q] @ self.UP[k][q]
                self.VP[k][q] = Sq[q].T @ self.VP[k][q]
            self.U[k][q], self.V[k][q], r[q] = new[q]
        for tag, a, b, F in fills:
            if tag == "P":
                upd = self.U[k][a].T @ F @ self.V[k][b]
            elif tag == "Q":
                upd = self.U[k][a].T @ F
            else:
                upd = F @ self.V[k][b]
            if (a, b) in M:
                M[(a, b)] = M[(a, b)] + upd
            else:
                M[(a, b)] = upd

    def _transition(self, k):
        """Level k -> k-1: non-leaf particles are the children's multipoles,
        P2P from the children's M2L, parent bases re-orthonormalised."""
        T = self.tree
        kp = k - 1
        rk = self.r[k]
        for P_ in range(4 ** kp):
            ch = [4 * P_ + c for c in range(4) if rk[4 * P_ + c] > 0]
            self.n[kp][P_] = int(sum(rk[c] for c in ch))
        Rt = {}
        for P_ in range(4 ** kp):
            if self.n[kp][P_] == 0:
                rold = self.r[kp][P_]
                Rt[P_] = (_z(0, rold), _z(0, rold))
                self.r[kp][P_] = 0
                continue
            chP = [4 * P_ + c for c in range(4) if rk[4 * P_ + c] > 0]
            for Q_ in T.neighbours(kp, P_):
                if self.n[kp][Q_] == 0:
                    continue
                chQ = [4 * Q_ + c for c in range(4) if rk[4 * Q_ + c] > 0]
                rows = []
                for a in chP:
                    rows.append(np.hstack([self.M[k].get((a, b), _z(rk[a], rk[b])) for b in chQ]))
                self.P[kp][(P_, Q_)] = np.vstack(rows)
            Qu, Ru = hh.qr(np.vstack([self.UP[k][c] for c in chP]))
            Qv, Rv = hh.qr(np.vstack([self.VP[k][c] for c in chP]))
            mq, nq = Qu.shape[0], Ru.shape[1]
            self.work["transition"] += 2.0 * (2.0 * mq * nq * nq - 2.0 / 3.0 * nq ** 3)
            self.U[kp][P_], self.V[kp][P_] = Qu, Qv
            self.r[kp][P_] = Qu.shape[1]
            Rt[P_] = (Ru, Rv)
        # z_P -> Ru z_P and y_P = Rv^T y^_P: M2L(P) row times Ru, column y_P times Rv^T
        for key in list(self.M[kp].keys()):
            a, b = key
            self.M[kp][key] = Rt[a][0] @ self.M[kp][key] @ Rt[b][1].T
        if kp > 2:
            for P_ in list(self.UP[kp].keys()):
                if P_ in Rt:
                    self.UP[kp][P_] = Rt[P_][0] @ self.UP[kp][P_]
                    self.VP[kp][P_] = Rt[P_][1] @ self.VP[kp][P_]

    # --------------------------------------------------------------------- solve
    def solve(self, b):
        """Algorithm 2 with the forward replay of the eliminations on b.
        b: (N,) or (N, nrhs) in the caller's point order."""
        T, kap = self.tree, self.tree.kappa
        b = np.asarray(b, dtype=np.float64)
        squeeze = b.ndim == 1
        Bt = b.reshape(T.N, -1)[T.perm]
        nr = Bt.shape[1]
        st, en = T.leaf_start, T.leaf_end
        bk = {i: Bt[st[i]:en[i]].copy() for i in range(4 ** kap) if self.n[kap][i] > 0}
        snap = {k: {} for k in range(2, kap + 1)}
        cks = {}
        for k in range(kap, 1, -1):
            ck = defaultdict(lambda: None)
            for rec in self.records[k]:
                i, ni, ri = rec["i"], rec["ni"], rec["ri"]
                snap[k][i] = bk[i].copy()
                wv = sla.lu_solve(rec["lu"], np.vstack([bk[i], np.zeros((ri, nr))]))
                wx, wz = wv[:ni], wv[ni:]
                for q, Pqi in zip(rec["Q"], rec["Pqi"]):
                    bk[q] = bk[q] - Pqi @ wx
                for p_, Lpi in zip(rec["E"], rec["Lpi"]):
                    ck[p_] = (ck[p_] if ck[p_] is not None else np.zeros((Lpi.shape[0], nr))) - Lpi @ wx
                ck[i] = (ck[i] if ck[i] is not None else np.zeros((ri, nr))) + wz
            cks[k] = ck
            if k > 2:
                bk = {}
                for P_ in range(4 ** (k - 1)):
                    if self.n[k - 1][P_] > 0:
                        parts = [ck[4 * P_ + c] if ck[4 * P_ + c] is not None
                                 else np.zeros((self.r[k][4 * P_ + c], nr))
                                 for c in range(4) if self.r[k][4 * P_ + c] > 0]
                        bk[P_] = np.vstack(parts)
        ck = cks[2]
        rhs = np.vstack([ck[c] if ck[c] is not None else np.zeros((self.r[2][c], nr))
                         for c in self.top_ids]) if self.top_ids else np.zeros((0, nr))
        ytop = sla.lu_solve(self.top_lu, rhs) if self.top_lu is not None else rhs
        y = {c: ytop[self.top_offs[a]:self.top_offs[a + 1]] for a, c in enumerate(self.top_ids)}
        for k in range(2, kap + 1):
            x = {}
            for rec in reversed(self.records[k]):
                i, ni, ri = rec["i"], rec["ni"], rec["ri"]
                top = snap[k][i].copy()
                for q, Piq in zip(rec["Q"], rec["Piq"]):
                    top -= Piq @ x[q]
                for p_, Qip in zip(rec["E"], rec["Qip"]):
                    top -= Qip @ y[p_]
                sol = sla.lu_solve(rec["lu"], np.vstack([top, y.get(i, np.zeros((ri, nr)))]))
                x[i] = sol[:ni]
            if k < kap:
                y = {}
                for P_, xv in x.items():
                    off = 0
                    for c in range(4):
                        ch = 4 * P_ + c
                        rc = self.r[k + 1][ch]
                        if rc > 0:
                            y[ch] = xv[off:off + rc]
                            off += rc
        Xt = np.zeros((T.N, nr))
        for i, xv in x.items():
            Xt[st[i]:en[i]] = xv
        out = np.empty_like(Xt)
        out[T.perm] = Xt
        return out[:, 0] if squeeze else out

    # ------------------------------------------------------- FMM product, refine
    def apply(self, x):
        """A~ x in the caller's order (FMM passes + diagonal)."""
        T = self.tree
        x = np.asarray(x, dtype=np.float64)
        X = x.reshape(T.N, -1)[T.perm]
        Y = fmm_apply_offdiag(T, self.kernel, self.p, X) + self.d[:, None] * X
        out = np.empty_like(Y)
        out[T.perm] = Y
        return out.reshape(x.shape)

    def solve_refined(self, b, tol: float, maxit: int = 30):
        """FP64 iterative refinement x <- x + solve(b - A~ x) until the
        relative residual (per column) is <= tol."""
        b = np.asarray(b, dtype=np.float64)
        x = self.solve(b)
        hist = []
        nb = np.linalg.norm(b.reshape(b.shape[0], -1), axis=0)
        for _ in range(maxit):
            res = b - self.apply(x)
            rel = np.linalg.norm(res.reshape(b.shape[0], -1), axis=0) / nb
            hist.append(float(rel.max()))
            if rel.max() <= tol:
                break
            x = x + self.solve(res)
        return x, hist
