// Internal interface between the host orchestrator (ifmm_host.hip) and the
// device kernels (ifmm_linalg.hip, ifmm_fmm.hip).  Matrices are column-major.
// Every batched kernel reads an array of descriptors planned on the host;
// an entry whose sizes are zero is a no-op.
//
// Scalar types: the factor's blocks are FP64 or FP32 (the mixed-precision
// factor); pivot inverses, the top system, the FMM product and all solution
// vectors are FP64.  A descriptor records the scalar type of each operand in
// `ty`, set by its constructor from the pointer types it is given, and a
// launch runs the kernel instantiation for that type combination (all
// descriptors of one launch share it).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace ifmm {

constexpr int kMaxRank = 128;   // largest multipole/local rank supported
constexpr int kMaxP = 8;        // largest Chebyshev order per dimension

// 0 for double, 1 for float.
template <class T>
constexpr int tcode() {
  static_assert(std::is_same<T, double>::value || std::is_same<T, float>::value, "FP64 or FP32 only");
  return std::is_same<T, float>::value ? 1 : 0;
}
// Keeps a parameter out of template argument deduction.
template <class X>
struct nodeduce {
  using type = X;
};

// C = alpha * op(A) op(B) + beta * C; beta == 0 never reads C.
// ty: bit 0 A is FP32, bit 1 B is FP32, bit 2 C is FP32.  The products are
// accumulated in FP64 when A or B is FP64, else in FP32.
struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  int M, N, K;
  int lda, ldb, ldc;
  int opA, opB;  // 0: as stored, 1: transposed
  double alpha, beta;
  int ty;
  GemmDesc() = default;
  template <class TA, class TB, class TC>
  __host__ GemmDesc(const TA* a, const TB* b, TC* c, int M_, int N_, int K_, int lda_, int ldb_, int ldc_,
                    int opA_, int opB_, double al, double be)
      : A(a), B(b), C(c), M(M_), N(N_), K(K_), lda(lda_), ldb(ldb_), ldc(ldc_), opA(opA_), opB(opB_),
        alpha(al), beta(be), ty(tcode<TA>() | tcode<TB>() << 1 | tcode<TC>() << 2) {}
};

// C = alpha * op(A) + beta * C (M x N); beta == 0 never reads C; A null
// reads as zero.  ty: bit 0 A is FP32, bit 1 C is FP32.
struct AddDesc {
  const void* A;
  void* C;
  int M, N, lda, ldc, trans;
  double alpha, beta;
  int ty;
  AddDesc() = default;
  template <class TA, class TC>
  __host__ AddDesc(const TA* a, TC* c, int M_, int N_, int lda_, int ldc_, int tr, double al, double be)
      : A(a), C(c), M(M_), N(N_), lda(lda_), ldc(ldc_), trans(tr), alpha(al), beta(be),
        ty(tcode<TA>() | tcode<TC>() << 1) {}
  template <class TC>
  __host__ AddDesc(std::nullptr_t, TC* c, int M_, int N_, int lda_, int ldc_, int tr, double al, double be)
      : A(nullptr), C(c), M(M_), N(N_), lda(lda_), ldc(ldc_), trans(tr), alpha(al), beta(be),
        ty(tcode<TC>() | tcode<TC>() << 1) {}
};

// Householder QR in place: Q (n x K, K = min(n, m)) overwrites A, R (K x m)
// is written to R; sign-normalised so that R_jj >= 0.
struct QrDesc {
  void* A;
  void* R;
  int n, m, lda, ldr;
  int ty;
  QrDesc() = default;
  template <class U>
  __host__ QrDesc(U* a, typename nodeduce<U*>::type r, int n_, int m_, int lda_, int ldr_)
      : A(a), R(r), n(n_), m(m_), lda(lda_), ldr(ldr_), ty(tcode<U>()) {}
};

// Column-pivoted Householder QR for up to kmax steps, in place.  Reflector j
// is u_j (u_j[0] = 1 implicit) stored below the diagonal of column j, with
// tau[j] and alpha[j] (the signed diagonal).  rank = number of leading steps
// whose pivot norm exceeds eps * first pivot norm; with stop_at_rank the
// factorisation stops at the first pivot at or below that threshold.
struct RrqrDesc {
  void* A;
  void* tau;
  void* alpha;
  int* rank;
  int* steps;
  int n, m, lda, kmax;
  double eps;
  int stop_at_rank;
  int ty;
  void* Q;  // optional: Q (n x r, r = min(rank, kmax)) of the pivoted steps, ld ldq
  int ldq;
  int fill_t = -1;  // register kernel: touch t of the launch's FillCopy whose fill columns are read in place
  RrqrDesc() = default;
  template <class U>
  __host__ RrqrDesc(U* a, typename nodeduce<U*>::type tau_, typename nodeduce<U*>::type alpha_, int* rank_,
                    int* steps_, int n_, int m_, int lda_, int kmax_, double eps_, int stop,
                    typename nodeduce<U*>::type q = nullptr, int ldq_ = 0)
      : A(a), tau(tau_), alpha(alpha_), rank(rank_), steps(steps_), n(n_), m(m_), lda(lda_), kmax(kmax_),
        eps(eps_), stop_at_rank(stop), ty(tcode<U>()), Q(q), ldq(ldq_) {}
};


// One block of a vertical stack whose R factor is wanted.
struct BlkRef {
  const void* p;
  int ld, rows, trans;  // the stacked block is p (rows x cols) or p^T
};
// R (r x r, upper triangular, R_jj >= 0) of the QR of the stack of nblk
// blocks starting at blocks[first]; each block has r columns, of R's type.
struct StackQrDesc {
  void* R;
  int r, ldr, first, nblk;
  int ty;
  StackQrDesc() = default;
  template <class U>
  __host__ StackQrDesc(U* R_, int r_, int ldr_, int first_, int nblk_)
      : R(R_), r(r_), ldr(ldr_), first(first_), nblk(nblk_), ty(tcode<U>()) {}
};

// Basis change of the far-field blocks of a set of clusters whose bases
// changed ("touched"), with the block geometry resolved on the device.  For a
// touched cluster q (touch t) with new-from-old basis map T_t (r_new x r_old,
// ld rpad) and every far-field partner l in q's 6 x 6 window with r_old[l] > 0:
//   M(q, l) <- T_t M(q, l) T_{tidx[l]}^T   (the right factor only if l is touched)
//   M(l, q) <- M(l, q) T_t^T               (only if col_blocks and l is untouched)
// and the parent transfer block UP(q) <- T_t UP(q) when r_par[q / 4] > 0.
// touch_q / tidx null mean the identity (touch t is cluster t).
struct TouchXform {
  void* M;            // 36 blocks per cluster, sM elements each, ld rpad
  void* UP;           // one block per cluster, sM elements, ld rpad (null: none)
  const void* Tm;     // per touch, rpad x rpad
  const int* touch_q; // [nt]
  const int* tidx;    // [nc], -1 when untouched
  const int* r_old;   // [nc] ranks before the change
  const int* r_new;   // [nt]
  const int* r_par;   // [nc / 4] parent ranks, or null
  int nt, nside, rpad, col_blocks;
  size_t sM;
  // optional: the new bases Unew (per touch, sU elements, ld npad) replace
  // U of their clusters (n[q] x r_new[t]), one more workgroup per touch
  const void* Unew;
  void* U;
  const int* n;       // [nc] cluster sizes
  size_t sU;
  int npad;
};

// Ranks of a compression, finished on the device so that the basis change
// can be queued before the host reads them: for touch t (cluster q[t]),
// r_new[t] = min(rank[2 t], n[q[t]], r_cap), also written to r_lvl[q[t]] and
// to the row count M of the t-th descriptor of g when those are given.
struct RankFin {
  const int* rank;  // pivoted-QR ranks, two ints per touch (rank, steps)
  const int* q;     // [nt] touched clusters
  const int* n;     // [nc] cluster sizes
  int* r_new;       // [nt] out
  int* r_lvl;       // [nc] level ranks to patch, or null
  GemmDesc* g;      // [nt] descriptors whose M is the new rank, or null
  int nt, r_cap;
};
void launch_rank_finalize(const RankFin& a, hipStream_t s);

// Far-field weights with the block lists found on the device: for cluster
// q = ids[t], R of the stack of M(q, l)^T over the far-field partners l of
// q's 6 x 6 window (r[l] rows each) and of the parent term Z_t (r_par[q / 4]
// rows, ld rpad) when Z and r_par are given.  The stack is split in S
// segments of window slots (one workgroup each); segment s writes its R to
// out + (t * S + s) * so, or to out + q * so when S == 1 and out_by_id.
struct WinStack {
  const void* M;
  const void* Z;
  void* out;
  const int* ids;    // [nt]
  const int* r;      // [nc]
  const int* r_par;  // [nc / 4] or null
  size_t sM, so;
  int rpad, nside, ldo, nt, S, out_by_id;
  int max_rows;  // largest block of a stack (the ranks of the level and of z)
};

// One eliminated cluster of a colour batch (Algorithm 1, one Schur step):
// the units of its 3 x 3 neighbourhood, slot s = 3 (dx + 1) + (dy + 1),
// slot 4 being the cluster's own multipoles.  kind 1: the particles of a
// not yet eliminated neighbour; 2: the multipoles of an eliminated neighbour
// (or of the cluster itself); 0: absent.  off: column offset of the unit in
// the batch workspace X (X = D^-1 B, m x sum of unit sizes, ld mpad).
struct ElimRec {
  int i, ni, ri, m;
  int cl[9], kind[9], size[9], off[9];
};
// Level blocks and batch workspaces of the elimination kernels.  Blocks are
// in the factor's type, the pivot inverses in FP64.  F holds the fill of
// the unit pairs at Chebyshev distance 2 (pair index pair[9 sa + sb] >= 0),
// fpad x fpad each, npair per elimination.
struct ElimArgs {
  void* P;
  void* Qm;
  void* L;
  void* M;
  void* U;
  double* Dinv;
  void* X;
  void* F;
  const ElimRec* rec;
  const int* rk;  // cluster ranks after the batch's compression (steps 4, 5)
  void* tmp;      // r x fill products, rpad x fpad per (record, pair) (step 4)
  size_t sP, sQ, sL, sM, sU, sD, sX;
  int nb, npad, rpad, mpad, fpad, npair;
  signed char pair[81];
  unsigned char plist[81];  // 9 sa + sb of pair index 0 .. npair - 1
};

// Level transition k -> k-1 with device-side geometry: for parent P, its
// neighbour Q in slot sp of P's 3 x 3 neighbourhood and children c of P, c2
// of Q with nonzero ranks, P2P^(k-1)(P, Q) gets M^(k)(c, c2) at rows
// choff[4P + c], columns choff[4Q + c2]; U^(k-1)(P) gets the children's
// transfer blocks UP^(k)(4P + c) (cr x r_par[P]) at rows choff[4P + c].
struct TransArgs {
  const void* CM;    // child level M2L blocks, 36 per child, ld rpad
  const void* CUP;   // child level transfer blocks, ld rpad
  void* P;           // parent level near-field blocks, 9 per parent, ld npad
  void* U;           // parent level bases, ld npad
  const int* choff;  // [4 nc]
  const int* cr;     // [4 nc] child ranks
  const int* r_par;  // [nc] parent ranks before re-orthonormalisation
  size_t sM, sP, sU;
  int npad, rpad, nside, nc;
};

// One colour batch of Algorithm 2 with the elimination records of the
// factorisation.  Vectors (FP64, nrhs columns) of level k, per cluster j:
// b_j = bv + j sv, the snapshot of b_j taken at elimination bv + (nc + j) sv,
// x_j = bv + (2 nc + j) sv (sv = npad nrhs, ld npad); c_j = cv + j svc and
// y_j = cv + (nc + j) svc (svc = rpad nrhs, ld rpad).
//  forward:  snapshot b_i; w = D_i^-1 [b_i; 0]; b_q -= P_qi w^x (uneliminated
//            neighbours), c_p -= L_pi w^x (eliminated ones); c_i += w^z;
//  backward: r = [snapshot_i - sum_q P_iq x_q - sum_p Q_ip y_p; y_i];
//            x_i = (D_i^-1 r)^x.
// Same-colour clusters have disjoint neighbourhoods, so no two records of a
// batch write the same vector.
struct SolveArgs {
  const ElimRec* rec;
  const void* P;
  const void* Qm;
  const void* L;
  const double* Dinv;
  double* bv;
  double* cv;
  size_t sP, sQ, sL, sD;
  int nb, nc, npad, rpad, mpad, nrhs;
};

// M2L blocks in orthonormal coordinates, M_il = R_i K(dx, dy) R_l^T, for every
// cluster i and every l of its interaction list (window slot sl, offset
// (dx, dy) = position of l minus position of i), FP64 products, stored in the
// factor type.  R: per cluster rpad x p2 (ld rpad); table: 49 blocks p2 x p2
// at offset index 7 (dx + 3) + (dy + 3).
struct M2LAssemble {
  const double* R;
  const double* table;
  void* M;
  const int* r;
  size_t sR, sM;
  int nc, nside, rpad, p2;
};

// Inverse of a square FP64 matrix in place (Gauss-Jordan, partial pivoting).
struct InvDesc {
  double* A;
  int m, lda;
};

// Morton keys by bit interleaving with masks (bit b of x -> bit 2b, bit b
// of y -> bit 2b + 1), for coordinates below 2^15.
__host__ __device__ inline unsigned spread_bits(unsigned x) {
  x &= 0x0000ffffu;
  x = (x | (x << 8)) & 0x00ff00ffu;
  x = (x | (x << 4)) & 0x0f0f0f0fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}
__host__ __device__ inline unsigned gather_bits(unsigned x) {
  x &= 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0f0f0f0fu;
  x = (x | (x >> 4)) & 0x00ff00ffu;
  x = (x | (x >> 8)) & 0x0000ffffu;
  return x;
}
__host__ __device__ inline int demorton_x(int key) { return (int)gather_bits((unsigned)key); }
__host__ __device__ inline int demorton_y(int key) { return (int)gather_bits((unsigned)key >> 1); }
__host__ __device__ inline int morton2(int x, int y) {
  return (int)(spread_bits((unsigned)x) | (spread_bits((unsigned)y) << 1));
}
// Slot of cluster (jx, jy) in the 6 x 6 window of cluster (ix, iy) -- the
// children of the parent's 3 x 3 neighbourhood, which holds N_i and I_i --
// or -1 outside it.
__host__ __device__ inline int win_slot(int ix, int iy, int jx, int jy) {
  const int sx = jx - (2 * (ix >> 1) - 2), sy = jy - (2 * (iy >> 1) - 2);
  if (sx < 0 || sx > 5 || sy < 0 || sy > 5) return -1;
  return sx * 6 + sy;
}

struct Status {
  int singular;     // a zero pivot met
  int bad_cluster;  // first descriptor index that met it
};

// ---------------------------------------------------------------- launchers
// `ty` is the type code shared by the descriptors of the launch.
// plain: every descriptor has opA = opB = 0 (then N <= 4 runs as batched
// matrix-vector products).
void launch_gemm(const GemmDesc* d, int nd, int max_m, int max_n, int ty, int plain, hipStream_t s);
void launch_add(const AddDesc* d, int nd, int max_m, int max_n, int ty, hipStream_t s);
void launch_touch_xform(const TouchXform& a, int ty, hipStream_t s);
void launch_transition(const TransArgs& a, int ty, hipStream_t s);
void launch_m2l_assemble(const M2LAssemble& a, int ty, hipStream_t s);
// Step 0..3 of a colour batch (0, 1: forward; 2, 3: backward); wk holds
// mpad x nrhs doubles per record; max_rows bounds the rows of the step.
void launch_solve(const SolveArgs& a, int step, double* wk, int max_rows, int ty, hipStream_t s);
// The elimination steps of a colour batch (one record per eliminated
// cluster, geometry resolved on the device):
//   0 build the pivot blocks D = [[P_ii, U_i], [U_i^T, 0]] (FP64);
//   1 X_u = D^-1 [B_u; 0] for every unit u (X_centre = -D^-1 [0; I]);
//   2 Schur updates target(a, b) -= C_a X_b over all unit pairs (fill of
//     pairs at distance 2 goes to F);
//   3 M2L(i) row: L_iq / M_ip += X^z_u;
//   4, 5 projection of the compressed fill into M2L with the new bases:
//     M_qq' += U_q^T F_qq' U_q' (step 4 forms U_q^T F_qq'), M_qp += U_q^T F_qp,
//     M_pq += F_pq U_q.
// max_m / max_n bound the row / column sizes for the tiling.
void launch_elim(const ElimArgs& a, int step, int max_m, int max_n, int ty, hipStream_t s);
// Unpivoted Householder QR (Q in place, R out), one workgroup per matrix;
// lds > 0: every matrix staged in LDS ((n + 1) m elements, lds bytes at most).
constexpr size_t kQrLdsBytes = 64 * 1024;
inline size_t qr_lds_bytes(int n, int m, int ty) { return (ty ? 4 : 8) * (size_t)(n + 1) * m; }
void launch_qr(const QrDesc* d, int nd, size_t lds, int ty, hipStream_t s);
// The same QR by one wave per matrix (m <= 64, n <= nr rows in registers;
// nr = qr_wave_rows(n, m, ty): 32, 64 or 96 rows, and 128 in FP32; 0 when
// the matrix does not fit).  max_k bounds min(n, m) over the batch (LDS of
// the reflectors: max_k nr elements).
int qr_wave_rows(int n, int m, int ty);
void launch_qr_wave(const QrDesc* d, int nd, int nr, int max_k, int ty, hipStream_t s);
// Pivoted QR with the whole matrix staged in LDS: (n + 1) * m + m elements
// must fit in `lds` <= kRrqrLdsBytes.  max_n: the largest row count.
constexpr size_t kRrqrLdsBytes = 159 * 1024;
void launch_rrqr_lds(const RrqrDesc* d, int nd, size_t lds, int max_n, int ty, hipStream_t s);
// Same arithmetic on the matrix in place (one workgroup per matrix, the
// matrix L2-resident, column norms in LDS): max_m columns at most.
void launch_rrqr_global(const RrqrDesc* d, int nd, int max_m, int max_n, int ty, hipStream_t s);
// Pivoted QR with each column in the registers of one thread, and Q when
// d.Q is set: every matrix has m <= kRrqrRegCols and n <= nr, with nr one of
// rrqr_reg_rows(ty); LDS holds the kmax x nr reflectors.
constexpr int kRrqrRegCols = 512;
int rrqr_reg_rows(int n, int ty);  // smallest register row class >= n, 0 if none
bool rrqr_reg_reads_fill(int nr, int ty);  // the row class's kernel can read fills in place (fill_t)
size_t rrqr_reg_lds(int nr, int kmax, int ty);
// fc (host copy, pointers rebased; or null): the fills of descriptors with
// fill_t >= 0 are read from their blocks (columns from col0 on) instead of A.
struct FillCopy;
void launch_rrqr_reg(const RrqrDesc* d, int nd, int max_m, int nr, int max_kmax, int ty, const FillCopy* fc,
                     hipStream_t s);
// Q of RrqrDescs whose pivoted QR ran in the LDS / in-place kernels (rank and
// steps read on the device); every n <= max_n <= 512, kmax <= max_kmax.
void launch_formq_rr(const RrqrDesc* d, int nd, int max_n, int max_kmax, int ty, hipStream_t s);
void launch_stackqr(const StackQrDesc* d, const BlkRef* b, int nd, int max_r, int ty, hipStream_t s);
void launch_stackqr_win(const WinStack& a, int max_r, int ty, hipStream_t s);
// The same weights (S == 1) from the FP64 Gram matrix of the stack and its
// Cholesky factor; max_r <= rpad <= kMaxRank.
void launch_gram_win(const WinStack& a, int max_r, int ty, hipStream_t s);
// Whole-matrix FP64 Gauss-Jordan inverse with the matrix in registers (one
// workgroup per matrix), every m <= kGjRegMax.
constexpr int kGjRegMax = 192;
void launch_gj_reg(const InvDesc* d, int nd, int max_m, Status* st, hipStream_t s);
// Fill of the touched clusters into their pivoted-QR inputs: touch t = (b,
// sq, nq, col0) takes, for every unit s2 of record b whose unit pair (sq, s2)
// carries fill, the nq x size[s2] block F(b, pair) (ld fpad) into columns
// col0 + (sizes of the earlier such units) of A + t per (ld npad).
struct FillCopy {
  const ElimRec* rec;
  const int* touch;  // 5 ints per touch: b, sq, nq, col0, and 1 where its pivoted QR reads the fills in place
  const void* F;
  void* A;
  size_t per;
  int fpad, npad, npair, nt;
  signed char pair[81];
};
void launch_fill_copy(const FillCopy& a, int ty, hipStream_t s);
// Blocked Gauss-Jordan pieces (panel of nb <= 64 columns starting at j0).
void launch_gj_panel(const InvDesc* d, int nd, int max_m, int j0, int nb, int* piv, int ldp,
                     Status* st, hipStream_t s);
void launch_gj_rest(const InvDesc* d, int nd, int max_m, int j0, int nb, const int* piv, int ldp,
                    double* tmp, size_t ldt, hipStream_t s);
void launch_gj_unpermute(const InvDesc* d, int nd, int max_m, const int* piv, int ldp, hipStream_t s);

// ---------------------------------------------------------- problem kernels
struct KernelFn {
  int kind;   // ifmm_kernel_kind: 0 1/r, 1 exp(-r/ell), 2-4 the numerical section's kernels (a = ell),
              // 5 d/d ell exp(-r/ell)
  double ell;
};

// Chebyshev L2P at the points of each leaf: S (n_i x p^2) into dst + i*stride.
void launch_leaf_interp(const double* pts, const int* leaf_start, const int* leaf_n,
                        int nleaf, int kappa, double lox, double loy, double size, int p,
                        double* dst, size_t stride, int ld, int max_n, hipStream_t s);
// Near-field blocks of the leaves: dst[i][slot] = K(x_i, x_j), diagonal of the
// self block replaced by d; P is FP64 (f32 = 0) or FP32 (f32 = 1).  When near
// is given, the same values also go to the FP64 near field of the product:
// leaf i's n_i x c_i block (c_i = the points of its 3 x 3 neighbours in slot
// order, ld n_i, self pairs 0) at near + near_off[i].
void launch_near_field(const double* pts, const int* leaf_start, const int* leaf_n,
                       const int* nbr9, int nleaf, KernelFn kf, const double* d,
                       void* P, int f32, size_t slot_stride, int ld, int max_n, double* near,
                       const size_t* near_off, hipStream_t s);
// Kernel between the Chebyshev nodes of two boxes of half-width h whose
// centres differ by (dx, dy) * 2h, for the 49 offsets dx, dy in [-3, 3].
void launch_m2l_table(KernelFn kf, int p, double h, double* dst, hipStream_t s);

// FMM product passes (Chebyshev coordinates, tree order).
struct FmmLevel {
  int k, nc;
  double* W;  // multipole node values [nc][p2][nrhs]
  double* G;  // local node values     [nc][p2][nrhs]
  const double* table;  // 49 x p2 x p2
};
void launch_p2m(const double* pts, const int* leaf_start, const int* leaf_n, int nleaf,
                int kappa, double lox, double loy, double size, int p, const double* x, int ldx,
                int nrhs, double* W, hipStream_t s);
void launch_m2m(const double* E, int p, int nc_parent, const double* Wc, double* Wp, int nrhs,
                hipStream_t s);
// Raise a kernel's dynamic LDS limit to the 160 KiB of a gfx950 CU (once per
// kernel; thread-safe).
void allow_lds(const void* fn);
void launch_m2l(int p, int k, const double* table, const double* W, double* G, int nrhs,
                hipStream_t s);
void launch_l2l(const double* E, int p, int nc_parent, const double* Gp, double* Gc, int nrhs,
                hipStream_t s);
void launch_l2p_p2p(const double* pts, const int* leaf_start, const int* leaf_n, const int* nbr9,
                    int nleaf, int kappa, double lox, double loy, double size, int p,
                    KernelFn kf, const double* G, const double* x, int ldx, const double* d,
                    double* y, int ldy, int nrhs, hipStream_t s);
// L2P + near field from the stored blocks (launch_near_field), + d x when d.
void launch_l2p_near(const double* pts, const int* leaf_start, const int* leaf_n, const int* nbr9,
                     int nleaf, int kappa, double lox, double loy, double size, int p, const double* near,
                     const size_t* near_off, const double* G, const double* x, int ldx, const double* d,
                     double* y, int ldy, int nrhs, hipStream_t s);
// out[r] += sum_i x[i + r*ld]^2 (out must be zeroed first).
void launch_colnorm2(const double* x, int n, int nrhs, int ld, double* out, hipStream_t s);
void launch_gather_rows(const double* src, int ld_src, const int* idx, int n, int nrhs,
                        double* dst, int ld_dst, hipStream_t s);
void launch_scatter_rows(const double* src, int ld_src, const int* idx, int n, int nrhs,
                         double* dst, int ld_dst, hipStream_t s);

// Quadtree of n points (x, y interleaved, any order) at depth kappa, on the
// stream: key_in / key_out / idx are n-int scratch, tmp holds
// tree_scratch_bytes(n, 4^kappa, 2 kappa); leaf_n (4^kappa ints) must be
// zeroed.  Out: perm (tree position -> original index, stable within a leaf),
// leaf_n, leaf_start (exclusive prefix sum), spts (coordinates in tree order),
// *bad = 1 for a point not finite or outside [lo, lo + size]^2.
hipError_t tree_scratch_bytes(int n, int nleaf, int bits, size_t* bytes);
hipError_t launch_tree_build(const double* pts, int n, double lox, double loy, double size, int kappa,
                             int* key_in, int* key_out, int* idx, int* perm, int* leaf_n,
                             int* leaf_start, int* bad, double* spts, void* tmp, size_t tmp_bytes,
                             hipStream_t s);
// *bad = 1 when two points of one leaf coincide.
void launch_tree_distinct(const double* spts, const int* leaf_start, const int* leaf_n, int nleaf,
                          int* bad, hipStream_t s);
// Sets *bad when an entry of v[0..n) is not finite.
void launch_check_finite(const double* v, int n, int* bad, hipStream_t s);
// Rows of each leaf of a tree-order vector (ld ldv, nrhs columns) into the
// leaf's block (blk + i bstride, ld ldb), and back.
void launch_leaf_gather(const double* v, int ldv, double* blk, size_t bstride, int ldb, const int* leaf_start,
                        const int* leaf_n, int nleaf, int nrhs, hipStream_t s);
void launch_leaf_scatter(const double* blk, size_t bstride, int ldb, double* v, int ldv, const int* leaf_start,
                         const int* leaf_n, int nleaf, int nrhs, hipStream_t s);
void launch_fill(double* x, size_t n, double v, hipStream_t s);
void launch_add_const(double* x, size_t n, double v, hipStream_t s);
// bytes (a multiple of 4) from device memory into pinned host memory given
// by its device address, by a kernel (see ifmm_tree.hip).
void launch_copy_to_host(const void* src, void* dst_dev, size_t bytes, hipStream_t s);
// bytes from pinned host memory given by its device address (16-byte
// aligned, as is dst) into device memory, by a kernel.
void launch_copy_from_host(const void* src_dev, void* dst, size_t bytes, hipStream_t s);

}  // namespace ifmm
