// Batched dense linear algebra for the IFMM on gfx950 (FP64 and FP32).
//
// Every kernel consumes an array of descriptors planned on the host, one
// independent small problem per descriptor (the clusters of one colour batch
// never share a block, so their problems run concurrently).  Wave size 64,
// 256-thread workgroups; matrices are column-major.  Kernels are templates
// over the scalar type of their operands; the pivot inverse is FP64 only.
#include "ifmm_internal.h"

#include <mutex>
#include <unordered_set>

namespace ifmm {

namespace {

constexpr int WG = 256;
constexpr int WAVE = 64;

template <class T>
__device__ inline T wave_sum(T v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Block-wide sum over NT threads; every thread gets the result.  red must
// hold NT/WAVE values.
template <class T, int NT = WG>
__device__ inline T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  T t = 0;
  for (int i = 0; i < NT / WAVE; ++i) t += red[i];
  return t;
}

// Block-wide argmax of (value, index): largest value, smallest index on ties.
template <class T, int NT = WG>
__device__ inline void block_argmax(T v, int idx, T* rv, int* ri, T& bv, int& bi) {
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    T ov = __shfl_xor(v, o, WAVE);
    int oi = __shfl_xor(idx, o, WAVE);
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) { rv[w] = v; ri[w] = idx; }
  __syncthreads();
  bv = rv[0];
  bi = ri[0];
  for (int i = 1; i < NT / WAVE; ++i)
    if (rv[i] > bv || (rv[i] == bv && ri[i] < bi)) { bv = rv[i]; bi = ri[i]; }
}

// Sum over the 16 lanes of a lane group (lanes 16g .. 16g+15 of a wave).
constexpr int GRP = 16;
template <class T>
__device__ inline T grp_sum(T v) {
  v += __shfl_xor(v, 1, WAVE);
  v += __shfl_xor(v, 2, WAVE);
  v += __shfl_xor(v, 4, WAVE);
  v += __shfl_xor(v, 8, WAVE);
  return v;
}

// ------------------------------------------------------------------- GEMM
// 64 x 64 output tile (m0, n0) of one product on the matrix cores, operands
// loaded straight into registers: each of the four waves owns a 32 x 32
// quarter as 2 x 2 blocks of 16 x 16, advanced by v_mfma_*_16x16x4 (FP32
// operands with FP32 accumulation when A and B are FP32, else FP64 operands
// and accumulation), K by 16 per iteration.
// Lane layouts of the 16x16x4 instructions (lane l, accumulator register r):
// A(i, k) from lane i + 16 k, B(k, j) from lane j + 16 k; the FP32 result
// D(4 (l / 16) + r, l % 16), the FP64 result D(4 r + l / 16, l % 16).
// Lane l feeds k = k0 + 4 (l / 16) + s to MFMA step s (s = 0..3): any
// assignment of the 16 k values to (lane group, step) sums the same
// products, and this one gives a lane four consecutive k, loaded as one
// 16-byte access where the operand is contiguous in k (FP32 B as stored, FP32
// A transposed).  FP32 results are stored four rows per lane at once.
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));

__device__ inline mf4 mfma16(float a, float b, mf4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ inline md4 mfma16(double a, double b, md4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline int mfma_row(float, int l, int r) { return 4 * (l / 16) + r; }
__device__ inline int mfma_row(double, int l, int r) { return 4 * r + l / 16; }

template <class TA, class TB, class TC>
__device__ void gemm_tile(const GemmDesc& d, int m0, int n0) {
  using Acc = typename std::conditional<std::is_same<TA, float>::value && std::is_same<TB, float>::value,
                                        float, double>::type;
  using V4 = typename std::conditional<std::is_same<Acc, float>::value, mf4, md4>::type;
  constexpr bool kF = std::is_same<Acc, float>::value;
  const TA* __restrict__ Ap = static_cast<const TA*>(d.A);
  const TB* __restrict__ Bp = static_cast<const TB*>(d.B);
  TC* Cp = static_cast<TC*>(d.C);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int wm = m0 + (w & 1) * 32, wn = n0 + (w >> 1) * 32;
  if (wm >= d.M || wn >= d.N) return;  // no barrier below: a wave may leave
  const int li = lane % 16, lk = lane / 16;
  // this lane's rows / columns of the two 16-blocks, and their validity
  const int r0 = wm + li, r1 = wm + 16 + li, c0 = wn + li, c1 = wn + 16 + li;
  const bool vr0 = r0 < d.M, vr1 = r1 < d.M, vc0 = c0 < d.N, vc1 = c1 < d.N;
  // the wave's second 16-row / 16-column block lies (partly) inside the
  // product: else its MFMAs are skipped (wave-uniform; padded blocks of the
  // many 36- to 100-wide operands would otherwise double the MFMA work)
  const bool two_m = wm + 16 < d.M, two_n = wn + 16 < d.N;
  const size_t sa = d.opA ? 1 : (size_t)d.lda, ra = d.opA ? (size_t)d.lda : 1;  // A(i, k) = Ap[i ra + k sa]
  const size_t sb = d.opB ? (size_t)d.ldb : 1, cb = d.opB ? 1 : (size_t)d.ldb;  // B(k, j) = Bp[k sb + j cb]
  const bool vecB = kF && d.opB == 0 && (d.ldb & 3) == 0 && (reinterpret_cast<uintptr_t>(Bp) & 15) == 0;
  const bool vecA = kF && d.opA == 1 && (d.lda & 3) == 0 && (reinterpret_cast<uintptr_t>(Ap) & 15) == 0;
  V4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = V4{0, 0, 0, 0};
  for (int k0 = 0; k0 < d.K; k0 += 16) {
    const int kb = k0 + 4 * lk;
    const bool full = kb + 3 < d.K;
    Acc a[4][2], b[4][2];
    if (vecA && full) {
      const mf4 x0 = vr0 ? *reinterpret_cast<const mf4*>(Ap + r0 * ra + kb) : mf4{0, 0, 0, 0};
      const mf4 x1 = vr1 ? *reinterpret_cast<const mf4*>(Ap + r1 * ra + kb) : mf4{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        a[s][0] = (Acc)x0[s];
        a[s][1] = (Acc)x1[s];
      }
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kb + s;
        const bool vk = k < d.K;
        a[s][0] = vk && vr0 ? (Acc)Ap[r0 * ra + k * sa] : Acc(0);
        a[s][1] = vk && vr1 ? (Acc)Ap[r1 * ra + k * sa] : Acc(0);
      }
    }
    if (vecB && full) {
      const mf4 y0 = vc0 ? *reinterpret_cast<const mf4*>(Bp + kb + c0 * cb) : mf4{0, 0, 0, 0};
      const mf4 y1 = vc1 ? *reinterpret_cast<const mf4*>(Bp + kb + c1 * cb) : mf4{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        b[s][0] = (Acc)y0[s];
        b[s][1] = (Acc)y1[s];
      }
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kb + s;
        const bool vk = k < d.K;
        b[s][0] = vk && vc0 ? (Acc)Bp[k * sb + c0 * cb] : Acc(0);
        b[s][1] = vk && vc1 ? (Acc)Bp[k * sb + c1 * cb] : Acc(0);
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      acc[0][0] = mfma16(a[s][0], b[s][0], acc[0][0]);
      if (two_n) acc[0][1] = mfma16(a[s][0], b[s][1], acc[0][1]);
      if (two_m) acc[1][0] = mfma16(a[s][1], b[s][0], acc[1][0]);
      if (two_m && two_n) acc[1][1] = mfma16(a[s][1], b[s][1], acc[1][1]);
    }
  }
  const Acc al = (Acc)d.alpha, be = (Acc)d.beta;
  const bool vecC = kF && std::is_same<TC, float>::value && (d.ldc & 3) == 0 &&
                    (reinterpret_cast<uintptr_t>(Cp) & 15) == 0;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int gm0 = wm + 16 * bi + mfma_row(Acc(0), lane, 0), gn = wn + 16 * bj + li;
      if (gn >= d.N) continue;
      if (vecC && gm0 + 3 < d.M) {  // four rows of one column at once
        mf4* c = reinterpret_cast<mf4*>(Cp + gm0 + (size_t)gn * d.ldc);
        mf4 v;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = (float)(al * acc[bi][bj][r]);
        if (d.beta != 0.0) {
          const mf4 o = *c;
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = (float)fma(al, (Acc)acc[bi][bj][r], be * (Acc)o[r]);
        }
        *c = v;
        continue;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = wm + 16 * bi + mfma_row(Acc(0), lane, r);
        if (gm < d.M) {
          TC* c = Cp + gm + (size_t)gn * d.ldc;
          const Acc v = acc[bi][bj][r];
          *c = (TC)(d.beta == 0.0 ? al * v : fma(al, v, be * (Acc)*c));
        }
      }
    }
}

template <class TA, class TB, class TC>
__global__ __launch_bounds__(WG) void k_gemm(const GemmDesc* __restrict__ descs, int tiles_m) {
  const GemmDesc d = descs[blockIdx.x];
  const int tm = blockIdx.y % tiles_m, tn = blockIdx.y / tiles_m;
  const int m0 = tm * 64, n0 = tn * 64;
  if (d.C == nullptr || m0 >= d.M || n0 >= d.N) return;
  gemm_tile<TA, TB, TC>(d, m0, n0);
}

// Products with few right-hand columns (N <= 4, A and B as stored): the
// solve's matrix-vector work.  A 64-row tile per workgroup; the four waves
// split K, each lane owns a row (coalesced column reads of A), and the
// partial sums meet in LDS.
constexpr int GEMV_N = 4;
template <class TA, class TB, class TC>
__global__ __launch_bounds__(WG) void k_gemv(const GemmDesc* __restrict__ descs) {
  using Acc = typename std::conditional<std::is_same<TA, float>::value && std::is_same<TB, float>::value,
                                        float, double>::type;
  const GemmDesc d = descs[blockIdx.x];
  const int m0 = blockIdx.y * WAVE;
  if (d.C == nullptr || m0 >= d.M) return;
  const TA* __restrict__ A = static_cast<const TA*>(d.A);
  const TB* __restrict__ B = static_cast<const TB*>(d.B);
  __shared__ Acc part[WG / WAVE][GEMV_N][WAVE];
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int i = m0 + lane;
  Acc acc[GEMV_N];
#pragma unroll
  for (int c = 0; c < GEMV_N; ++c) acc[c] = 0;
  if (i < d.M) {
    for (int k = w; k < d.K; k += WG / WAVE) {
      const Acc a = (Acc)A[i + (size_t)k * d.lda];
#pragma unroll
      for (int c = 0; c < GEMV_N; ++c)
        if (c < d.N) acc[c] = fma(a, (Acc)B[k + (size_t)c * d.ldb], acc[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < GEMV_N; ++c) part[w][c][lane] = acc[c];
  __syncthreads();
  if (w == 0 && i < d.M) {
    TC* Cp = static_cast<TC*>(d.C);
    for (int c = 0; c < d.N; ++c) {
      Acc v = part[0][c][lane];
      for (int q = 1; q < WG / WAVE; ++q) v += part[q][c][lane];
      TC* cc = Cp + i + (size_t)c * d.ldc;
      *cc = (TC)(d.beta == 0.0 ? (Acc)d.alpha * v : fma((Acc)d.alpha, v, (Acc)d.beta * (Acc)*cc));
    }
  }
}

// --------------------------------------------------------- ELIMINATION
__device__ inline int e9_dx(int s) { return s / 3 - 1; }
__device__ inline int e9_dy(int s) { return s % 3 - 1; }

// Descriptor of step 1 for unit u of record r (false: nothing to do).
template <class T>
__device__ bool elim_x_desc(const ElimArgs& a, const ElimRec& r, int b, int u, GemmDesc& g) {
  if (!r.kind[u] || u == 4) return false;
  T* X = static_cast<T*>(a.X) + (size_t)b * a.sX + (size_t)r.off[u] * a.mpad;
  const T* B = r.kind[u] == 1 ? static_cast<const T*>(a.P) + ((size_t)r.i * 9 + u) * a.sP
                              : static_cast<const T*>(a.Qm) + ((size_t)r.i * 9 + u) * a.sQ;
  g.A = a.Dinv + (size_t)r.i * a.sD;
  g.B = B;
  g.C = X;
  g.M = r.m;
  g.N = r.size[u];
  g.K = r.ni;
  g.lda = a.mpad;
  g.ldb = a.npad;
  g.ldc = a.mpad;
  g.opA = 0;
  g.opB = 0;
  g.alpha = 1.0;
  g.beta = 0.0;
  return true;
}

// Descriptor of step 2 for the unit pair (sa, sb) of record r.  The pivot
// column block of row unit sa -- P_qi (particles q) or L_pi (multipoles of an
// eliminated p) -- is read as the transpose of its symmetric partner in the
// pivot row, P_iq or Qm_ip (the reordered extended system is symmetric, and
// the elimination keeps both partners equal up to rounding): the record's
// own blocks, just read by X = D^-1 B, with each lane's four consecutive k
// contiguous in memory (one 16-byte load).  FP32 only: FP64 operands take
// one 8-byte load per k either way, and the stored orientation keeps the
// lanes of a load on consecutive rows.
template <class T>
__device__ bool elim_schur_desc(const ElimArgs& a, const ElimRec& r, int b, int sa, int sb, GemmDesc& g) {
  if (sa == 4 || !r.kind[sa] || !r.kind[sb]) return false;
  const int ka = r.kind[sa], kb = r.kind[sb], ca = r.cl[sa];
  constexpr bool kT = std::is_same<T, float>::value;
  if (kT) {
    g.A = ka == 1 ? static_cast<const T*>(a.P) + ((size_t)r.i * 9 + sa) * a.sP
                  : static_cast<const T*>(a.Qm) + ((size_t)r.i * 9 + sa) * a.sQ;
    g.lda = a.npad;
  } else {
    g.A = ka == 1 ? static_cast<const T*>(a.P) + ((size_t)ca * 9 + (8 - sa)) * a.sP
                  : static_cast<const T*>(a.L) + ((size_t)ca * 9 + (8 - sa)) * a.sL;
    g.lda = ka == 1 ? a.npad : a.rpad;
  }
  g.B = static_cast<const T*>(a.X) + (size_t)b * a.sX + (size_t)r.off[sb] * a.mpad;
  g.ldb = a.mpad;
  const bool adj = abs(e9_dx(sa) - e9_dx(sb)) <= 1 && abs(e9_dy(sa) - e9_dy(sb)) <= 1;
  g.beta = 1.0;
  if (ka == 2 && kb == 2) {
    const int cb = r.cl[sb];
    const int sl = win_slot(demorton_x(ca), demorton_y(ca), demorton_x(cb), demorton_y(cb));
    g.C = static_cast<T*>(a.M) + ((size_t)ca * 36 + sl) * a.sM;
    g.ldc = a.rpad;
  } else if (!adj) {
    g.C = static_cast<T*>(a.F) + ((size_t)b * a.npair + a.pair[9 * sa + sb]) * a.fpad * a.fpad;
    g.ldc = a.fpad;
    g.beta = 0.0;
  } else {
    const int st9 = 3 * (e9_dx(sb) - e9_dx(sa) + 1) + (e9_dy(sb) - e9_dy(sa) + 1);
    if (ka == 1 && kb == 1) {
      g.C = static_cast<T*>(a.P) + ((size_t)ca * 9 + st9) * a.sP;
      g.ldc = a.npad;
    } else if (ka == 1) {
      g.C = static_cast<T*>(a.Qm) + ((size_t)ca * 9 + st9) * a.sQ;
      g.ldc = a.npad;
    } else {
      g.C = static_cast<T*>(a.L) + ((size_t)ca * 9 + st9) * a.sL;
      g.ldc = a.rpad;
    }
  }
  g.M = r.size[sa];
  g.N = r.size[sb];
  g.K = r.ni;
  g.opA = kT ? 1 : 0;
  g.opB = 0;
  g.alpha = -1.0;
  return true;
}

// Descriptor of projection step 4 or 5 for the pair (sa, sb) of record r.
template <class T>
__device__ bool elim_proj_desc(const ElimArgs& a, const ElimRec& r, int b, int sa, int sb, int step, GemmDesc& g) {
  const int pi = a.pair[9 * sa + sb];
  if (pi < 0) return false;
  const int ka = r.kind[sa], kb = r.kind[sb];
  if (!ka || !kb || (ka == 2 && kb == 2)) return false;
  if (step == 4 && !(ka == 1 && kb == 1)) return false;
  const int ca = r.cl[sa], cb = r.cl[sb];
  const T* F = static_cast<const T*>(a.F) + ((size_t)b * a.npair + pi) * a.fpad * a.fpad;
  T* tm = static_cast<T*>(a.tmp) + ((size_t)b * a.npair + pi) * a.rpad * a.fpad;
  const T* U = static_cast<const T*>(a.U);
  g.opA = 0;
  g.opB = 0;
  g.alpha = 1.0;
  g.beta = 1.0;
  g.ldc = a.rpad;
  g.C = static_cast<T*>(a.M) + ((size_t)ca * 36 + win_slot(demorton_x(ca), demorton_y(ca), demorton_x(cb), demorton_y(cb))) * a.sM;
  if (ka == 1 && kb == 1 && step == 4) {  // tm = U_a^T F
    g.A = U + (size_t)ca * a.sU;
    g.lda = a.npad;
    g.opA = 1;
    g.B = F;
    g.ldb = a.fpad;
    g.C = tm;
    g.M = a.rk[ca];
    g.N = r.size[sb];
    g.K = r.size[sa];
    g.beta = 0.0;
  } else if (ka == 1 && kb == 1) {  // M += tm U_b
    g.A = tm;
    g.lda = a.rpad;
    g.B = U + (size_t)cb * a.sU;
    g.ldb = a.npad;
    g.M = a.rk[ca];
    g.N = a.rk[cb];
    g.K = r.size[sb];
  } else if (ka == 1) {  // M += U_a^T F
    g.A = U + (size_t)ca * a.sU;
    g.lda = a.npad;
    g.opA = 1;
    g.B = F;
    g.ldb = a.fpad;
    g.M = a.rk[ca];
    g.N = r.size[sb];
    g.K = r.size[sa];
  } else {  // M += F U_b
    g.A = F;
    g.lda = a.fpad;
    g.B = U + (size_t)cb * a.sU;
    g.ldb = a.npad;
    g.M = r.size[sa];
    g.N = a.rk[cb];
    g.K = r.size[sb];
  }
  return true;
}

// The products of steps 2, 4 and 5 run one workgroup per (record, item) --
// step 2: one of the 72 unit pairs with row unit != 4; steps 4, 5: one of
// the pairs at Chebyshev distance 2 -- looping over the item's 64 x 64
// output tiles.  The order is XCD-aware: a launch's workgroups go
// round-robin to the 8 XCDs (linear id mod 8), so record b's items take the
// linear ids congruent to b mod 8 and run back to back on one XCD, where the
// record's operand blocks (pivot column, X, bases, fill) stay in that XCD's
// L2 for all its products instead of being fetched from HBM once per
// product (measured: the Schur updates' HBM fetches fall 4.4x).  Step 1
// (X = D^-1 B) keeps the record-fastest 2D grid (nb, units x tiles): with
// its FP64 D^-1 operand the XCD-aware order measured slower (each record's
// 54 tiles then read the same D^-1 lines at the same time).
constexpr int kXcd = 8;
__host__ __device__ constexpr int elim_items(int step, int npair) { return step == 2 ? 72 : npair; }

// grid (nb, units * tiles): step 0 and 3 are elementwise; 1, 2, 4, 5
// products over the XCD-aware linear grid above.  One instantiation per
// step: each gets the registers of its own step only (the FP64-accumulating
// step 1 needs twice those of the FP32 products).
template <class T, int STEP>
__global__ __launch_bounds__(WG) void k_elim(const ElimArgs a, int tiles_m, int tiles_n) {
  constexpr int step = STEP;
  if (step == 2 || step >= 4) {
    const int items = elim_items(step, a.npair);
    const int L = blockIdx.x, j = L / kXcd;
    const int b = (j / items) * kXcd + L % kXcd, y = j % items;
    if (b >= a.nb) return;
    const ElimRec& r = a.rec[b];
    GemmDesc g;
    if (step == 2) {
      const int sa = y / 9 + (y / 9 >= 4 ? 1 : 0), sb = y % 9;
      if (!elim_schur_desc<T>(a, r, b, sa, sb, g)) return;
      for (int n0 = 0; n0 < g.N; n0 += 64)
        for (int m0 = 0; m0 < g.M; m0 += 64) gemm_tile<T, T, T>(g, m0, n0);
    } else {
      const int sa = a.plist[y] / 9, sb = a.plist[y] % 9;
      if (!elim_proj_desc<T>(a, r, b, sa, sb, step, g)) return;
      for (int n0 = 0; n0 < g.N; n0 += 64)
        for (int m0 = 0; m0 < g.M; m0 += 64) gemm_tile<T, T, T>(g, m0, n0);
    }
    return;
  }
  const int b = blockIdx.x;
  const ElimRec& r = a.rec[b];
  const int per = tiles_m * tiles_n;
  const int unit = blockIdx.y / per, tile = blockIdx.y % per;
  const int m0 = (tile % tiles_m) * 64, n0 = (tile / tiles_m) * 64;
  if (step == 1) {
    if (unit == 4) {  // X_centre = -D^-1[:, ni:m]
      if (!r.kind[4]) return;
      const double* D = a.Dinv + (size_t)r.i * a.sD + (size_t)r.ni * a.mpad;
      T* X = static_cast<T*>(a.X) + (size_t)b * a.sX + (size_t)r.off[4] * a.mpad;
      for (int e = threadIdx.x; e < 64 * 64; e += WG) {
        const int row = m0 + e % 64, col = n0 + e / 64;
        if (row < r.m && col < r.ri) X[row + (size_t)col * a.mpad] = (T)(-D[row + (size_t)col * a.mpad]);
      }
      return;
    }
    GemmDesc g;
    if (!elim_x_desc<T>(a, r, b, unit, g) || m0 >= g.M || n0 >= g.N) return;
    gemm_tile<double, T, T>(g, m0, n0);
  } else if (step == 0) {  // D = [[P_ii, U], [U^T, 0]]
    double* D = a.Dinv + (size_t)r.i * a.sD;
    const T* Pii = static_cast<const T*>(a.P) + ((size_t)r.i * 9 + 4) * a.sP;
    const T* U = static_cast<const T*>(a.U) + (size_t)r.i * a.sU;
    for (int e = threadIdx.x; e < 64 * 64; e += WG) {
      const int row = m0 + e % 64, col = n0 + e / 64;
      if (row >= r.m || col >= r.m) continue;
      double v;
      if (row < r.ni && col < r.ni) v = (double)Pii[row + (size_t)col * a.npad];
      else if (row < r.ni) v = (double)U[row + (size_t)(col - r.ni) * a.npad];
      else if (col < r.ni) v = (double)U[col + (size_t)(row - r.ni) * a.npad];
      else v = 0.0;
      D[row + (size_t)col * a.mpad] = v;
    }
  } else {  // step 3: M2L(i) row += X^z_u
    if (!r.kind[unit]) return;
    const T* Xz = static_cast<const T*>(a.X) + (size_t)b * a.sX + r.ni + (size_t)r.off[unit] * a.mpad;
    T* C;
    if (r.kind[unit] == 1) {
      C = static_cast<T*>(a.L) + ((size_t)r.i * 9 + unit) * a.sL;
    } else {
      const int cb = r.cl[unit];
      const int sl = win_slot(demorton_x(r.i), demorton_y(r.i), demorton_x(cb), demorton_y(cb));
      C = static_cast<T*>(a.M) + ((size_t)r.i * 36 + sl) * a.sM;
    }
    for (int e = threadIdx.x; e < 64 * 64; e += WG) {
      const int row = m0 + e % 64, col = n0 + e / 64;
      if (row < r.ri && col < r.size[unit]) C[row + (size_t)col * a.rpad] += Xz[row + (size_t)col * a.mpad];
    }
  }
}

// -------------------------------------------------------------------- ADD
// Computed in FP64, stored in C's type.
template <class TA, class TC>
__global__ __launch_bounds__(WG) void k_add(const AddDesc* __restrict__ descs, int tiles_m) {
  const AddDesc d = descs[blockIdx.x];
  const int tm = blockIdx.y % tiles_m, tn = blockIdx.y / tiles_m;
  const int m0 = tm * 64, n0 = tn * 64;
  if (d.C == nullptr || m0 >= d.M || n0 >= d.N) return;
  const TA* Ap = static_cast<const TA*>(d.A);
  TC* Cp = static_cast<TC*>(d.C);
  for (int e = threadIdx.x; e < 64 * 64; e += WG) {
    const int i = m0 + e % 64, j = n0 + e / 64;
    if (i < d.M && j < d.N) {
      const double a = Ap == nullptr ? 0.0
                       : (double)(d.trans ? Ap[j + (size_t)i * d.lda] : Ap[i + (size_t)j * d.lda]);
      TC* c = Cp + i + (size_t)j * d.ldc;
      *c = (TC)(d.beta == 0.0 ? d.alpha * a : fma(d.alpha, a, d.beta * (double)*c));
    }
  }
}

// out(i, j, sum_k A(i, k) B(k, j)) for an M x N result, by 16 x 16 MFMA
// blocks spread over the waves (k advanced 16 at a time, operands loaded for
// four MFMA steps before they issue).  No barrier inside.
template <class T, class AFn, class BFn, class OFn>
__device__ void wg_mfma(int M, int N, int K, AFn A, BFn B, OFn out) {
  using V4 = typename std::conditional<std::is_same<T, float>::value, mf4, md4>::type;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int li = lane % 16, lk = lane / 16;
  const int bm = (M + 15) / 16, bn = (N + 15) / 16;
  for (int blk = w; blk < bm * bn; blk += WG / WAVE) {
    const int i0 = (blk % bm) * 16, j0 = (blk / bm) * 16;
    const int i = i0 + li, j = j0 + li;
    V4 acc = V4{0, 0, 0, 0};
    for (int k0 = 0; k0 < K; k0 += 16) {
      T av[4], bv[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = k0 + 4 * s + lk;
        av[s] = (i < M && k < K) ? A(i, k) : T(0);
        bv[s] = (j < N && k < K) ? B(k, j) : T(0);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = mfma16(av[s], bv[s], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = i0 + mfma_row(T(0), lane, r);
      if (row < M && j < N) out(row, j, acc[r]);
    }
  }
}

// X <- T X S (T: r_new x r_old or null; S: c_old x c_new, transposed when
// transS, or null) by one workgroup, Z = T X staged in LDS (rpad x rpad),
// both products on the matrix cores.
template <class T>
__device__ void xform_block(T* X, const T* Tm, const T* Sm, int r_old, int c_old, int r_new, int c_new,
                            int ldx, int ldt, int lds, int transS, T* Z, int ldz) {
  const int rz = Tm ? r_new : r_old;
  if (Tm) {
    wg_mfma<T>(r_new, c_old, r_old, [&](int i, int k) { return Tm[i + (size_t)k * ldt]; },
               [&](int k, int j) { return X[k + (size_t)j * ldx]; }, [&](int i, int j, T v) { Z[i + j * ldz] = v; });
  } else {
    for (int e = threadIdx.x; e < rz * c_old; e += WG) {
      const int i = e % rz, j = e / rz;
      Z[i + j * ldz] = X[i + (size_t)j * ldx];
    }
  }
  __syncthreads();
  if (Sm) {
    wg_mfma<T>(rz, c_new, c_old, [&](int i, int k) { return Z[i + k * ldz]; },
               [&](int k, int j) { return transS ? Sm[j + (size_t)k * lds] : Sm[k + (size_t)j * lds]; },
               [&](int i, int j, T v) { X[i + (size_t)j * ldx] = v; });
  } else {
    for (int e = threadIdx.x; e < rz * c_old; e += WG) {
      const int i = e % rz, j = e / rz;
      X[i + (size_t)j * ldx] = Z[i + j * ldz];
    }
  }
  __syncthreads();
}

// One workgroup per (cluster, window slot).
template <class T>
__global__ __launch_bounds__(WG) void k_m2l_assemble(const M2LAssemble a) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* Z = reinterpret_cast<double*>(smem);  // r_i x p2, ld rpad
  const int i = blockIdx.x, sl = blockIdx.y;
  const int ri = a.r[i];
  if (ri == 0) return;
  const int ix = demorton_x(i), iy = demorton_y(i);
  const int jx = 2 * (ix >> 1) - 2 + sl / 6, jy = 2 * (iy >> 1) - 2 + sl % 6;
  if (jx < 0 || jy < 0 || jx >= a.nside || jy >= a.nside) return;
  const int dx = jx - ix, dy = jy - iy;
  T* M = static_cast<T*>(a.M) + ((size_t)i * 36 + sl) * a.sM;
  if (abs(dx) <= 1 && abs(dy) <= 1) {  // a neighbour's slot: the fill-in accumulates there from zero
    for (size_t e = threadIdx.x; e < a.sM; e += WG) M[e] = T(0);
    return;
  }
  const int l = morton2(jx, jy);
  const int rl = a.r[l];
  if (rl == 0) return;
  const double* Ri = a.R + (size_t)i * a.sR;
  const double* Rl = a.R + (size_t)l * a.sR;
  const double* K = a.table + (size_t)((dx + 3) * 7 + (dy + 3)) * a.p2 * a.p2;
  const int p2 = a.p2, ld = a.rpad;
  wg_mfma<double>(ri, p2, p2, [&](int x, int k) { return Ri[x + (size_t)k * ld]; },
                  [&](int k, int y) { return K[k + (size_t)y * p2]; }, [&](int x, int y, double v) { Z[x + y * ld] = v; });
  __syncthreads();
  wg_mfma<double>(ri, rl, p2, [&](int x, int k) { return Z[x + k * ld]; },
                  [&](int k, int y) { return Rl[y + (size_t)k * ld]; }, [&](int x, int y, double v) { M[x + y * ld] = (T)v; });
}

// One thread per touched cluster (RankFin).
__global__ __launch_bounds__(WG) void k_rank_finalize(const RankFin a) {
  const int t = blockIdx.x * WG + threadIdx.x;
  if (t >= a.nt) return;
  const int q = a.q[t];
  const int rn = min(min(a.rank[2 * t], a.n[q]), a.r_cap);
  a.r_new[t] = rn;
  if (a.r_lvl) a.r_lvl[q] = rn;
  if (a.g) a.g[t].M = rn;
}

// One workgroup per (touch, unit of its elimination record).
template <class T>
__global__ __launch_bounds__(WG) void k_fill_copy(const FillCopy a) {
  const int t = blockIdx.x, s2 = blockIdx.y;
  if (a.touch[5 * t + 4]) return;  // its pivoted QR reads the fill blocks in place
  const int b = a.touch[5 * t], sq = a.touch[5 * t + 1], nq = a.touch[5 * t + 2], col0 = a.touch[5 * t + 3];
  const ElimRec& r = a.rec[b];
  const int pidx = a.pair[9 * sq + s2];
  if (pidx < 0 || !r.kind[s2]) return;
  int col = col0;
  for (int u = 0; u < s2; ++u)
    if (a.pair[9 * sq + u] >= 0 && r.kind[u]) col += r.size[u];
  const int w = r.size[s2];
  const T* src = static_cast<const T*>(a.F) + ((size_t)b * a.npair + pidx) * a.fpad * a.fpad;
  T* dst = static_cast<T*>(a.A) + (size_t)t * a.per + (size_t)col * a.npad;
  for (int e = threadIdx.x; e < nq * w; e += WG) {
    const int i = e % nq, j = e / nq;
    dst[i + (size_t)j * a.npad] = src[i + (size_t)j * a.fpad];
  }
}

// One workgroup per (touch, window slot); slot 36 is the parent transfer
// block, slot 37 (when Unew is given) the copy of the new basis into U.
template <class T>
__global__ __launch_bounds__(WG) void k_touch_xform(const TouchXform a) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* Z = reinterpret_cast<T*>(smem);
  const int t = blockIdx.x, sl = blockIdx.y;
  const int q = a.touch_q ? a.touch_q[t] : t;
  if (sl == 37) {  // U(q) <- Unew(t)
    const int nq = a.n[q], rn = a.r_new[t];
    const T* src = static_cast<const T*>(a.Unew) + (size_t)t * a.sU;
    T* dst = static_cast<T*>(a.U) + (size_t)q * a.sU;
    for (int e = threadIdx.x; e < nq * rn; e += WG) {
      const int i = e % nq, j = e / nq;
      dst[i + (size_t)j * a.npad] = src[i + (size_t)j * a.npad];
    }
    return;
  }
  const int rq = a.r_old[q];
  if (rq == 0) return;
  const int rn = a.r_new[t];
  const T* Tq = static_cast<const T*>(a.Tm) + (size_t)t * a.rpad * a.rpad;
  T* M = static_cast<T*>(a.M);
  if (sl == 36) {
    if (a.UP == nullptr || a.r_par == nullptr) return;
    const int rP = a.r_par[q >> 2];
    if (rP == 0) return;
    xform_block<T>(static_cast<T*>(a.UP) + (size_t)q * a.sM, Tq, nullptr, rq, rP, rn, rP, a.rpad, a.rpad, a.rpad,
                   0, Z, a.rpad);
    return;
  }
  const int qx = demorton_x(q), qy = demorton_y(q);
  const int jx = 2 * (qx >> 1) - 2 + sl / 6, jy = 2 * (qy >> 1) - 2 + sl % 6;
  if (jx < 0 || jy < 0 || jx >= a.nside || jy >= a.nside) return;
  if (abs(jx - qx) <= 1 && abs(jy - qy) <= 1) return;
  const int l = morton2(jx, jy);
  const int rl = a.r_old[l];
  if (rl == 0) return;
  const int tl = a.tidx ? a.tidx[l] : l;
  const T* Tl = tl >= 0 ? static_cast<const T*>(a.Tm) + (size_t)tl * a.rpad * a.rpad : nullptr;
  xform_block<T>(M + ((size_t)q * 36 + sl) * a.sM, Tq, Tl, rq, rl, rn, tl >= 0 ? a.r_new[tl] : rl, a.rpad, a.rpad,
                 a.rpad, 1, Z, a.rpad);
  if (tl < 0 && a.col_blocks) {
    const int ls = win_slot(jx, jy, qx, qy);
    xform_block<T>(M + ((size_t)l * 36 + ls) * a.sM, nullptr, Tq, rl, rq, rl, rn, a.rpad, a.rpad, a.rpad, 1, Z,
                   a.rpad);
  }
}

// grid (parent, 9 * 16 + 4): neighbour slot x child pair, then the 4 children's
// transfer blocks.
template <class T>
__global__ __launch_bounds__(WG) void k_transition(const TransArgs a) {
  const int P = blockIdx.x, y = blockIdx.y;
  const T* src;
  T* dst;
  int rows, cols, lds = a.rpad;
  if (y < 144) {
    const int sp = y / 16, c = (y / 4) % 4, c2 = y % 4;
    const int px = demorton_x(P), py = demorton_y(P);
    const int qx = px + sp / 3 - 1, qy = py + sp % 3 - 1;
    if (qx < 0 || qy < 0 || qx >= a.nside || qy >= a.nside) return;
    const int Q = morton2(qx, qy);
    const int ch = 4 * P + c, ch2 = 4 * Q + c2;
    rows = a.cr[ch];
    cols = a.cr[ch2];
    if (rows == 0 || cols == 0) return;
    const int sl = win_slot(demorton_x(ch), demorton_y(ch), demorton_x(ch2), demorton_y(ch2));
    src = static_cast<const T*>(a.CM) + ((size_t)ch * 36 + sl) * a.sM;
    dst = static_cast<T*>(a.P) + ((size_t)P * 9 + sp) * a.sP + a.choff[4 * P + c] +
          (size_t)a.choff[4 * Q + c2] * a.npad;
  } else {
    const int c = y - 144, ch = 4 * P + c;
    rows = a.cr[ch];
    cols = a.r_par[P];
    if (rows == 0 || cols == 0) return;
    src = static_cast<const T*>(a.CUP) + (size_t)ch * a.sM;
    dst = static_cast<T*>(a.U) + (size_t)P * a.sU + a.choff[4 * P + c];
  }
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  for (int j = w; j < cols; j += WG / WAVE)
    for (int i = lane; i < rows; i += WAVE) dst[i + (size_t)j * a.npad] = src[i + (size_t)j * lds];
}

// ------------------------------------------------------------------ SOLVE
// Four launches per colour batch, each over (record, [unit,] 64-row tile):
//   step 0: w = D_i^-1 [b_i; 0] into the work vector, b_i snapshotted;
//   step 1: unit u != 4: b_q -= P_qi w^x or c_p -= L_pi w^x; unit 4:
//           c_i += w^z;
//   step 2: r = [snapshot_i - sum_u A_u v_u; y_i] into the work vector;
//   step 3: x_i = (D_i^-1 r)^x.
// Right-hand columns in groups of SV_C (one at a time for a single right-hand
// side: NC = 1 keeps the registers of one column); the waves split the inner dimension
// and meet in LDS.  wk: per record mpad x nrhs doubles.
constexpr int SV_C = 4;

// sum_k A(row, k) X(k, c) for this lane's row, the waves splitting k;
// returns the full sums to wave 0 (acc valid there only).
template <int NC, class TA, int NT = WG, class XFn>
__device__ inline void tile_dot(const TA* __restrict__ A, size_t lda, int row, bool live, int K, XFn X, int nc,
                                double* part, double* acc) {
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  constexpr int NW = NT / WAVE;
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  if (live) {
    // eight loads of A in flight per lane before their products, the last
    // round's indices clamped and its values zeroed (no remainder loop):
    // one memory round trip per 8 NW columns
    constexpr int U = 8;
    for (int k = w; k < K; k += U * NW) {
      TA av[U];
#pragma unroll
      for (int t = 0; t < U; ++t) av[t] = A[row + (size_t)min(k + t * NW, K - 1) * lda];
#pragma unroll
      for (int t = 0; t < U; ++t) {
        const int kk = min(k + t * NW, K - 1);
        const double v = k + t * NW < K ? (double)av[t] : 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c)
          if (c < nc) acc[c] = fma(v, X(kk, c), acc[c]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) part[(w * NC + c) * WAVE + lane] = acc[c];
  __syncthreads();
  if (w == 0)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double v = part[c * WAVE + lane];
      for (int q = 1; q < NW; ++q) v += part[(q * NC + c) * WAVE + lane];
      acc[c] = v;
    }
}

// The vector a product multiplies (K values per right-hand side column) is
// staged in LDS first: every lane reads it there, not through the caches.
// One instantiation per step (each with the registers of its own step).
// NT threads per workgroup: WG, or 4 WG on colour batches of few records,
// where a row tile's inner dimension split four times finer gives each
// record more loads in flight.
template <class T, int STEP, int NC, int NT = WG>
__global__ __launch_bounds__(NT) void k_solve(const SolveArgs a, double* __restrict__ wk, int tiles) {
  constexpr int step = STEP;
  __shared__ double part[(NT / WAVE) * NC * WAVE];
  extern __shared__ __align__(16) unsigned char smem[];
  double* xs = reinterpret_cast<double*>(smem);  // [NC][mpad]
  auto stage = [&](const double* src, size_t ld, int K, int ncol) {
    __syncthreads();
    for (int e = threadIdx.x; e < K * ncol; e += NT) {
      const int k = e % K, c = e / K;
      xs[k + c * a.mpad] = src[k + c * ld];
    }
    __syncthreads();
  };
  auto XL = [&](int k, int c) { return xs[k + c * a.mpad]; };
  const int b = blockIdx.x;
  const ElimRec& r = a.rec[b];
  const int unit = blockIdx.y / tiles, tile = blockIdx.y % tiles;
  const int ni = r.ni, ri = r.ri, m = r.m;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int row = tile * WAVE + lane;
  const size_t sv = (size_t)a.npad * a.nrhs, svc = (size_t)a.rpad * a.nrhs;
  double* wb = wk + (size_t)b * a.mpad * a.nrhs;  // ld mpad
  const double* D = a.Dinv + (size_t)r.i * a.sD;
  double* snap = a.bv + ((size_t)a.nc + r.i) * sv;
  double acc[NC];
  for (int c0 = 0; c0 < a.nrhs; c0 += NC) {
    const int nc = min(NC, a.nrhs - c0);
    if (step == 0) {
      if (tile * WAVE >= m) return;
      const double* bi = a.bv + (size_t)r.i * sv + (size_t)c0 * a.npad;
      stage(bi, a.npad, ni, nc);
      tile_dot<NC, double, NT>(D, a.mpad, row, row < m, ni, XL, nc, part, acc);
      if (w == 0 && row < m)
        for (int c = 0; c < nc; ++c) wb[row + (size_t)(c0 + c) * a.mpad] = acc[c];
      if (tile == 0 && w == 1)
        for (int k = lane; k < ni; k += WAVE)
          for (int c = 0; c < nc; ++c) snap[k + (size_t)(c0 + c) * a.npad] = bi[k + (size_t)c * a.npad];
    } else if (step == 1) {
      if (!r.kind[unit]) return;
      if (unit == 4) {
        if (tile * WAVE >= ri) return;
        double* ci = a.cv + (size_t)r.i * svc + (size_t)c0 * a.rpad;
        if (w == 0 && row < ri)
          for (int c = 0; c < nc; ++c) ci[row + (size_t)c * a.rpad] += wb[ni + row + (size_t)(c0 + c) * a.mpad];
        continue;
      }
      const int cl = r.cl[unit], sz = r.size[unit];
      if (tile * WAVE >= sz) return;
      const bool part1 = r.kind[unit] == 1;
      const T* A = part1 ? static_cast<const T*>(a.P) + ((size_t)cl * 9 + (8 - unit)) * a.sP
                         : static_cast<const T*>(a.L) + ((size_t)cl * 9 + (8 - unit)) * a.sL;
      const int ld = part1 ? a.npad : a.rpad;
      stage(wb + (size_t)c0 * a.mpad, a.mpad, ni, nc);
      tile_dot<NC, T, NT>(A, ld, row, row < sz, ni, XL, nc, part, acc);
      double* tg = part1 ? a.bv + (size_t)cl * sv + (size_t)c0 * a.npad : a.cv + (size_t)cl * svc + (size_t)c0 * a.rpad;
      if (w == 0 && row < sz)
        for (int c = 0; c < nc; ++c) tg[row + (size_t)c * ld] -= acc[c];
    } else if (step == 2) {
      if (tile * WAVE >= m) return;
      if (w == 0 && row >= ni && row < m) {  // rows ni .. m-1: y_i
        const double* yi = a.cv + ((size_t)a.nc + r.i) * svc + (size_t)c0 * a.rpad;
        for (int c = 0; c < nc; ++c) wb[row + (size_t)(c0 + c) * a.mpad] = yi[row - ni + (size_t)c * a.rpad];
      }
      if (tile * WAVE >= ni) continue;
      // every neighbour's vector staged at once (unit order, column stride kst),
      // then one pass over all neighbour blocks and one reduction
      const int kst = 8 * max(a.npad, a.rpad);
      __syncthreads();
      for (int u = 0, off = 0; u < 9; ++u) {
        if (u == 4 || !r.kind[u]) continue;
        const int cl = r.cl[u], sz = r.size[u];
        const bool part1 = r.kind[u] == 1;
        const double* src = part1 ? a.bv + ((size_t)2 * a.nc + cl) * sv + (size_t)c0 * a.npad
                                  : a.cv + ((size_t)a.nc + cl) * svc + (size_t)c0 * a.rpad;
        const int lds = part1 ? a.npad : a.rpad;
        for (int e = threadIdx.x; e < sz * nc; e += NT) {
          const int k = e % sz, c = e / sz;
          xs[off + k + c * kst] = src[k + (size_t)c * lds];
        }
        off += sz;
      }
      __syncthreads();
      double tot[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) tot[c] = 0.0;
      if (row < ni) {
        for (int u = 0, off = 0; u < 9; ++u) {
          if (u == 4 || !r.kind[u]) continue;
          const int sz = r.size[u];
          const T* A = r.kind[u] == 1 ? static_cast<const T*>(a.P) + ((size_t)r.i * 9 + u) * a.sP
                                      : static_cast<const T*>(a.Qm) + ((size_t)r.i * 9 + u) * a.sQ;
          constexpr int U = 8, NW = NT / WAVE;
          for (int k = w; k < sz; k += U * NW) {
            T av[U];
#pragma unroll
            for (int t = 0; t < U; ++t) av[t] = A[row + (size_t)min(k + t * NW, sz - 1) * a.npad];
#pragma unroll
            for (int t = 0; t < U; ++t) {
              const int kk = min(k + t * NW, sz - 1);
              const double v = k + t * NW < sz ? (double)av[t] : 0.0;
#pragma unroll
              for (int c = 0; c < NC; ++c)
                if (c < nc) tot[c] = fma(v, xs[off + kk + c * kst], tot[c]);
            }
          }
          off += sz;
        }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) part[(w * NC + c) * WAVE + lane] = tot[c];
      __syncthreads();
      if (w == 0 && row < ni)
        for (int c = 0; c < nc; ++c) {
          double v = part[c * WAVE + lane];
          for (int q = 1; q < NT / WAVE; ++q) v += part[(q * NC + c) * WAVE + lane];
          wb[row + (size_t)(c0 + c) * a.mpad] = snap[row + (size_t)(c0 + c) * a.npad] - v;
        }
    } else {
      if (tile * WAVE >= ni) return;
      stage(wb + (size_t)c0 * a.mpad, a.mpad, m, nc);
      tile_dot<NC, double, NT>(D, a.mpad, row, row < ni, m, XL, nc, part, acc);
      double* xi = a.bv + ((size_t)2 * a.nc + r.i) * sv + (size_t)c0 * a.npad;
      if (w == 0 && row < ni)
        for (int c = 0; c < nc; ++c) xi[row + (size_t)c * a.npad] = acc[c];
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------------- QR
template <class T, bool kLds>
__global__ __launch_bounds__(WG) void k_qr(const QrDesc* __restrict__ descs) {
  extern __shared__ __align__(16) unsigned char smem[];
  const QrDesc d = descs[blockIdx.x];
  const int n = d.n, m = d.m, K = min(n, m);
  if (d.A == nullptr || K == 0 || K > kMaxRank) return;
  T* gA = static_cast<T*>(d.A);
  T* R = static_cast<T*>(d.R);
  // staged in LDS (stride n + 1) or worked on in place
  const size_t lda = kLds ? (size_t)n + 1 : (size_t)d.lda;
  T* A = kLds ? reinterpret_cast<T*>(smem) : gA;
  if (kLds) {
    for (int e = threadIdx.x; e < n * m; e += WG) {
      const int i = e % n, c = e / n;
      A[i + c * lda] = gA[i + (size_t)c * d.lda];
    }
    __syncthreads();
  }
  __shared__ T red[WG / WAVE];
  __shared__ T tau_s[kMaxRank], alpha_s[kMaxRank];
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE, nw = WG / WAVE;
  for (int j = 0; j < K; ++j) {
    T part = 0;
    for (int i = j + threadIdx.x; i < n; i += WG) part += A[i + j * lda] * A[i + j * lda];
    const T nrm = sqrt(block_sum(part, red));
    const T x0 = A[j + j * lda];
    T alpha = 0, tau = 0, v0 = 1;
    if (nrm > 0) {
      alpha = x0 >= 0 ? -nrm : nrm;
      v0 = x0 - alpha;
      tau = -v0 / alpha;
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < n; i += WG) A[i + j * lda] = nrm > 0 ? A[i + j * lda] / v0 : T(0);
    if (threadIdx.x == 0) { tau_s[j] = tau; alpha_s[j] = alpha; }
    __syncthreads();
    for (int c = j + 1 + w; c < m; c += nw) {
      T s = 0;
      for (int i = j + 1 + lane; i < n; i += WAVE) s += A[i + j * lda] * A[i + c * lda];
      s = wave_sum(s) + A[j + c * lda];
      const T ts = tau * s;
      for (int i = j + 1 + lane; i < n; i += WAVE) A[i + c * lda] -= ts * A[i + j * lda];
      if (lane == 0) A[j + c * lda] -= ts;
    }
    __syncthreads();
    // row j of R is final now
    for (int c = threadIdx.x; c < m; c += WG)
      R[j + (size_t)c * d.ldr] = c < j ? T(0) : (c == j ? alpha : A[j + c * lda]);
    __syncthreads();
  }
  // form Q in place (backward accumulation)
  for (int j = K - 1; j >= 0; --j) {
    const T tau = tau_s[j];
    for (int c = j + 1 + w; c < K; c += nw) {
      T s = 0;
      for (int i = j + 1 + lane; i < n; i += WAVE) s += A[i + j * lda] * A[i + c * lda];
      s = wave_sum(s) + A[j + c * lda];
      const T ts = tau * s;
      for (int i = j + 1 + lane; i < n; i += WAVE) A[i + c * lda] -= ts * A[i + j * lda];
      if (lane == 0) A[j + c * lda] -= ts;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += WG) {
      T v;
      if (i < j) v = 0;
      else if (i == j) v = 1 - tau;
      else v = -tau * A[i + j * lda];
      A[i + j * lda] = v;
    }
    __syncthreads();
  }
  // sign normalisation: R_jj >= 0
  for (int j = 0; j < K; ++j) {
    if (alpha_s[j] < 0) {
      for (int i = threadIdx.x; i < n; i += WG) A[i + j * lda] = -A[i + j * lda];
      for (int c = j + threadIdx.x; c < m; c += WG) R[j + (size_t)c * d.ldr] = -R[j + (size_t)c * d.ldr];
    }
  }
  if (kLds) {
    __syncthreads();
    for (int e = threadIdx.x; e < n * K; e += WG) {
      const int i = e % n, c = e / n;
      gA[i + (size_t)c * d.lda] = A[i + c * lda];
    }
  }
}

// The same factorisation with one wave per matrix for m <= 64 columns and
// n <= NR rows: lane c holds column c in registers.  Step j: lane j publishes
// its column; the wave forms the reflector (the norm by a butterfly sum, so
// every lane holds the same value) and keeps it in LDS for Q; every column
// right of j takes x - tau (u^T x) u.  Row j of column c is final after step
// j, so R is written from the registers at the end; Q = H_0 ... H_{K-1}
// [I_K; 0] is formed column by column from the LDS reflectors.  Same
// reflector convention and sign normalisation as k_qr.
template <class T, int NR>
__global__ __launch_bounds__(WAVE) void k_qr_wave(const QrDesc* __restrict__ descs) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* refl = reinterpret_cast<T*>(smem);  // [K][NR]
  __shared__ T xs[NR];
  __shared__ T tau_s[WAVE], alpha_s[WAVE];
  const QrDesc d = descs[blockIdx.x];
  const int n = d.n, m = d.m, K = min(n, m);
  if (d.A == nullptr || K == 0 || m > WAVE || n > NR) return;
  T* gA = static_cast<T*>(d.A);
  T* R = static_cast<T*>(d.R);
  const size_t lda = d.lda;
  const int c = threadIdx.x;
  const bool live = c < m;
  T col[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) col[i] = (live && i < n) ? gA[i + (size_t)c * lda] : T(0);
  for (int j = 0; j < K; ++j) {
    if (c == j) {
#pragma unroll
      for (int i = 0; i < NR; ++i) xs[i] = col[i];
    }
    __syncthreads();
    T part = 0;
    for (int i = c; i < n; i += WAVE)
      if (i >= j) part = fma(xs[i], xs[i], part);
    const T nrm = sqrt(wave_sum(part));
    const T x0 = xs[j];
    T alpha = 0, tau = 0, v0 = 1;
    if (nrm > 0) {
      alpha = x0 >= 0 ? -nrm : nrm;
      v0 = x0 - alpha;
      tau = -v0 / alpha;
    }
    for (int i = c; i < NR; i += WAVE)
      refl[j * NR + i] = i < j ? T(0) : i == j ? T(1) : (i < n && nrm > 0 ? xs[i] / v0 : T(0));
    if (c == 0) {
      tau_s[j] = tau;
      alpha_s[j] = alpha;
    }
    __syncthreads();
    if (live && c > j) {
      const T* u = refl + j * NR;
      T sa = 0, sb = 0;
#pragma unroll
      for (int i = 0; i < NR; i += 2) {
        sa = fma(u[i], col[i], sa);
        if (i + 1 < NR) sb = fma(u[i + 1], col[i + 1], sb);
      }
      const T ts = tau * (sa + sb);
      asm volatile("" ::: "memory");  // read u again below instead of holding NR more registers
#pragma unroll
      for (int i = 0; i < NR; ++i) col[i] = fma(-ts, u[i], col[i]);
    }
  }
  // R (K x m), rows with a negative alpha negated
  if (live) {
    T* Rc = R + (size_t)c * d.ldr;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      if (i < K) {
        const T v = i < c ? col[i] : (i == c ? alpha_s[c] : T(0));
        Rc[i] = alpha_s[i] < 0 ? -v : v;
      }
    }
  }
  if (c >= K) return;
#pragma unroll
  for (int i = 0; i < NR; ++i) col[i] = i == c ? T(1) : T(0);
  for (int jj = K - 1; jj >= 0; --jj) {
    const T* u = refl + jj * NR;
    T sa = 0, sb = 0;
#pragma unroll
    for (int i = 0; i < NR; i += 2) {
      sa = fma(u[i], col[i], sa);
      if (i + 1 < NR) sb = fma(u[i + 1], col[i + 1], sb);
    }
    const T ts = tau_s[jj] * (sa + sb);
    asm volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i < NR; ++i) col[i] = fma(-ts, u[i], col[i]);
    asm volatile("" ::: "memory");
  }
  const T sg = alpha_s[c] < 0 ? T(-1) : T(1);
  T* Qc = gA + (size_t)c * lda;
#pragma unroll
  for (int i = 0; i < NR; ++i)
    if (i < n) Qc[i] = sg * col[i];
}

// ------------------------------------------------------------------- RRQR
// The whole matrix is staged in LDS (stride n + 1), or worked on in place.
// Each column of the trailing matrix is handled by a group of 16 lanes (16
// consecutive rows per access), two columns at a time where registers
// allow, so a workgroup has 64 or more columns in flight; dot products and
// norms reduce with shuffles inside the group.  Norms are recomputed exactly
// every step, so the pivot's norm over rows j.. is the pivot value itself.
// A step costs three barriers: the pivot search, the column swap (with the
// previous reflector's column scaled to u = x / v0 and alpha put on its
// diagonal: no thread reads it any more), and the update, which works from
// the unscaled x with 1 / v0 folded into its scalars.
template <class T, int IL, int NV>
__device__ inline void rrqr_update_cols(T* A, size_t lda, T* nrm, int n, int m, int j, T tau, T iv0, int rl,
                                        int slot, int nslot) {
  const T* x = A + j * lda;
  T ur[NV];
#pragma unroll
  for (int t = 0; t < NV; ++t) {
    const int i = j + 1 + rl + GRP * t;
    ur[t] = i < n ? x[i] : T(0);
  }
  int c = j + 1 + slot;
  for (; IL == 2 && c + nslot < m; c += 2 * nslot) {
    T* ca = A + c * lda;
    T* cb = A + (c + nslot) * lda;
    T va[NV], vb[NV];
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      const int i = j + 1 + rl + GRP * t;
      va[t] = i < n ? ca[i] : T(0);
      vb[t] = i < n ? cb[i] : T(0);
    }
    T sa0 = 0, sa1 = 0, sb0 = 0, sb1 = 0;
#pragma unroll
    for (int t = 0; t < NV; t += 2) {
      sa0 = fma(ur[t], va[t], sa0);
      sa1 = fma(ur[t + 1], va[t + 1], sa1);
      sb0 = fma(ur[t], vb[t], sb0);
      sb1 = fma(ur[t + 1], vb[t + 1], sb1);
    }
    const T tsa = tau * fma(grp_sum(sa0 + sa1), iv0, ca[j]);
    const T tsb = tau * fma(grp_sum(sb0 + sb1), iv0, cb[j]);
    const T ua = tsa * iv0, ub = tsb * iv0;
    T qa0 = 0, qa1 = 0, qb0 = 0, qb1 = 0;
#pragma unroll
    for (int t = 0; t < NV; t += 2) {
      const int i0 = j + 1 + rl + GRP * t, i1 = i0 + GRP;
      const T a0 = fma(-ua, ur[t], va[t]), a1 = fma(-ua, ur[t + 1], va[t + 1]);
      const T b0 = fma(-ub, ur[t], vb[t]), b1 = fma(-ub, ur[t + 1], vb[t + 1]);
      if (i0 < n) {
        ca[i0] = a0;
        cb[i0] = b0;
      }
      if (i1 < n) {
        ca[i1] = a1;
        cb[i1] = b1;
      }
      qa0 = fma(a0, a0, qa0);
      qa1 = fma(a1, a1, qa1);
      qb0 = fma(b0, b0, qb0);
      qb1 = fma(b1, b1, qb1);
    }
    const T qa = grp_sum(qa0 + qa1), qb = grp_sum(qb0 + qb1);
    if (rl == 0) {
      ca[j] -= tsa;
      cb[j] -= tsb;
      nrm[c] = sqrt(qa);
      nrm[c + nslot] = sqrt(qb);
    }
  }
  for (; c < m; c += nslot) {
    T* col = A + c * lda;
    T cv[NV];
#pragma unroll
    for (int t = 0; t < NV; ++t) {
      const int i = j + 1 + rl + GRP * t;
      cv[t] = i < n ? col[i] : T(0);
    }
    T s0 = 0, s1 = 0;
#pragma unroll
    for (int t = 0; t < NV; t += 2) {
      s0 = fma(ur[t], cv[t], s0);
      s1 = fma(ur[t + 1], cv[t + 1], s1);
    }
    const T ts = tau * fma(grp_sum(s0 + s1), iv0, col[j]);
    const T us = ts * iv0;
    T q0 = 0, q1 = 0;
#pragma unroll
    for (int t = 0; t < NV; t += 2) {
      const int i0 = j + 1 + rl + GRP * t, i1 = i0 + GRP;
      const T v0 = fma(-us, ur[t], cv[t]);
      const T v1 = fma(-us, ur[t + 1], cv[t + 1]);
      if (i0 < n) col[i0] = v0;
      if (i1 < n) col[i1] = v1;
      q0 = fma(v0, v0, q0);
      q1 = fma(v1, v1, q1);
    }
    const T q = grp_sum(q0 + q1);
    if (rl == 0) {
      col[j] -= ts;
      nrm[c] = sqrt(q);
    }
  }
}

template <class T, int NT, bool kLds, int NV>
__global__ __launch_bounds__(NT) void k_rrqr(const RrqrDesc* __restrict__ descs) {
  extern __shared__ __align__(16) unsigned char smem[];
  const RrqrDesc d = descs[blockIdx.x];
  const int n = d.n, m = d.m;
  const int K = min(min(n, m), d.kmax);
  if (d.A == nullptr) return;
  T* gA = static_cast<T*>(d.A);
  T* gtau = static_cast<T*>(d.tau);
  T* galpha = static_cast<T*>(d.alpha);
  // staged in LDS (stride n + 1), or worked on in place (L2-resident) with
  // only the column norms in LDS
  const size_t lda = kLds ? (size_t)n + 1 : (size_t)d.lda;
  T* A = kLds ? reinterpret_cast<T*>(smem) : gA;
  T* nrm = kLds ? A + lda * m : reinterpret_cast<T*>(smem);
  if (kLds)
    for (int e = threadIdx.x; e < n * m; e += NT) {
      const int i = e % n, c = e / n;
      A[i + c * lda] = gA[i + (size_t)c * d.lda];
    }
  constexpr int NW = NT / WAVE;
  __shared__ T rv[2][NW];
  __shared__ int ri[2][NW];
  const int rl = threadIdx.x % GRP;         // row lane inside the group
  const int slot = threadIdx.x / GRP;       // column slot of the group
  constexpr int NSLOT = NT / GRP;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  for (int c = slot; c < m; c += NSLOT) {
    const T* col = A + c * lda;
    T q = 0;
    for (int i = rl; i < n; i += GRP) q = fma(col[i], col[i], q);
    q = grp_sum(q);
    if (rl == 0) nrm[c] = sqrt(q);
  }
  __syncthreads();
  int rank = 0, steps = K;
  bool counting = true;
  T first = 0;
  // column j - 1 below its diagonal still holds x: scaled by 1 / v0 (0 for
  // a zero column), alpha on the diagonal
  auto finish = [&](int jp, T v0, T alpha, bool zero) {
    T* col = A + jp * lda;
    for (int i = jp + 1 + threadIdx.x; i < n; i += NT) col[i] = zero ? T(0) : col[i] / v0;
    if (threadIdx.x == 0) col[jp] = alpha;
  };
  T pv0 = 1, palpha = 0;
  bool pzero = true;
  for (int j = 0; j < K; ++j) {
    T bv = -1;
    int bi = m;
    for (int c = j + threadIdx.x; c < m; c += NT)
      if (nrm[c] > bv || (nrm[c] == bv && c < bi)) { bv = nrm[c]; bi = c; }
    for (int o = WAVE / 2; o > 0; o >>= 1) {
      const T ov = __shfl_xor(bv, o, WAVE);
      const int oi = __shfl_xor(bi, o, WAVE);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    // the buffers alternate between steps: the previous step's readers are
    // past the barrier that ended that step
    if (lane == 0) { rv[j & 1][w] = bv; ri[j & 1][w] = bi; }
    __syncthreads();
    T piv = rv[j & 1][0];
    int cp = ri[j & 1][0];
    for (int q = 1; q < NW; ++q) {
      const T v = rv[j & 1][q];
      const int i = ri[j & 1][q];
      if (v > piv || (v == piv && i < cp)) { piv = v; cp = i; }
    }
    if (j == 0) first = piv;
    if (counting && first > 0 && (double)piv > d.eps * (double)first) rank = j + 1;
    else counting = false;
    if (!counting && d.stop_at_rank) {  // uniform: every thread holds the same pivot
      steps = j;
      break;
    }
    if (j > 0) finish(j - 1, pv0, palpha, pzero);
    if (cp != j) {
      for (int i = threadIdx.x; i < n; i += NT) {
        const T t = A[i + j * lda];
        A[i + j * lda] = A[i + cp * lda];
        A[i + cp * lda] = t;
      }
      if (threadIdx.x == 0) { const T t = nrm[j]; nrm[j] = nrm[cp]; nrm[cp] = t; }
    }
    __syncthreads();
    const T xn = piv;
    const T x0 = A[j + j * lda];
    T alpha = 0, tau = 0, v0 = 1, iv0 = 0;
    if (xn > 0) {
      alpha = x0 >= 0 ? -xn : xn;
      v0 = x0 - alpha;
      tau = -v0 / alpha;
      iv0 = T(1) / v0;
    }
    if (threadIdx.x == 0) { gtau[j] = tau; galpha[j] = alpha; }
    if constexpr (NV > 0) {
      // n <= GRP NV: this lane's rows of x and of each column it updates
      // stay in registers (one read and one write of the trailing matrix per
      // step)
      constexpr int IL = sizeof(T) * NV <= 64 ? 2 : 1;  // two columns' rows and addresses fit the registers
      rrqr_update_cols<T, IL, NV>(A, lda, nrm, n, m, j, tau, iv0, rl, slot, NSLOT);
    } else {
      const T* x = A + j * lda;
      for (int c = j + 1 + slot; c < m; c += NSLOT) {
        T* col = A + c * lda;
        // two independent partial sums per lane (short, latency-bound loops)
        T s0 = 0, s1 = 0;
        int i = j + 1 + rl;
        for (; i + GRP < n; i += 2 * GRP) {
          s0 = fma(x[i], col[i], s0);
          s1 = fma(x[i + GRP], col[i + GRP], s1);
        }
        if (i < n) s0 = fma(x[i], col[i], s0);
        const T ts = tau * fma(grp_sum(s0 + s1), iv0, col[j]);
        const T us = ts * iv0;
        T q0 = 0, q1 = 0;
        i = j + 1 + rl;
        for (; i + GRP < n; i += 2 * GRP) {
          const T v0 = fma(-us, x[i], col[i]);
          const T v1 = fma(-us, x[i + GRP], col[i + GRP]);
          col[i] = v0;
          col[i + GRP] = v1;
          q0 = fma(v0, v0, q0);
          q1 = fma(v1, v1, q1);
        }
        if (i < n) {
          const T v0 = fma(-us, x[i], col[i]);
          col[i] = v0;
          q0 = fma(v0, v0, q0);
        }
        const T q = grp_sum(q0 + q1);
        if (rl == 0) {
          col[j] -= ts;
          nrm[c] = sqrt(q);
        }
      }
    }
    pv0 = v0;
    palpha = alpha;
    pzero = !(xn > 0);
    __syncthreads();
  }
  if (steps > 0) finish(steps - 1, pv0, palpha, pzero);
  if (kLds) {
    __syncthreads();
    for (int e = threadIdx.x; e < n * steps; e += NT) {
      const int i = e % n, c = e / n;
      gA[i + (size_t)c * d.lda] = A[i + c * lda];
    }
  }
  if (threadIdx.x == 0) { *d.rank = rank; *d.steps = steps; }
}

// Pivoted QR with each column of the matrix in the registers of one thread
// (m <= blockDim.x columns, n <= NR rows), then Q.  Step j: the remaining
// column with the largest norm over rows j..n-1 (the first on ties) is the
// pivot; its thread publishes the column and its wave forms the reflector
// u = (0, 1, x_{j+1:} / v0) with alpha = -sign(x_j) ||x_{j:}||, v0 = x_j - alpha,
// tau = -v0 / alpha, keeps it in LDS (for the update and for Q) and writes it
// to column j of A (alpha on the diagonal) with tau and alpha.  Every other
// remaining column takes x - tau (u^T x) u and its new trailing norm.  The
// steps stop at the first pivot norm <= eps times the first one (the rank).
// Q = H_0 ... H_{kk-1} [I_r; 0] (kk = min(r, steps)), column j negated where
// alpha_j < 0, is formed by the threads of its columns from the LDS
// reflectors.
// FILL: the instantiations that may read a touch's fill columns in place
// (FP32 columns of up to 96 rows; the others keep the plain column loads,
// whose register allocation their main loop runs best with).  FP32 columns
// of 96 rows are held to 168 registers, three waves per SIMD.
template <class T, int NR>
constexpr bool kRrqrFill = sizeof(T) == 4 && NR <= 96;
template <class T, int NR>
__global__ __launch_bounds__(512, (sizeof(T) == 4 && NR == 96) ? 3 : 1) void k_rrqr_reg(
    const RrqrDesc* __restrict__ descs, const FillCopy fc) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ T xs[NR], mk[NR];
  __shared__ T tau_s[kMaxRank], alpha_s[kMaxRank];
  __shared__ T part_v[512 / WAVE];
  __shared__ int part_i[512 / WAVE];
  const RrqrDesc d = descs[blockIdx.x];
  const int n = d.n, m = d.m;
  const int K = min(min(n, m), min(d.kmax, kMaxRank));
  if (d.A == nullptr) return;
  T* refl = reinterpret_cast<T*>(smem);  // [K][NR]
  T* gA = static_cast<T*>(d.A);
  T* gtau = static_cast<T*>(d.tau);
  T* galpha = static_cast<T*>(d.alpha);
  const size_t lda = d.lda;
  const int c = threadIdx.x, lane = c % WAVE, w = c / WAVE, nw = blockDim.x / WAVE;
  const bool live = c < m;
  T col[NR];
  // FP64 columns of more than 64 rows leave few registers beside them: a
  // compiler barrier every CH rows keeps the LDS reads of u from being
  // hoisted ahead of their FMAs all at once
  constexpr int CH = (sizeof(T) == 8 && NR > 64) ? 16 : NR;
  // column c: from A, or (fill_t >= 0, c >= col0) from the fill block of the
  // unit it belongs to, as the fill copy would have placed it
  const T* src = gA + (size_t)c * lda;
  if (kRrqrFill<T, NR> && live && d.fill_t >= 0 && fc.touch) {
    const int* tc = fc.touch + 5 * d.fill_t;
    const int b = tc[0], sq = tc[1], col0 = tc[3];
    if (c >= col0) {
      const ElimRec& r = fc.rec[b];
      src = nullptr;
      int cs = col0;
      for (int u = 0; u < 9; ++u) {
        const int pidx = fc.pair[9 * sq + u];
        if (pidx < 0 || !r.kind[u]) continue;
        if (c < cs + r.size[u]) {
          src = static_cast<const T*>(fc.F) + ((size_t)b * fc.npair + pidx) * fc.fpad * fc.fpad +
                (size_t)(c - cs) * fc.fpad;
          break;
        }
        cs += r.size[u];
      }
    }
  }
  T q0 = 0;
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    col[i] = (live && src && i < n) ? src[i] : T(0);
    q0 = fma(col[i], col[i], q0);
  }
  T nrm = sqrt(q0);
  bool done = !live;
  int rank = 0, steps = K;
  bool counting = true;
  T first = 0;
  for (int j = 0; j < K; ++j) {
    T bv = done ? T(-1) : nrm;
    int bi = done ? m : c;
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
      const T ov = __shfl_xor(bv, o, WAVE);
      const int oi = __shfl_xor(bi, o, WAVE);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      part_v[w] = bv;
      part_i[w] = bi;
    }
    __syncthreads();
    T piv = part_v[0];
    int cp = part_i[0];
    for (int q = 1; q < nw; ++q) {
      const T v = part_v[q];
      const int i = part_i[q];
      if (v > piv || (v == piv && i < cp)) {
        piv = v;
        cp = i;
      }
    }
    if (j == 0) first = piv;
    if (counting && first > 0 && (double)piv > d.eps * (double)first) rank = j + 1;
    else counting = false;
    if ((!counting && d.stop_at_rank) || cp >= m) {  // uniform
      steps = j;
      break;
    }
    if (w == cp / WAVE) {  // the pivot column's wave forms the reflector
      if (c == cp) {
#pragma unroll
        for (int i = 0; i < NR; ++i) xs[i] = col[i];
        done = true;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // the pivot's norm over rows j.. is the pivot value itself
      const T xn = piv;
      const T x0 = xs[j];
      T alpha = 0, tau = 0, iv = 0;
      if (xn > 0) {
        alpha = x0 >= 0 ? -xn : xn;
        const T v0 = x0 - alpha;
        tau = -v0 / alpha;
        iv = T(1) / v0;
      }
      for (int i = lane; i < NR; i += WAVE) {
        const T u = i < j ? T(0) : i == j ? T(1) : (i < n ? xs[i] * iv : T(0));
        refl[j * NR + i] = u;
        mk[i] = i > j ? T(1) : T(0);
        if (i > j && i < n) gA[i + (size_t)j * lda] = u;
      }
      if (lane == 0) {
        tau_s[j] = tau;
        alpha_s[j] = alpha;
        gA[j + (size_t)j * lda] = alpha;
        gtau[j] = tau;
        galpha[j] = alpha;
      }
    }
    __syncthreads();
    if (!done) {
      const T* u = refl + j * NR;
      const T tau = tau_s[j];
      T sa = 0, sb = 0;
#pragma unroll
      for (int i = 0; i < NR; i += 2) {
        sa = fma(u[i], col[i], sa);
        if (i + 1 < NR) sb = fma(u[i + 1], col[i + 1], sb);
        if ((i + 2) % CH == 0 && i + 2 < NR) asm volatile("" ::: "memory");
      }
      const T ts = tau * (sa + sb);
      // read u again from LDS below instead of holding NR more registers
      asm volatile("" ::: "memory");
      T qa = 0, qb = 0;
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        col[i] = fma(-ts, u[i], col[i]);
        const T v = col[i] * mk[i];
        if (i & 1) qb = fma(v, col[i], qb);
        else qa = fma(v, col[i], qa);
        if ((i + 1) % CH == 0 && i + 1 < NR) asm volatile("" ::: "memory");
      }
      nrm = sqrt(qa + qb);
    }
  }
  if (threadIdx.x == 0) {
    *d.rank = rank;
    *d.steps = steps;
  }
  if (d.Q == nullptr) return;
  const int r = min(rank, d.kmax), kk = min(r, steps);
  __syncthreads();
  if (c < r) {
#pragma unroll
    for (int i = 0; i < NR; ++i) col[i] = i == c ? T(1) : T(0);
    for (int jj = kk - 1; jj >= 0; --jj) {
      const T* u = refl + jj * NR;
      T sa = 0, sb = 0;
#pragma unroll
      for (int i = 0; i < NR; i += 2) {
        sa = fma(u[i], col[i], sa);
        if (i + 1 < NR) sb = fma(u[i + 1], col[i + 1], sb);
        if ((i + 2) % CH == 0 && i + 2 < NR) asm volatile("" ::: "memory");
      }
      const T ts = tau_s[jj] * (sa + sb);
      asm volatile("" ::: "memory");
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        col[i] = fma(-ts, u[i], col[i]);
        if ((i + 1) % CH == 0 && i + 1 < NR) asm volatile("" ::: "memory");
      }
      asm volatile("" ::: "memory");
    }
    const T sg = (c < kk && alpha_s[c] < 0) ? T(-1) : T(1);
    T* Q = static_cast<T*>(d.Q) + (size_t)c * d.ldq;
#pragma unroll
    for (int i = 0; i < NR; ++i)
      if (i < n) Q[i] = sg * col[i];
  }
}

// Q of a pivoted QR done by k_rrqr (rank and steps read on the device):
// the kk reflectors are staged in LDS, then each column of Q is formed by G
// consecutive lanes holding NR rows each (rows g NR .. g NR + NR - 1), the
// products with the reflectors reduced over the G lanes.  No barrier after
// the staging.
template <class T, int NR, int G>
__global__ __launch_bounds__(512) void k_formq_rr(const RrqrDesc* __restrict__ descs) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* refl = reinterpret_cast<T*>(smem);  // [kk][G NR]
  __shared__ T tau_s[kMaxRank];
  __shared__ int neg_s[kMaxRank];
  constexpr int LD = G * NR;
  const RrqrDesc dd = descs[blockIdx.x];
  if (dd.Q == nullptr) return;
  const int r = min(min(*dd.rank, dd.kmax), kMaxRank), kk = min(r, *dd.steps);
  if (r <= 0) return;
  const int n = dd.n;
  const size_t lda = dd.lda, ldq = dd.ldq;
  const T* A = static_cast<const T*>(dd.A);
  for (int e = threadIdx.x; e < kk * LD; e += blockDim.x) {
    const int i = e % LD, j = e / LD;
    refl[e] = i < j || i >= n ? T(0) : i == j ? T(1) : A[i + (size_t)j * lda];
  }
  for (int j = threadIdx.x; j < kk; j += blockDim.x) {
    tau_s[j] = static_cast<const T*>(dd.tau)[j];
    neg_s[j] = static_cast<const T*>(dd.alpha)[j] < 0;
  }
  __syncthreads();
  const int g = threadIdx.x % G;
  T* Q = static_cast<T*>(dd.Q);
  for (int c = threadIdx.x / G; c < r; c += blockDim.x / G) {
    T q[NR];
#pragma unroll
    for (int t = 0; t < NR; ++t) q[t] = g * NR + t == c ? T(1) : T(0);
    for (int j = kk - 1; j >= 0; --j) {
      const T* u = refl + (size_t)j * LD + g * NR;
      T sa = 0;
#pragma unroll
      for (int t = 0; t < NR; ++t) sa = fma(u[t], q[t], sa);
#pragma unroll
      for (int o = 1; o < G; o <<= 1) sa += __shfl_xor(sa, o, WAVE);
      const T ts = tau_s[j] * sa;
      asm volatile("" ::: "memory");
#pragma unroll
      for (int t = 0; t < NR; ++t) q[t] = fma(-ts, u[t], q[t]);
      asm volatile("" ::: "memory");
    }
    const T sg = (c < kk && neg_s[c]) ? T(-1) : T(1);
#pragma unroll
    for (int t = 0; t < NR; ++t) {
      const int i = g * NR + t;
      if (i < n) Q[i + (size_t)c * ldq] = sg * q[t];
    }
  }
}

// The same for matrices whose reflectors do not fit in LDS: reflectors read
// from the matrix in place, one wave per column.
template <class T>
__global__ __launch_bounds__(WG) void k_formq_rr_glb(const RrqrDesc* __restrict__ descs) {
  const RrqrDesc dd = descs[blockIdx.x];
  if (dd.Q == nullptr) return;
  const int r = min(*dd.rank, dd.kmax), kk = min(r, *dd.steps);
  if (r <= 0) return;
  const int n = dd.n;
  const size_t lda = dd.lda, ldq = dd.ldq;
  const T* A = static_cast<const T*>(dd.A);
  const T* tauv = static_cast<const T*>(dd.tau);
  const T* alphav = static_cast<const T*>(dd.alpha);
  T* Q = static_cast<T*>(dd.Q);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE, nw = WG / WAVE;
  for (int e = threadIdx.x; e < n * r; e += WG) {
    const int i = e % n, j = e / n;
    Q[i + j * ldq] = i == j ? T(1) : T(0);
  }
  __syncthreads();
  for (int j = kk - 1; j >= 0; --j) {
    const T tau = tauv[j];
    for (int c = j + w; c < r; c += nw) {
      T s = 0;
      for (int i = j + 1 + lane; i < n; i += WAVE) s += A[i + j * lda] * Q[i + c * ldq];
      s = wave_sum(s) + Q[j + c * ldq];
      const T ts = tau * s;
      for (int i = j + 1 + lane; i < n; i += WAVE) Q[i + c * ldq] -= ts * A[i + j * lda];
      if (lane == 0) Q[j + c * ldq] -= ts;
    }
    __syncthreads();
  }
  for (int j = 0; j < kk && j < r; ++j)
    if (alphav[j] < 0)
      for (int i = threadIdx.x; i < n; i += WG) Q[i + j * ldq] = -Q[i + j * ldq];
}

// --------------------------------------------------------------- STACK QR
// R of a tall stack [B_0; B_1; ...] processed block by block: the running R
// (r x r) and a chunk of the current block live in LDS.  A Householder step
// only touches row j of R and the chunk rows.  Each trailing column is handled
// by a 16-lane group (lanes over chunk rows, shuffle reductions), every group
// forms the reflector of column j itself, so a step costs one barrier.
template <class T, class BlockFn>
__device__ void stackqr_body(T* lds, int r, int nblk, BlockFn block, int chunk, T* Rout, size_t ldr) {
  const int ldc = chunk + 1;
  T* R = lds;          // r x r, ld r
  T* C = R + r * r;    // chunk x r, ld chunk + 1
  const int rl = threadIdx.x % GRP, slot = threadIdx.x / GRP;
  constexpr int NSLOT = WG / GRP;
  for (int e = threadIdx.x; e < r * r; e += WG) R[e] = 0;
  __syncthreads();
  // The chunk is filled with consecutive rows of the stack, across block
  // boundaries, so each r-step Householder sweep covers up to `chunk` rows.
  int b = 0, off = 0;
  while (b < nblk) {
    int cr = 0;
    while (b < nblk && cr < chunk) {
      const BlkRef B = block(b);
      const T* Bp = static_cast<const T*>(B.p);
      const int take = min(chunk - cr, B.rows - off);
      for (int e = threadIdx.x; e < take * r; e += WG) {
        int i, j;
        if (B.trans) { j = e % r; i = e / r; } else { i = e % take; j = e / take; }
        const int gi = off + i;
        C[cr + i + j * ldc] = B.trans ? Bp[j + (size_t)gi * B.ld] : Bp[gi + (size_t)j * B.ld];
      }
      cr += take;
      off += take;
      if (off >= B.rows) {
        ++b;
        off = 0;
      }
    }
    __syncthreads();
    {
      for (int j = 0; j < r; ++j) {
        const T* cj = C + j * ldc;
        // four independent partial sums per lane: the LDS loads of one
        // iteration do not wait for the previous fma
        T p0 = 0, p1 = 0, p2 = 0, p3 = 0;
        int i = rl;
        for (; i + 3 * GRP < cr; i += 4 * GRP) {
          p0 = fma(cj[i], cj[i], p0);
          p1 = fma(cj[i + GRP], cj[i + GRP], p1);
          p2 = fma(cj[i + 2 * GRP], cj[i + 2 * GRP], p2);
          p3 = fma(cj[i + 3 * GRP], cj[i + 3 * GRP], p3);
        }
        for (; i < cr; i += GRP) p0 = fma(cj[i], cj[i], p0);
        T s2 = grp_sum((p0 + p1) + (p2 + p3));
        const T rjj = R[j + j * r];
        const T nrm = sqrt(rjj * rjj + s2);
        if (s2 == 0 || nrm == 0) continue;  // nothing below the diagonal: H = I
        // H = I - tau u u^T with u = [1; C_j / v0], tau = -v0 / alpha in [1, 2]:
        // no product of two small quantities is formed, so repeated stacking of
        // nearly annihilated columns cannot overflow the scale.
        const T alpha = rjj >= 0 ? -nrm : nrm;
        const T v0 = rjj - alpha;
        const T tau = -v0 / alpha;
        const T iv0 = T(1) / v0;
        for (int c = j + 1 + slot; c < r; c += NSLOT) {
          T* cc = C + c * ldc;
          T q0 = 0, q1 = 0, q2 = 0, q3 = 0;
          int i = rl;
          for (; i + 3 * GRP < cr; i += 4 * GRP) {
            q0 = fma(cj[i], cc[i], q0);
            q1 = fma(cj[i + GRP], cc[i + GRP], q1);
            q2 = fma(cj[i + 2 * GRP], cc[i + 2 * GRP], q2);
            q3 = fma(cj[i + 3 * GRP], cc[i + 3 * GRP], q3);
          }
          for (; i < cr; i += GRP) q0 = fma(cj[i], cc[i], q0);
          const T rjc = R[j + c * r];
          const T sc = tau * (grp_sum((q0 + q1) + (q2 + q3)) * iv0 + rjc);
          const T su = sc * iv0;
#pragma unroll 4
          for (int i2 = rl; i2 < cr; i2 += GRP) cc[i2] = fma(-su, cj[i2], cc[i2]);
          if (rl == 0) R[j + c * r] = rjc - sc;
        }
        __syncthreads();  // trailing columns final; R_jj and column j no longer read
        if (threadIdx.x == 0) R[j + j * r] = alpha;
      }
      __syncthreads();
    }
  }
  for (int e = threadIdx.x; e < r * r; e += WG) {
    const int i = e % r, j = e / r;
    T v = j < i ? T(0) : R[i + j * r];
    if (R[i + i * r] < 0) v = -v;
    Rout[i + (size_t)j * ldr] = v;
  }
}

template <class T>
__global__ __launch_bounds__(WG) void k_stackqr(const StackQrDesc* __restrict__ descs,
                                                const BlkRef* __restrict__ blocks, int chunk) {
  extern __shared__ __align__(16) unsigned char smem[];
  const StackQrDesc d = descs[blockIdx.x];
  if (d.R == nullptr || d.r == 0) return;
  const BlkRef* bl = blocks + d.first;
  stackqr_body<T>(reinterpret_cast<T*>(smem), d.r, d.nblk, [&](int b) { return bl[b]; }, chunk,
                  static_cast<T*>(d.R), d.ldr);
}

// The blocks of cluster q's stack in segment sg of S (window slots
// [36 sg / S, 36 (sg + 1) / S), the last segment also the parent term z_t),
// listed by the first wave: lane sl tests slot sl, and a ballot compacts the
// list in slot order (no lane waits on another's loads).
template <class T>
__device__ void win_blocks(const WinStack& a, int q, int t, int sg, int S, BlkRef* bl, int& nb) {
  const int lane = threadIdx.x % WAVE;
  const int qx = demorton_x(q), qy = demorton_y(q);
  const int s0 = 36 * sg / S, s1 = 36 * (sg + 1) / S;
  const int sl = s0 + lane;
  int rows = 0;
  if (sl < s1) {
    const int jx = 2 * (qx >> 1) - 2 + sl / 6, jy = 2 * (qy >> 1) - 2 + sl % 6;
    if (jx >= 0 && jy >= 0 && jx < a.nside && jy < a.nside && (abs(jx - qx) > 1 || abs(jy - qy) > 1))
      rows = a.r[morton2(jx, jy)];
  }
  const unsigned long long mask = __ballot(rows > 0);
  const int pos = __popcll(mask & ((1ull << lane) - 1));
  if (rows > 0) bl[pos] = BlkRef{static_cast<const T*>(a.M) + ((size_t)q * 36 + sl) * a.sM, a.rpad, rows, 1};
  const int c = __popcll(mask);
  if (lane == 0) {
    int n = c;
    if (sg == S - 1 && a.Z && a.r_par && a.r_par[q >> 2] > 0)
      bl[n++] = BlkRef{static_cast<const T*>(a.Z) + (size_t)t * a.sM, a.rpad, a.r_par[q >> 2], 0};
    nb = n;
  }
}

// Far-field weight of cluster q = ids[t] with its blocks found on the device:
// the stack of M(q, l)^T over the partners l of q's window (rows r[l]),
// then the parent term z_t (rows r_par[q / 4], when given).  Segment s of
// S takes window slots [36 s / S, 36 (s + 1) / S) (the last one also z_t) and
// writes its R to out + (t * S + s) * so, or out + q * so when S == 1 and
// out_by_id.
template <class T>
__global__ __launch_bounds__(WG) void k_stackqr_win(const WinStack a, int chunk) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ BlkRef bl[37];
  __shared__ int nb;
  const int t = blockIdx.x, sg = blockIdx.y;
  const int q = a.ids[t];
  const int r = a.r[q];
  if (r == 0) return;
  if (threadIdx.x < WAVE) win_blocks<T>(a, q, t, sg, a.S, bl, nb);
  __syncthreads();
  T* out = static_cast<T*>(a.out) + (a.S == 1 && a.out_by_id ? (size_t)q : (size_t)t * a.S + sg) * a.so;
  stackqr_body<T>(reinterpret_cast<T*>(smem), r, nb, [&](int b) { return bl[b]; }, chunk, out, a.ldo);
}

// R with R^T R = G (r x r in LDS, overwritten) by a right-looking Cholesky
// over the workgroup: row j of R goes to rowj, then (once every thread has
// read G_jj) into row j of G while the trailing upper triangle takes the
// rank-1 update, lane on rows j + 1 + lane (+ 64 ...), wave w on columns
// j + 1 + w (+ NW ...).  A pivot at or below 8 r eps_64 max_i G_ii gives a
// zero row.  R goes to the weight slot of cluster q (or of stack t).
template <class T>
__device__ void gram_chol(const WinStack& a, int q, int t, int r, double* G, double* rowj) {
  constexpr int NW = WG / WAVE;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  double gmax = 0.0;
  for (int j = 0; j < r; ++j) gmax = fmax(gmax, G[j + j * r]);
  const double tol = 8.0 * r * 2.220446049250313e-16 * gmax;
  for (int j = 0; j < r; ++j) {
    const double d = G[j + j * r];
    const double rjj = d > tol ? sqrt(d) : 0.0;
    for (int c = j + threadIdx.x; c < r; c += WG) rowj[c] = c == j ? rjj : (rjj > 0.0 ? G[j + c * r] / rjj : 0.0);
    __syncthreads();  // every thread has read G_jj
    for (int c = j + threadIdx.x; c < r; c += WG) G[j + c * r] = rowj[c];
    for (int c = j + 1 + w; c < r; c += NW) {
      const double rjc = rowj[c];
      for (int aa = j + 1 + lane; aa <= c; aa += WAVE) G[aa + c * r] -= rowj[aa] * rjc;
    }
    __syncthreads();
  }
  T* out = static_cast<T*>(a.out) + (a.out_by_id ? (size_t)q : (size_t)t) * a.so;
  for (int e = threadIdx.x; e < r * r; e += WG) {
    const int i = e % r, j = e / r;
    out[i + (size_t)j * a.ldo] = j < i ? T(0) : (T)G[i + j * r];
  }
}

// Far-field weight of cluster q = ids[t] from the Gram matrix of its stack:
// G = sum_l M(q, l) M(q, l)^T (+ z^T z for the parent term), the blocks
// staged GRAM_NB at a time in LDS and multiplied on the FP64 matrix cores
// (16 x 16 blocks of the upper triangle of G spread over the waves, four rows
// of the stack per v_mfma_f64_16x16x4), then R with R^T R = G by Cholesky
// over the workgroup (a pivot at or below 8 r eps_64 max_i G_ii, a direction the
// stack does not reach above FP64 rounding, gives a zero row).  R equals the
// R factor of the stack (positive diagonal) up to rounding in every
// direction above sqrt(eps_64) of the largest; used for the FP32 factor,
// where those below are FP32 noise.  Output as k_stackqr_win with S == 1.
constexpr int GRAM_NB = 4;
template <class T, int MAXP>
__global__ __launch_bounds__(WG) void k_gram_win(const WinStack a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ BlkRef bl[37];
  __shared__ int nb;
  __shared__ double rowj[kMaxRank];
  const int t = blockIdx.x;
  const int q = a.ids[t];
  const int r = a.r[q];
  if (r == 0) return;
  const int rp1 = a.max_rows + 1;
  const size_t bsz = (size_t)r * rp1;                // one staged block, [col][row]
  double* G = reinterpret_cast<double*>(smem);       // r x r
  T* Bs = reinterpret_cast<T*>(G + (size_t)r * r);   // GRAM_NB blocks
  if (threadIdx.x < WAVE) win_blocks<T>(a, q, t, 0, 1, bl, nb);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int li = lane % 16, lk = lane / 16;
  const int nbk = (r + 15) / 16, npair = nbk * (nbk + 1) / 2;
  constexpr int NW = WG / WAVE;
  // this wave's upper blocks (bi <= bj) of G: pair index w, w + NW, ... (< MAXP NW)
  int pbi[MAXP], pbj[MAXP];
#pragma unroll
  for (int u = 0; u < MAXP; ++u) {
    int pidx = w + u * NW, bi = 0;
    while (bi < nbk && pidx >= nbk - bi) {
      pidx -= nbk - bi;
      ++bi;
    }
    pbi[u] = w + u * NW < npair ? bi : -1;
    pbj[u] = bi + pidx;
  }
  md4 acc[MAXP];
#pragma unroll
  for (int u = 0; u < MAXP; ++u) acc[u] = md4{0, 0, 0, 0};
  __syncthreads();
  for (int b0 = 0; b0 < nb; b0 += GRAM_NB) {
    const int b1 = min(nb, b0 + GRAM_NB);
    __syncthreads();
    for (int b = b0; b < b1; ++b) {
      const BlkRef B = bl[b];
      const T* Bp = static_cast<const T*>(B.p);
      T* dst = Bs + (b - b0) * bsz;
      for (int e = threadIdx.x; e < B.rows * r; e += WG) {
        int i, j;
        if (B.trans) { j = e % r; i = e / r; } else { i = e % B.rows; j = e / B.rows; }
        dst[i + j * rp1] = B.trans ? Bp[j + (size_t)i * B.ld] : Bp[i + (size_t)j * B.ld];
      }
    }
    __syncthreads();
    for (int b = b0; b < b1; ++b) {
      const int rows = bl[b].rows;
      const T* src = Bs + (b - b0) * bsz;
      for (int k0 = 0; k0 < rows; k0 += 4) {
        const int row = k0 + lk;
#pragma unroll
        for (int u = 0; u < MAXP; ++u) {
          if (pbi[u] < 0) continue;
          const int ca = 16 * pbi[u] + li, cb = 16 * pbj[u] + li;
          const double xa = row < rows && ca < r ? (double)src[row + ca * rp1] : 0.0;
          const double xb = row < rows && cb < r ? (double)src[row + cb * rp1] : 0.0;
          acc[u] = mfma16(xa, xb, acc[u]);
        }
      }
    }
  }
  __syncthreads();
  // G(16 bi + i, 16 bj + j) = acc(i, j): lane j + 16 (i % 4), register i / 4
#pragma unroll
  for (int u = 0; u < MAXP; ++u) {
    if (pbi[u] < 0) continue;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int gi = 16 * pbi[u] + mfma_row(0.0, lane, rr), gj = 16 * pbj[u] + li;
      if (gi < r && gj < r) {
        G[gi + gj * r] = acc[u][rr];
        G[gj + gi * r] = acc[u][rr];
      }
    }
  }
  __syncthreads();
  gram_chol<T>(a, q, t, r, G, rowj);
}

// The same weight with the stack's blocks read straight from memory: wave w
// takes blocks w, w + NW, ... and accumulates every upper 16 x 16 block pair
// of G over its rows (NBK column blocks, r <= 16 NBK; four rows of the stack
// per v_mfma_f64_16x16x4, NBK loads feeding NBK (NBK + 1) / 2 independent
// accumulators); the waves' partial G are added in wave order (the same
// result on every run), then the Cholesky above.
template <class T, int NBK>
__global__ __launch_bounds__(WG) void k_gram_rows(const WinStack a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ BlkRef bl[37];
  __shared__ int nb;
  __shared__ double rowj[kMaxRank];
  constexpr int NW = WG / WAVE, NP = NBK * (NBK + 1) / 2;
  const int t = blockIdx.x;
  const int q = a.ids[t];
  const int r = a.r[q];
  if (r == 0) return;
  double* G = reinterpret_cast<double*>(smem);  // r x r
  if (threadIdx.x < WAVE) win_blocks<T>(a, q, t, 0, 1, bl, nb);
  for (int e = threadIdx.x; e < r * r; e += WG) G[e] = 0.0;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int li = lane % 16, lk = lane / 16;
  const int nbk = (r + 15) / 16;
  md4 acc[NP];
#pragma unroll
  for (int u = 0; u < NP; ++u) acc[u] = md4{0, 0, 0, 0};
  __syncthreads();
  const int nbl = nb;
  for (int b = w; b < nbl; b += NW) {
    const BlkRef B = bl[b];
    const T* Bp = static_cast<const T*>(B.p);
    // stack row k, column c: B^T (k, c) = p[c + k ld] or B (k, c) = p[k + c ld]
    const size_t sr = B.trans ? (size_t)B.ld : 1, sc = B.trans ? 1 : (size_t)B.ld;
#pragma unroll 2
    for (int k0 = 0; k0 < B.rows; k0 += 4) {
      const int row = k0 + lk;
      double x[NBK];
#pragma unroll
      for (int c = 0; c < NBK; ++c) {
        const int col = 16 * c + li;
        x[c] = row < B.rows && col < r ? (double)Bp[row * sr + col * sc] : 0.0;
      }
      int u = 0;
#pragma unroll
      for (int bi = 0; bi < NBK; ++bi)
#pragma unroll
        for (int bj = bi; bj < NBK; ++bj, ++u)
          if (bj < nbk) acc[u] = mfma16(x[bi], x[bj], acc[u]);
    }
  }
  // G(16 bi + i, 16 bj + j) += acc(i, j): lane j + 16 (i % 4), register i / 4
  for (int ww = 0; ww < NW; ++ww) {
    if (w == ww) {
      int u = 0;
#pragma unroll
      for (int bi = 0; bi < NBK; ++bi)
#pragma unroll
        for (int bj = bi; bj < NBK; ++bj, ++u) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int gi = 16 * bi + mfma_row(0.0, lane, rr), gj = 16 * bj + li;
            if (gi < r && gj < r) {
              G[gi + gj * r] += acc[u][rr];
              if (bi != bj) G[gj + gi * r] += acc[u][rr];
            }
          }
        }
    }
    __syncthreads();
  }
  gram_chol<T>(a, q, t, r, G, rowj);
}

// ------------------------------------------------------- BLOCKED INVERSE
// Gauss-Jordan by panels of nb columns.  The panel kernel runs the nb
// unblocked steps restricted to the panel columns (pivot search over the
// rows not yet used, row swap, scaling, elimination of every other row), so
// the panel ends as [A11^-1 on the pivot rows; -A21 A11^-1 elsewhere].  The
// remaining columns receive the same row swaps and then one rank-nb update
// (two GEMM shapes planned on the host).  A final pass undoes the column
// permutation.
template <bool kLds>
__global__ __launch_bounds__(WG) void k_gj_panel(const InvDesc* __restrict__ descs, int j0, int nb,
                                                 int* __restrict__ piv_all, int ldp, Status* st) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* f = reinterpret_cast<double*>(smem);  // m entries (+ the m x nb panel when kLds)
  const InvDesc d = descs[blockIdx.x];
  const int m = d.m;
  if (d.A == nullptr || j0 >= m) return;
  const int nbe = min(nb, m - j0);
  double* A;
  size_t lda;
  int c0;  // column index of panel column 0 inside A
  if (kLds) {
    A = f + m;
    lda = m;
    c0 = 0;
    for (int t = threadIdx.x / WAVE; t < nbe; t += WG / WAVE)
      for (int i = threadIdx.x % WAVE; i < m; i += WAVE) A[i + t * lda] = d.A[i + (size_t)(j0 + t) * d.lda];
    __syncthreads();
  } else {
    A = d.A + (size_t)j0 * d.lda;
    lda = d.lda;
    c0 = 0;
  }
  (void)c0;
  int* piv = piv_all + (size_t)blockIdx.x * ldp;
  __shared__ double rowj[64];
  __shared__ double rv[WG / WAVE];
  __shared__ int ri[WG / WAVE];
  bool bad = false;
  for (int t = 0; t < nbe; ++t) {
    const int j = j0 + t;  // global row / column index of the pivot
    double bv = -1.0;
    int bi = m;
    for (int i = j + threadIdx.x; i < m; i += WG) {
      const double a = fabs(A[i + t * lda]);
      if (a > bv || (a == bv && i < bi)) { bv = a; bi = i; }
    }
    double pv;
    int p;
    block_argmax(bv, bi, rv, ri, pv, p);
    if (threadIdx.x == 0) piv[j] = p;
    if (p != j && threadIdx.x < nbe) {
      const int c = threadIdx.x;
      const double tmp = A[j + c * lda];
      A[j + c * lda] = A[p + c * lda];
      A[p + c * lda] = tmp;
    }
    __syncthreads();
    const double djj = A[j + t * lda];
    if (djj == 0.0) bad = true;
    const double inv = 1.0 / djj;
    double* fcol = kLds ? f : nullptr;
    __shared__ double fbuf_small[1];
    (void)fbuf_small;
    if (kLds) {
      for (int i = threadIdx.x; i < m; i += WG) fcol[i] = A[i + t * lda];
    } else {
      for (int i = threadIdx.x; i < m; i += WG) f[i] = A[i + t * lda];
      fcol = f;
    }
    if (threadIdx.x < nbe) {
      const int c = threadIdx.x;
      rowj[c] = c == t ? inv : A[j + c * lda] * inv;
    }
    __syncthreads();
    for (int tc = threadIdx.x / WAVE; tc < nbe; tc += WG / WAVE) {
      double* col = A + tc * lda;
      const double rc = rowj[tc];
      for (int i = threadIdx.x % WAVE; i < m; i += WAVE) {
        if (i == j) col[i] = rc;
        else if (tc == t) col[i] = -fcol[i] * inv;
        else col[i] = fma(-fcol[i], rc, col[i]);
      }
    }
    __syncthreads();
  }
  if (kLds) {
    for (int t = threadIdx.x / WAVE; t < nbe; t += WG / WAVE)
      for (int i = threadIdx.x % WAVE; i < m; i += WAVE) d.A[i + (size_t)(j0 + t) * d.lda] = A[i + t * lda];
  }
  if (bad && threadIdx.x == 0 && st) {
    if (atomicExch(&st->singular, 1) == 0) st->bad_cluster = blockIdx.x;
  }
}

// Whole-matrix Gauss-Jordan with the matrix in registers (one workgroup per
// matrix, m <= min(TR RA, TC RB)): thread (tr, tc) of a TR x TC grid (rows
// fastest) holds rows tr + TR a and columns tc + TC b.  Rows are never
// swapped: step j takes as pivot the largest |M(i, j)| over the rows not yet
// used (the smallest i on ties), publishes column j and the pivot row through
// LDS (double-buffered, two barriers per step) and every thread updates its
// tile.  With piv[j] the pivot row of step j and pinv its inverse, the
// inverse is A^-1(pinv[i], piv[c]) = M(i, c), applied in the write-back.
template <int TR, int TC, int RA, int RB>
__global__ __launch_bounds__(TR * TC) void k_gj_reg(const InvDesc* __restrict__ descs, Status* st) {
  static_assert(RA <= 32, "row-slot mask");
  static_assert(TR <= WAVE && WAVE % TR == 0, "a column's owners share one wave");
  __shared__ double fcol[2][TR * RA];
  __shared__ double prow[2][TC * RB];
  __shared__ int pbuf[2];
  __shared__ int piv[TC * RB];
  __shared__ int pinv[TR * RA];
  const InvDesc d = descs[blockIdx.x];
  const int m = d.m;
  if (d.A == nullptr || m <= 0) return;
  const int tr = threadIdx.x % TR, tc = threadIdx.x / TR;
  const size_t lda = d.lda;
  double M[RA][RB];
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int i = tr + TR * a, c = tc + TC * b;
      M[a][b] = (i < m && c < m) ? d.A[i + c * lda] : 0.0;
    }
  unsigned used = 0;  // bit a: row tr + TR a has been a pivot
  bool bad = false;
#pragma unroll
  for (int bj = 0; bj < RB; ++bj) {
    for (int jj = 0; jj < TC; ++jj) {
      const int j = bj * TC + jj;
      if (j >= m) break;
      const int buf = j & 1;
      // the TR lanes holding column j publish it and pick the pivot
      if (tc == jj) {
        double bv = -1.0;
        int bi = 1 << 30;
#pragma unroll
        for (int a = 0; a < RA; ++a) {
          const int i = tr + TR * a;
          fcol[buf][i] = M[a][bj];
          double v = fabs(M[a][bj]);
          if (v != v) v = HUGE_VAL;  // NaN: a total order, and a valid index
          if (i < m && !((used >> a) & 1u) && (v > bv || bi >= m)) {
            bv = v;
            bi = i;
          }
        }
#pragma unroll
        for (int o = 1; o < TR; o <<= 1) {
          const double ov = __shfl_xor(bv, o, WAVE);
          const int oi = __shfl_xor(bi, o, WAVE);
          if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
          }
        }
        if (tr == 0) pbuf[buf] = bi;
      }
      __syncthreads();
      // the pivot row is the same for every thread: read as a scalar, so the
      // selection of its register slot below compiles to scalar branches
      // (not a chain of per-lane selects over every slot and column)
      const int p = __builtin_amdgcn_readfirstlane(pbuf[buf]);
      const int tp = p % TR, ap = p / TR;
      if (tr == tp) {
#pragma unroll
        for (int a = 0; a < RA; ++a)
          if (a == ap) {
#pragma unroll
            for (int b = 0; b < RB; ++b) prow[buf][tc + TC * b] = M[a][b];
            used |= 1u << a;
          }
      }
      if (threadIdx.x == 0) piv[j] = p;
      __syncthreads();
      const double pv = fcol[buf][p];
      if (pv == 0.0) bad = true;
      const double ip = 1.0 / pv;
      double rb[RB], fa[RA];
#pragma unroll
      for (int b = 0; b < RB; ++b) rb[b] = prow[buf][tc + TC * b] * ip;
      if (tc == jj) rb[bj] = ip;
#pragma unroll
      for (int a = 0; a < RA; ++a) fa[a] = fcol[buf][tr + TR * a];
#pragma unroll
      for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < RB; ++b) M[a][b] = fma(-fa[a], rb[b], M[a][b]);
      if (tc == jj) {
#pragma unroll
        for (int a = 0; a < RA; ++a) M[a][bj] = -fa[a] * ip;
      }
      if (tr == tp) {
#pragma unroll
        for (int a = 0; a < RA; ++a)
          if (a == ap) {
#pragma unroll
            for (int b = 0; b < RB; ++b) M[a][b] = rb[b];
          }
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < m; j += TR * TC) pinv[piv[j]] = j;
  __syncthreads();
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const int c = tc + TC * b;
    if (c >= m) continue;
    double* col = d.A + (size_t)piv[c] * lda;
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const int i = tr + TR * a;
      if (i < m) col[pinv[i]] = M[a][b];
    }
  }
  if (bad && threadIdx.x == 0 && st) {
    if (atomicExch(&st->singular, 1) == 0) st->bad_cluster = blockIdx.x;
  }
}

// The same panel steps with the panel in registers (m <= 64 RA, nb <= 8 RB):
// thread (tr, tc), tr < 64 the lane of wave tc, holds rows tr + 64 a and panel
// columns j0 + tc + 8 b.  Each step: the wave holding column j picks the pivot
// (largest |A(i, j)| over i >= j, smallest i on ties) and publishes the column;
// rows p and j are published; after one more barrier every thread updates its
// tile and rows j and p take their swapped, scaled / eliminated contents.
template <int RA, int RB>
__global__ __launch_bounds__(512) void k_gj_panel_reg(const InvDesc* __restrict__ descs, int j0, int nb,
                                                      int* __restrict__ piv_all, int ldp, Status* st) {
  constexpr int TR = WAVE, TC = 8;
  static_assert(TR * TC == 512, "eight waves");
  __shared__ double fcol[2][TR * RA];
  __shared__ double prow[2][TC * RB];
  __shared__ double rowj[2][TC * RB];
  __shared__ int pbuf[2];
  const InvDesc d = descs[blockIdx.x];
  const int m = d.m;
  if (d.A == nullptr || j0 >= m) return;
  const int nbe = min(nb, m - j0);
  const int tr = threadIdx.x % TR, tc = threadIdx.x / TR;
  const size_t lda = d.lda;
  int* piv = piv_all + (size_t)blockIdx.x * ldp;
  double M[RA][RB];
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int i = tr + TR * a, t = tc + TC * b;
      M[a][b] = (i < m && t < nbe) ? d.A[i + (size_t)(j0 + t) * lda] : 0.0;
    }
  bool bad = false;
#pragma unroll
  for (int bt = 0; bt < RB; ++bt) {
    for (int tt = 0; tt < TC; ++tt) {
      const int t = bt * TC + tt;
      if (t >= nbe) break;
      const int j = j0 + t, buf = t & 1;
      if (tc == tt) {
        // key: |A(i, t)| as unsigned bits + 1 (NaN above inf), 0 for rows < j
        unsigned long long bk = 0;
        int bi = m;
#pragma unroll
        for (int a = 0; a < RA; ++a) {
          const int i = tr + TR * a;
          fcol[buf][i] = M[a][bt];
          const unsigned long long k =
              (i >= j && i < m) ? ((unsigned long long)__double_as_longlong(M[a][bt]) & 0x7fffffffffffffffull) + 1 : 0;
          if (k > bk) {
            bk = k;
            bi = i;
          }
        }
#pragma unroll
        for (int o = 1; o < TR; o <<= 1) {
          const unsigned long long ok = __shfl_xor(bk, o, WAVE);
          const int oi = __shfl_xor(bi, o, WAVE);
          if (ok > bk || (ok == bk && oi < bi)) {
            bk = ok;
            bi = oi;
          }
        }
        if (tr == 0) pbuf[buf] = bi < m ? bi : j;
      }
      __syncthreads();
      const int p = __builtin_amdgcn_readfirstlane(pbuf[buf]);  // uniform: scalar slot selection below
      const int tp = p % TR, ap = p / TR, tj = j % TR, aj = j / TR;
      if (tr == tp) {
#pragma unroll
        for (int a = 0; a < RA; ++a)
          if (a == ap) {
#pragma unroll
            for (int b = 0; b < RB; ++b) prow[buf][tc + TC * b] = M[a][b];
          }
      }
      if (tr == tj) {
#pragma unroll
        for (int a = 0; a < RA; ++a)
          if (a == aj) {
#pragma unroll
            for (int b = 0; b < RB; ++b) rowj[buf][tc + TC * b] = M[a][b];
          }
      }
      if (threadIdx.x == 0) piv[j] = p;
      __syncthreads();
      const double pv = fcol[buf][p], fj = fcol[buf][j];
      if (pv == 0.0) bad = true;
      const double ip = 1.0 / pv;
      double rb[RB], fa[RA];
#pragma unroll
      for (int b = 0; b < RB; ++b) rb[b] = prow[buf][tc + TC * b] * ip;
      if (tc == tt) rb[bt] = ip;
#pragma unroll
      for (int a = 0; a < RA; ++a) fa[a] = fcol[buf][tr + TR * a];
#pragma unroll
      for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < RB; ++b) M[a][b] = fma(-fa[a], rb[b], M[a][b]);
      if (tc == tt) {
#pragma unroll
        for (int a = 0; a < RA; ++a) M[a][bt] = -fa[a] * ip;
      }
      if (p != j && tr == tp) {  // row p takes the old row j, eliminated
#pragma unroll
        for (int a = 0; a < RA; ++a)
          if (a == ap) {
#pragma unroll
            for (int b = 0; b < RB; ++b) M[a][b] = fma(-fj, rb[b], rowj[buf][tc + TC * b]);
            if (tc == tt) M[a][bt] = -fj * ip;
          }
      }
      if (tr == tj) {  // row j takes the scaled pivot row
#pragma unroll
        for (int a = 0; a < RA; ++a)
          if (a == aj) {
#pragma unroll
            for (int b = 0; b < RB; ++b) M[a][b] = rb[b];
          }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int i = tr + TR * a, t = tc + TC * b;
      if (i < m && t < nbe) d.A[i + (size_t)(j0 + t) * lda] = M[a][b];
    }
  if (bad && threadIdx.x == 0 && st) {
    if (atomicExch(&st->singular, 1) == 0) st->bad_cluster = blockIdx.x;
  }
}

// Row swaps of the panel applied to every other column, and rows j0..j0+nb-1
// of those columns copied to tmp (nb x m, ld nb).
__global__ __launch_bounds__(WG) void k_gj_rest(const InvDesc* __restrict__ descs, int j0, int nb,
                                                const int* __restrict__ piv_all, int ldp,
                                                double* __restrict__ tmp_all, size_t ldt) {
  const InvDesc d = descs[blockIdx.x];
  const int m = d.m;
  if (d.A == nullptr || j0 >= m) return;
  const int nbe = min(nb, m - j0);
  const int* piv = piv_all + (size_t)blockIdx.x * ldp;
  double* tmp = tmp_all + (size_t)blockIdx.x * ldt;
  const size_t lda = d.lda;
  for (int c = blockIdx.y * WG + threadIdx.x; c < m; c += gridDim.y * WG) {
    if (c >= j0 && c < j0 + nbe) continue;
    double* col = d.A + c * lda;
    for (int t = 0; t < nbe; ++t) {
      const int j = j0 + t, p = piv[j];
      if (p != j) {
        const double x = col[j];
        col[j] = col[p];
        col[p] = x;
      }
    }
    for (int t = 0; t < nbe; ++t) tmp[t + (size_t)c * nb] = col[j0 + t];
  }
}

__global__ __launch_bounds__(WG) void k_gj_unpermute(const InvDesc* __restrict__ descs,
                                                     const int* __restrict__ piv_all, int ldp) {
  const InvDesc d = descs[blockIdx.x];
  const int m = d.m;
  if (d.A == nullptr) return;
  const int* piv = piv_all + (size_t)blockIdx.x * ldp;
  const size_t lda = d.lda;
  for (int i = blockIdx.y * WG + threadIdx.x; i < m; i += gridDim.y * WG) {
    for (int j = m - 1; j >= 0; --j) {
      const int p = piv[j];
      if (p != j) {
        const double x = d.A[i + j * lda];
        d.A[i + j * lda] = d.A[i + p * lda];
        d.A[i + p * lda] = x;
      }
    }
  }
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

template <class TA, class TB, class TC>
void gemm_go(const GemmDesc* d, int nd, int tm, int tn, int max_m, bool gemv, hipStream_t s) {
  if (gemv) hipLaunchKernelGGL((k_gemv<TA, TB, TC>), dim3(nd, cdiv(max_m, WAVE)), dim3(WG), 0, s, d);
  else hipLaunchKernelGGL((k_gemm<TA, TB, TC>), dim3(nd, tm * tn), dim3(WG), 0, s, d, tm);
}

template <class TA, class TC>
void add_go(const AddDesc* d, int nd, int tm, int tn, hipStream_t s) {
  hipLaunchKernelGGL((k_add<TA, TC>), dim3(nd, tm * tn), dim3(WG), 0, s, d, tm);
}

// Raise a kernel's dynamic-LDS limit to the CU's 160 KiB once, before its
// first launch that needs more than the default 64 KiB.  Thread-safe (batched
// factorisations launch from several host threads) and monotonic: the limit
// only bounds what a launch may ask for, the LDS actually allocated (and the
// occupancy) is the launch's own request.
constexpr size_t kLdsLimit = 160 * 1024;
}  // namespace
void allow_lds(const void* fn) {
  static std::mutex mu;
  static std::unordered_set<const void*> done;
  std::lock_guard<std::mutex> lk(mu);
  if (!done.insert(fn).second) return;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit) != hipSuccess)
    (void)hipGetLastError();  // the launch reports a real shortfall
}
namespace {

// Chunk rows of the stacked-R kernels and their LDS bytes for rank r: up to
// max_chunk rows, within 64 KiB when 128 rows fit there (several workgroups
// per CU), else within 150 KiB of the 160 KiB LDS of a gfx950 CU.  The
// window stacks of a whole level run as one launch: short chunks keep more
// workgroups per CU in flight (measured: 128 rows beat 64, 256 and 1024).
template <class T>
size_t stackqr_lds(int max_r, int& chunk, int max_chunk) {
  const size_t rr = (size_t)max_r * max_r * sizeof(T);
  const size_t row = sizeof(T) * max_r;
  const size_t budget = rr + 129 * row <= 64 * 1024 ? 64 * 1024 : 150 * 1024;
  chunk = (int)((budget - rr) / row) - 1;
  if (chunk > max_chunk) chunk = max_chunk;
  if (chunk < 1) chunk = 1;
  return rr + (size_t)(chunk + 1) * row;
}

template <class T>
void stackqr_win_go(const WinStack& a, int max_r, hipStream_t s) {
  int chunk;
  const size_t lds = stackqr_lds<T>(max_r, chunk, 128);
  if (lds > 64 * 1024) {
    allow_lds(reinterpret_cast<const void*>(k_stackqr_win<T>));
  }
  hipLaunchKernelGGL(k_stackqr_win<T>, dim3(a.nt, a.S), dim3(WG), lds, s, a, chunk);
}

template <class T>
void stackqr_go(const StackQrDesc* d, const BlkRef* b, int nd, int max_r, hipStream_t s) {
  int chunk;
  const size_t lds = stackqr_lds<T>(max_r, chunk, 256);
  if (lds > 64 * 1024) {
    allow_lds(reinterpret_cast<const void*>(k_stackqr<T>));
  }
  hipLaunchKernelGGL(k_stackqr<T>, dim3(nd), dim3(WG), lds, s, d, b, chunk);
}

}  // namespace

void launch_gemm(const GemmDesc* d, int nd, int max_m, int max_n, int ty, int plain, hipStream_t s) {
  if (nd <= 0 || max_m <= 0 || max_n <= 0) return;
  const int tm = cdiv(max_m, 64), tn = cdiv(max_n, 64);
  const bool gemv = plain && max_n <= GEMV_N;
  switch (ty) {
    case 0: gemm_go<double, double, double>(d, nd, tm, tn, max_m, gemv, s); break;
    case 1: gemm_go<float, double, double>(d, nd, tm, tn, max_m, gemv, s); break;
    case 2: gemm_go<double, float, double>(d, nd, tm, tn, max_m, gemv, s); break;
    case 3: gemm_go<float, float, double>(d, nd, tm, tn, max_m, gemv, s); break;
    case 4: gemm_go<double, double, float>(d, nd, tm, tn, max_m, gemv, s); break;
    case 5: gemm_go<float, double, float>(d, nd, tm, tn, max_m, gemv, s); break;
    case 6: gemm_go<double, float, float>(d, nd, tm, tn, max_m, gemv, s); break;
    default: gemm_go<float, float, float>(d, nd, tm, tn, max_m, gemv, s); break;
  }
}

void launch_add(const AddDesc* d, int nd, int max_m, int max_n, int ty, hipStream_t s) {
  if (nd <= 0 || max_m <= 0 || max_n <= 0) return;
  const int tm = cdiv(max_m, 64), tn = cdiv(max_n, 64);
  switch (ty) {
    case 0: add_go<double, double>(d, nd, tm, tn, s); break;
    case 1: add_go<float, double>(d, nd, tm, tn, s); break;
    case 2: add_go<double, float>(d, nd, tm, tn, s); break;
    default: add_go<float, float>(d, nd, tm, tn, s); break;
  }
}

void launch_elim(const ElimArgs& a, int step, int max_m, int max_n, int ty, hipStream_t s) {
  if (a.nb <= 0 || max_m <= 0 || max_n <= 0) return;
  const int tm = cdiv(max_m, 64), tn = cdiv(max_n, 64);
  const bool xcd = step == 2 || step >= 4;
  const dim3 grid = xcd ? dim3((unsigned)(cdiv(a.nb, kXcd) * kXcd * elim_items(step, a.npair)))
                        : dim3(a.nb, (step == 0 ? 1 : 9) * tm * tn);
#define ELIM_GO(S)                                                                            \
  if (ty) hipLaunchKernelGGL((k_elim<float, S>), grid, dim3(WG), 0, s, a, tm, tn);   \
  else hipLaunchKernelGGL((k_elim<double, S>), grid, dim3(WG), 0, s, a, tm, tn);
  switch (step) {
    case 0: ELIM_GO(0) break;
    case 1: ELIM_GO(1) break;
    case 2: ELIM_GO(2) break;
    case 3: ELIM_GO(3) break;
    case 4: ELIM_GO(4) break;
    default: ELIM_GO(5) break;
  }
#undef ELIM_GO
}

void launch_transition(const TransArgs& a, int ty, hipStream_t s) {
  if (a.nc <= 0) return;
  const dim3 grid(a.nc, 148);
  if (ty) hipLaunchKernelGGL(k_transition<float>, grid, dim3(WG), 0, s, a);
  else hipLaunchKernelGGL(k_transition<double>, grid, dim3(WG), 0, s, a);
}

// Colour batches of fewer records than this run solve steps 0, 2 and 3 with
// 16 waves per workgroup (measured at the coarse levels of a 1M-point step:
// residual gathers 4.9 -> 3.9 ms, steps 0 and 3 2.5 -> 2.3 ms; batches of
// 450+ records lose with it).
constexpr int kSolveWideRecords = 256;

void launch_solve(const SolveArgs& a, int step, double* wk, int max_rows, int ty, hipStream_t s) {
  if (a.nb <= 0 || max_rows <= 0) return;
  const int tiles = cdiv(max_rows, WAVE);
  const dim3 grid(a.nb, (step == 1 ? 9 : 1) * tiles);
  // staged vectors: min(SV_C, nrhs) columns of mpad (step 2: of every
  // neighbour block, 8 max(npad, rpad))
  const size_t lds = sizeof(double) * std::min(SV_C, a.nrhs) *
                     (step == 2 ? (size_t)8 * std::max(a.npad, a.rpad) : (size_t)a.mpad);
#define SOLVE_GO(S, NT)                                                                                       \
  if (a.nrhs == 1) {                                                                                        \
    if (ty) hipLaunchKernelGGL((k_solve<float, S, 1, NT>), grid, dim3(NT), lds, s, a, wk, tiles);             \
    else hipLaunchKernelGGL((k_solve<double, S, 1, NT>), grid, dim3(NT), lds, s, a, wk, tiles);               \
  } else {                                                                                                  \
    if (ty) hipLaunchKernelGGL((k_solve<float, S, SV_C, NT>), grid, dim3(NT), lds, s, a, wk, tiles);          \
    else hipLaunchKernelGGL((k_solve<double, S, SV_C, NT>), grid, dim3(NT), lds, s, a, wk, tiles);            \
  }
  const bool wide = a.nb < kSolveWideRecords;
  switch (step) {
    case 0:
      if (wide) {
        SOLVE_GO(0, 4 * WG)
      } else {
        SOLVE_GO(0, WG)
      }
      break;
    case 1:  // a workgroup per (record, unit, tile) already: no wide form (measured slower)
      SOLVE_GO(1, WG)
      break;
    case 2:
      if (wide) {
        SOLVE_GO(2, 4 * WG)
      } else {
        SOLVE_GO(2, WG)
      }
      break;
    default:
      if (wide) {
        SOLVE_GO(3, 4 * WG)
      } else {
        SOLVE_GO(3, WG)
      }
      break;
  }
#undef SOLVE_GO
}

void launch_m2l_assemble(const M2LAssemble& a, int ty, hipStream_t s) {
  if (a.nc <= 0) return;
  const dim3 grid(a.nc, 36);
  const size_t lds = (size_t)a.rpad * a.p2 * sizeof(double);
  if (ty) hipLaunchKernelGGL(k_m2l_assemble<float>, grid, dim3(WG), lds, s, a);
  else hipLaunchKernelGGL(k_m2l_assemble<double>, grid, dim3(WG), lds, s, a);
}

void launch_rank_finalize(const RankFin& a, hipStream_t s) {
  if (a.nt <= 0) return;
  hipLaunchKernelGGL(k_rank_finalize, dim3(cdiv(a.nt, WG)), dim3(WG), 0, s, a);
}

void launch_fill_copy(const FillCopy& a, int ty, hipStream_t s) {
  if (a.nt <= 0) return;
  if (ty) hipLaunchKernelGGL(k_fill_copy<float>, dim3(a.nt, 9), dim3(WG), 0, s, a);
  else hipLaunchKernelGGL(k_fill_copy<double>, dim3(a.nt, 9), dim3(WG), 0, s, a);
}

void launch_touch_xform(const TouchXform& a, int ty, hipStream_t s) {
  if (a.nt <= 0) return;
  const dim3 grid(a.nt, a.Unew ? 38 : 37);
  const size_t lds = (size_t)a.rpad * a.rpad * (ty ? sizeof(float) : sizeof(double));
  if (ty) {
    if (lds > 64 * 1024) allow_lds(reinterpret_cast<const void*>(k_touch_xform<float>));
    hipLaunchKernelGGL(k_touch_xform<float>, grid, dim3(WG), lds, s, a);
  } else {
    if (lds > 64 * 1024) allow_lds(reinterpret_cast<const void*>(k_touch_xform<double>));
    hipLaunchKernelGGL(k_touch_xform<double>, grid, dim3(WG), lds, s, a);
  }
}

int qr_wave_rows(int n, int m, int ty) {
  if (m > WAVE || n <= 0) return 0;
  if (n <= 32) return 32;
  if (n <= 64) return 64;
  if (n <= 96) return 96;
  if (ty && n <= 128) return 128;
  return 0;
}

template <class T, int NR>
void qr_wave_go(const QrDesc* d, int nd, int max_k, hipStream_t s) {
  const size_t lds = (size_t)std::max(max_k, 1) * NR * sizeof(T);
  if (lds > 64 * 1024) allow_lds(reinterpret_cast<const void*>(k_qr_wave<T, NR>));
  hipLaunchKernelGGL((k_qr_wave<T, NR>), dim3(nd), dim3(WAVE), lds, s, d);
}

void launch_qr_wave(const QrDesc* d, int nd, int nr, int max_k, int ty, hipStream_t s) {
  if (nd <= 0) return;
  if (ty) {
    switch (nr) {
      case 32: qr_wave_go<float, 32>(d, nd, max_k, s); break;
      case 64: qr_wave_go<float, 64>(d, nd, max_k, s); break;
      case 96: qr_wave_go<float, 96>(d, nd, max_k, s); break;
      default: qr_wave_go<float, 128>(d, nd, max_k, s); break;
    }
  } else {
    switch (nr) {
      case 32: qr_wave_go<double, 32>(d, nd, max_k, s); break;
      case 64: qr_wave_go<double, 64>(d, nd, max_k, s); break;
      default: qr_wave_go<double, 96>(d, nd, max_k, s); break;
    }
  }
}

void launch_qr(const QrDesc* d, int nd, size_t lds, int ty, hipStream_t s) {
  if (nd <= 0) return;
  if (lds > kQrLdsBytes) return;
  if (lds) {
    if (ty) hipLaunchKernelGGL((k_qr<float, true>), dim3(nd), dim3(WG), lds, s, d);
    else hipLaunchKernelGGL((k_qr<double, true>), dim3(nd), dim3(WG), lds, s, d);
  } else {
    if (ty) hipLaunchKernelGGL((k_qr<float, false>), dim3(nd), dim3(WG), 0, s, d);
    else hipLaunchKernelGGL((k_qr<double, false>), dim3(nd), dim3(WG), 0, s, d);
  }
}

// The LDS pivoted QR runs 1024 threads per matrix: a staged matrix takes
// most of a CU's LDS, so the CU's parallelism has to come from one workgroup.
constexpr int RRQR_NT = 1024;
// Rows per lane of the register-held update (even, 16 NV >= max_n), 0 for
// the loop form.
template <class T, bool kLds>
void rrqr_go(const RrqrDesc* d, int nd, size_t lds, int max_n, hipStream_t s) {
  auto go = [&](auto kern) {
    if (kLds || lds > 64 * 1024) allow_lds(reinterpret_cast<const void*>(kern));
    hipLaunchKernelGGL(kern, dim3(nd), dim3(RRQR_NT), lds, s, d);
  };
  constexpr bool f32 = sizeof(T) == 4;  // registers: up to 24 FP32 or 18 FP64 rows per lane
  if (max_n <= 128) go(k_rrqr<T, RRQR_NT, kLds, 8>);
  else if (max_n <= 192) go(k_rrqr<T, RRQR_NT, kLds, 12>);
  else if (max_n <= 288) go(k_rrqr<T, RRQR_NT, kLds, 18>);
  else if (f32 && max_n <= 384) go(k_rrqr<T, RRQR_NT, kLds, f32 ? 24 : 0>);
  else go(k_rrqr<T, RRQR_NT, kLds, 0>);
}

void launch_rrqr_lds(const RrqrDesc* d, int nd, size_t lds, int max_n, int ty, hipStream_t s) {
  if (nd <= 0) return;
  if (ty) rrqr_go<float, true>(d, nd, lds, max_n, s);
  else rrqr_go<double, true>(d, nd, lds, max_n, s);
}

bool rrqr_reg_reads_fill(int nr, int ty) { return ty && nr <= 96; }

int rrqr_reg_rows(int n, int ty) {
  if (n <= 32) return 32;
  if (n <= 64) return 64;
  if (n <= 96) return 96;
  if (!ty) return 0;  // FP64 columns beyond 96 rows do not fit the register file
  if (n <= 128) return 128;
  return 0;
}

size_t rrqr_reg_lds(int nr, int kmax, int ty) {
  return (size_t)std::min(kmax, kMaxRank) * nr * (ty ? sizeof(float) : sizeof(double));
}

template <class T, int NR>
void rrqr_reg_go(const RrqrDesc* d, int nd, int nt, size_t lds, const FillCopy& fc, hipStream_t s) {
  // the kernel's static LDS is a few KiB: raise the dynamic limit to what
  // this launch asks for, when above the default
  if (lds > 64 * 1024) allow_lds(reinterpret_cast<const void*>(k_rrqr_reg<T, NR>));
  hipLaunchKernelGGL((k_rrqr_reg<T, NR>), dim3(nd), dim3(nt), lds, s, d, fc);
}

void launch_rrqr_reg(const RrqrDesc* d, int nd, int max_m, int nr, int max_kmax, int ty, const FillCopy* fcp,
                     hipStream_t s) {
  if (nd <= 0 || max_m <= 0) return;
  const int nt = std::min(kRrqrRegCols, (max_m + WAVE - 1) / WAVE * WAVE);
  const size_t lds = rrqr_reg_lds(nr, max_kmax, ty);
  FillCopy fc{};
  if (fcp) fc = *fcp;
  if (ty) {
    switch (nr) {
      case 32: rrqr_reg_go<float, 32>(d, nd, nt, lds, fc, s); break;
      case 64: rrqr_reg_go<float, 64>(d, nd, nt, lds, fc, s); break;
      case 96: rrqr_reg_go<float, 96>(d, nd, nt, lds, fc, s); break;
      case 128: rrqr_reg_go<float, 128>(d, nd, nt, lds, fc, s); break;
    }
  } else {
    switch (nr) {
      case 32: rrqr_reg_go<double, 32>(d, nd, nt, lds, fc, s); break;
      case 64: rrqr_reg_go<double, 64>(d, nd, nt, lds, fc, s); break;
      case 96: rrqr_reg_go<double, 96>(d, nd, nt, lds, fc, s); break;
    }
  }
}

template <class T, int NR, int G>
void formq_rr_go(const RrqrDesc* d, int nd, int max_kmax, hipStream_t s) {
  const size_t lds = (size_t)std::min(max_kmax, kMaxRank) * G * NR * sizeof(T);
  if (lds > 64 * 1024) allow_lds(reinterpret_cast<const void*>(k_formq_rr<T, NR, G>));
  hipLaunchKernelGGL((k_formq_rr<T, NR, G>), dim3(nd), dim3(512), lds, s, d);
}

// Q columns by groups of G lanes with NR rows each: G NR >= max_n.
void launch_formq_rr(const RrqrDesc* d, int nd, int max_n, int max_kmax, int ty, hipStream_t s) {
  if (nd <= 0 || max_n <= 0) return;
  const int rows = max_n <= 128 ? 128 : max_n <= 256 ? 256 : 512;
  if (max_n > 512 || (size_t)std::min(max_kmax, kMaxRank) * rows * (ty ? 4 : 8) > 144 * 1024) {
    if (ty) hipLaunchKernelGGL(k_formq_rr_glb<float>, dim3(nd), dim3(WG), 0, s, d);
    else hipLaunchKernelGGL(k_formq_rr_glb<double>, dim3(nd), dim3(WG), 0, s, d);
    return;
  }
  if (ty) {
    if (max_n <= 128) formq_rr_go<float, 32, 4>(d, nd, max_kmax, s);
    else if (max_n <= 256) formq_rr_go<float, 32, 8>(d, nd, max_kmax, s);
    else formq_rr_go<float, 64, 8>(d, nd, max_kmax, s);
  } else {
    if (max_n <= 128) formq_rr_go<double, 32, 4>(d, nd, max_kmax, s);
    else if (max_n <= 256) formq_rr_go<double, 32, 8>(d, nd, max_kmax, s);
    else formq_rr_go<double, 64, 8>(d, nd, max_kmax, s);
  }
}

void launch_rrqr_global(const RrqrDesc* d, int nd, int max_m, int max_n, int ty, hipStream_t s) {
  if (nd <= 0 || max_m <= 0) return;
  const size_t lds = (size_t)max_m * (ty ? sizeof(float) : sizeof(double));
  if (ty) rrqr_go<float, false>(d, nd, lds, max_n, s);
  else rrqr_go<double, false>(d, nd, lds, max_n, s);
}


template <class T, int MAXP>
void gram_win_go(const WinStack& a, size_t lds, hipStream_t s) {
  if (lds > 64 * 1024) allow_lds(reinterpret_cast<const void*>(k_gram_win<T, MAXP>));
  hipLaunchKernelGGL((k_gram_win<T, MAXP>), dim3(a.nt), dim3(WG), lds, s, a);
}

template <class T>
void gram_win_by_rank(const WinStack& a, int max_r, size_t lds, hipStream_t s) {
  const int nbk = (max_r + 15) / 16, np = nbk * (nbk + 1) / 2, per = (np + WG / WAVE - 1) / (WG / WAVE);
  if (per <= 1) gram_win_go<T, 1>(a, lds, s);
  else if (per <= 2) gram_win_go<T, 2>(a, lds, s);
  else if (per <= 4) gram_win_go<T, 4>(a, lds, s);
  else gram_win_go<T, 9>(a, lds, s);  // max_r <= kMaxRank = 128: 36 blocks
}

template <class T, int NBK>
void gram_rows_go(const WinStack& a, size_t lds, hipStream_t s) {
  if (lds > 64 * 1024) allow_lds(reinterpret_cast<const void*>(k_gram_rows<T, NBK>));
  hipLaunchKernelGGL((k_gram_rows<T, NBK>), dim3(a.nt), dim3(WG), lds, s, a);
}

void launch_gram_win(const WinStack& a, int max_r, int ty, hipStream_t s) {
  if (a.nt <= 0 || max_r <= 0) return;
  if (max_r <= 80) {  // blocks read in place, all block pairs per wave
    const size_t lds = sizeof(double) * (size_t)max_r * max_r;
    const int nbk = (max_r + 15) / 16;
#define GRAM_ROWS(T)                                  \
  switch (nbk) {                                      \
    case 1: gram_rows_go<T, 1>(a, lds, s); break;     \
    case 2: gram_rows_go<T, 2>(a, lds, s); break;     \
    case 3: gram_rows_go<T, 3>(a, lds, s); break;     \
    case 4: gram_rows_go<T, 4>(a, lds, s); break;     \
    default: gram_rows_go<T, 5>(a, lds, s); break;    \
  }
    if (ty) GRAM_ROWS(float) else GRAM_ROWS(double)
#undef GRAM_ROWS
    return;
  }
  const size_t lds = sizeof(double) * (size_t)max_r * max_r +
                     (ty ? sizeof(float) : sizeof(double)) * GRAM_NB * (size_t)max_r * (a.max_rows + 1);
  if (ty) gram_win_by_rank<float>(a, max_r, lds, s);
  else gram_win_by_rank<double>(a, max_r, lds, s);
}

void launch_stackqr_win(const WinStack& a, int max_r, int ty, hipStream_t s) {
  if (a.nt <= 0 || max_r <= 0) return;
  if (ty) stackqr_win_go<float>(a, max_r, s);
  else stackqr_win_go<double>(a, max_r, s);
}

void launch_stackqr(const StackQrDesc* d, const BlkRef* b, int nd, int max_r, int ty, hipStream_t s) {
  if (nd <= 0 || max_r <= 0) return;
  if (ty) stackqr_go<float>(d, b, nd, max_r, s);
  else stackqr_go<double>(d, b, nd, max_r, s);
}

void launch_gj_panel(const InvDesc* d, int nd, int max_m, int j0, int nb, int* piv, int ldp,
                     Status* st, hipStream_t s) {
  if (nd <= 0) return;
  if (nb <= 32 && max_m <= 768) {
    if (max_m <= 256) hipLaunchKernelGGL((k_gj_panel_reg<4, 4>), dim3(nd), dim3(512), 0, s, d, j0, nb, piv, ldp, st);
    else if (max_m <= 384) hipLaunchKernelGGL((k_gj_panel_reg<6, 4>), dim3(nd), dim3(512), 0, s, d, j0, nb, piv, ldp, st);
    else if (max_m <= 512) hipLaunchKernelGGL((k_gj_panel_reg<8, 4>), dim3(nd), dim3(512), 0, s, d, j0, nb, piv, ldp, st);
    else hipLaunchKernelGGL((k_gj_panel_reg<12, 4>), dim3(nd), dim3(512), 0, s, d, j0, nb, piv, ldp, st);
    return;
  }
  if (nb <= 64 && max_m <= 512) {
    if (max_m <= 256) hipLaunchKernelGGL((k_gj_panel_reg<4, 8>), dim3(nd), dim3(512), 0, s, d, j0, nb, piv, ldp, st);
    else if (max_m <= 384) hipLaunchKernelGGL((k_gj_panel_reg<6, 8>), dim3(nd), dim3(512), 0, s, d, j0, nb, piv, ldp, st);
    else hipLaunchKernelGGL((k_gj_panel_reg<8, 8>), dim3(nd), dim3(512), 0, s, d, j0, nb, piv, ldp, st);
    return;
  }
  const size_t lds = sizeof(double) * (size_t)max_m * (nb + 1);
  if (lds <= 150 * 1024) {
    if (lds > 64 * 1024) allow_lds(reinterpret_cast<const void*>(k_gj_panel<true>));
    hipLaunchKernelGGL(k_gj_panel<true>, dim3(nd), dim3(WG), lds, s, d, j0, nb, piv, ldp, st);
  } else {
    hipLaunchKernelGGL(k_gj_panel<false>, dim3(nd), dim3(WG), sizeof(double) * max_m, s, d, j0, nb, piv,
                       ldp, st);
  }
}

// Register Gauss-Jordan by size class: m <= 64 one wave, m <= 128 four waves,
// m <= 192 eight waves (kGjRegMax).
void launch_gj_reg(const InvDesc* d, int nd, int max_m, Status* st, hipStream_t s) {
  if (nd <= 0 || max_m <= 0) return;
  if (max_m <= 64) hipLaunchKernelGGL((k_gj_reg<8, 8, 8, 8>), dim3(nd), dim3(64), 0, s, d, st);
  else if (max_m <= 128) hipLaunchKernelGGL((k_gj_reg<32, 16, 4, 8>), dim3(nd), dim3(512), 0, s, d, st);
  else if (max_m <= kGjRegMax) hipLaunchKernelGGL((k_gj_reg<32, 16, 6, 12>), dim3(nd), dim3(512), 0, s, d, st);
}

void launch_gj_rest(const InvDesc* d, int nd, int max_m, int j0, int nb, const int* piv, int ldp,
                    double* tmp, size_t ldt, hipStream_t s) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(k_gj_rest, dim3(nd, cdiv(max_m, WG)), dim3(WG), 0, s, d, j0, nb, piv, ldp, tmp, ldt);
}

void launch_gj_unpermute(const InvDesc* d, int nd, int max_m, const int* piv, int ldp, hipStream_t s) {
  if (nd <= 0) return;
  hipLaunchKernelGGL(k_gj_unpermute, dim3(nd, cdiv(max_m, WG)), dim3(WG), 0, s, d, piv, ldp);
}

}  // namespace ifmm
