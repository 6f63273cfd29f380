// Kernel-function and Chebyshev operators of the FMM matrix on gfx950 (FP64):
// leaf interpolation matrices (L2P / P2M), near-field blocks (P2P), the M2L
// node-to-node kernel tables, and the passes of the FMM product used for the
// row-sum diagonal and for refinement residuals.  Points are in tree order.
#include "ifmm_internal.h"

namespace ifmm {

namespace {

typedef double md4 __attribute__((ext_vector_type(4)));

// K(r) of the built-in kernels (kind: ifmm_kernel_kind; ell is the length
// scale of the exp kernels and the parameter a of the numerical section's
// three singular kernels, each continuous at r = a with K(a) = 1 and with the
// limit 0 at r = 0).
__device__ inline double kval(KernelFn kf, double r) {
  const double a = kf.ell;
  switch (kf.kind) {
    case 0: return 1.0 / r;
    case 1: return exp(-r / a);
    case 2:  // r (log r - 1) / (a (log a - 1)) below a, log r / log a above
      if (r == 0.0) return 0.0;
      return r < a ? r * (log(r) - 1.0) / (a * (log(a) - 1.0)) : log(r) / log(a);
    case 3: return r < a ? r / a : a / r;
    case 4:  // r^3 (3 log r - 1) / (a^3 (3 log a - 1)) below a, r^2 log r / (a^2 log a) above
      if (r == 0.0) return 0.0;
      return r < a ? r * r * r * (3.0 * log(r) - 1.0) / (a * a * a * (3.0 * log(a) - 1.0))
                   : r * r * log(r) / (a * a * log(a));
    default: return r / (a * a) * exp(-r / a);  // 5: d/d ell of exp(-r / ell)
  }
}

__device__ inline double cheb_node(int p, int m) {
  return cos((2.0 * m + 1.0) * M_PI / (2.0 * p));  // m = 0..p-1
}

// l_m(s) for all m = 0..p-1.
__device__ inline void lagrange_all(int p, double s, double* out) {
  double t[kMaxP];
  for (int m = 0; m < p; ++m) t[m] = cheb_node(p, m);
  for (int m = 0; m < p; ++m) {
    double num = 1.0, den = 1.0;
    for (int k = 0; k < p; ++k)
      if (k != m) {
        num *= s - t[k];
        den *= t[m] - t[k];
      }
    out[m] = num / den;
  }
}

__device__ inline void leaf_box(int i, int kappa, double lox, double loy, double size,
                                double& cx, double& cy, double& h) {
  const double w = size / (double)(1 << kappa);
  cx = lox + (demorton_x(i) + 0.5) * w;
  cy = loy + (demorton_y(i) + 0.5) * w;
  h = 0.5 * w;
}

__global__ void k_leaf_interp(const double* __restrict__ pts, const int* __restrict__ start,
                              const int* __restrict__ cnt, int kappa, double lox, double loy,
                              double size, int p, double* dst, size_t stride, int ld) {
  const int i = blockIdx.x;
  const int n = cnt[i];
  double cx, cy, h;
  leaf_box(i, kappa, lox, loy, size, cx, cy, h);
  double* S = dst + (size_t)i * stride;
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    const double x = pts[2 * (start[i] + a)], y = pts[2 * (start[i] + a) + 1];
    double lx[kMaxP], ly[kMaxP];
    lagrange_all(p, (x - cx) / h, lx);
    lagrange_all(p, (y - cy) / h, ly);
    for (int mx = 0; mx < p; ++mx)
      for (int my = 0; my < p; ++my) S[a + (size_t)(mx * p + my) * ld] = lx[mx] * ly[my];
  }
}

// Near-field blocks of the factor; optionally also the FP64 near field of
// the product: leaf i's row block (n_i x the sources of its 3 x 3 neighbours
// in slot order, ld n_i) at near + near_off[i], zero on the self pairs.
template <class T>
__global__ void k_near(const double* __restrict__ pts, const int* __restrict__ start,
                       const int* __restrict__ cnt, const int* __restrict__ nbr9, KernelFn kf,
                       const double* __restrict__ d, T* P, size_t slot_stride, int ld,
                       double* __restrict__ near, const size_t* __restrict__ near_off) {
  const int i = blockIdx.x, s = blockIdx.y;
  const int j = nbr9[i * 9 + s];
  if (j < 0) return;
  const int ni = cnt[i], nj = cnt[j];
  T* B = P + ((size_t)i * 9 + s) * slot_stride;
  const int si = start[i], sj = start[j];
  double* Nb = nullptr;
  if (near) {
    int coff = 0;
    for (int u = 0; u < s; ++u) {
      const int ju = nbr9[i * 9 + u];
      if (ju >= 0) coff += cnt[ju];
    }
    Nb = near + near_off[i] + (size_t)coff * ni;
  }
  for (int e = threadIdx.x; e < ni * nj; e += blockDim.x) {
    const int a = e % ni, b = e / ni;
    double v;
    if (s == 4 && a == b) {
      v = d[si + a];
      if (Nb) Nb[e] = 0.0;
    } else {
      const double dx = pts[2 * (si + a)] - pts[2 * (sj + b)];
      const double dy = pts[2 * (si + a) + 1] - pts[2 * (sj + b) + 1];
      v = kval(kf, sqrt(dx * dx + dy * dy));
      if (Nb) Nb[e] = v;
    }
    B[a + (size_t)b * ld] = (T)v;
  }
}

__global__ void k_m2l_table(KernelFn kf, int p, double h, double* dst) {
  const int off = blockIdx.x;  // 0..48
  const int dx = off / 7 - 3, dy = off % 7 - 3;
  const int p2 = p * p;
  double* T = dst + (size_t)off * p2 * p2;
  for (int e = threadIdx.x; e < p2 * p2; e += blockDim.x) {
    const int m = e % p2, n = e / p2;
    const double xm = h * cheb_node(p, m / p), ym = h * cheb_node(p, m % p);
    const double xn = 2.0 * h * dx + h * cheb_node(p, n / p), yn = 2.0 * h * dy + h * cheb_node(p, n % p);
    const double ex = xm - xn, ey = ym - yn;
    T[m + (size_t)n * p2] = (dx == 0 && dy == 0 && m == n) ? 0.0 : kval(kf, sqrt(ex * ex + ey * ey));
  }
}

// ---------------------------------------------------------------- FMM passes
// Multipole/local node values are stored [cluster][rhs][p^2].
// P2M of every leaf: the Lagrange weights of a chunk of 64 points are
// formed once (one point per lane) and staged in LDS with the point values,
// then each lane accumulates one (node, column) coefficient over the chunk.
constexpr int P2M_WG = 64;
constexpr int P2M_RHS = 4;  // right-hand columns staged per pass
__global__ __launch_bounds__(P2M_WG) void k_p2m(const double* __restrict__ pts, const int* __restrict__ start,
                                                const int* __restrict__ cnt, int kappa, double lox, double loy,
                                                double size, int p, const double* __restrict__ x, int ldx,
                                                int nrhs, double* W) {
  const int i = blockIdx.x;
  const int p2 = p * p;
  const int n = cnt[i];
  double cx, cy, h;
  leaf_box(i, kappa, lox, loy, size, cx, cy, h);
  __shared__ double Lx[P2M_WG][kMaxP], Ly[P2M_WG][kMaxP], xs[P2M_RHS][P2M_WG];
  for (int r0 = 0; r0 < nrhs; r0 += P2M_RHS) {
    const int nr = min(P2M_RHS, nrhs - r0);
    double acc[(kMaxP * kMaxP * P2M_RHS + P2M_WG - 1) / P2M_WG];
    constexpr int NACC = (kMaxP * kMaxP * P2M_RHS + P2M_WG - 1) / P2M_WG;
#pragma unroll
    for (int q = 0; q < NACC; ++q) acc[q] = 0.0;
    for (int a0 = 0; a0 < n; a0 += P2M_WG) {
      const int a = a0 + threadIdx.x;
      if (a < n) {
        const int g = start[i] + a;
        lagrange_all(p, (pts[2 * g] - cx) / h, Lx[threadIdx.x]);
        lagrange_all(p, (pts[2 * g + 1] - cy) / h, Ly[threadIdx.x]);
        for (int r = 0; r < nr; ++r) xs[r][threadIdx.x] = x[g + (size_t)(r0 + r) * ldx];
      }
      __syncthreads();
      const int na = min(P2M_WG, n - a0);
#pragma unroll
      for (int q = 0; q < NACC; ++q) {
        const int e = threadIdx.x + q * P2M_WG;
        if (e >= p2 * nr) continue;
        const int m = e % p2, r = e / p2;
        const int mx = m / p, my = m % p;
        double v = acc[q];
        for (int b = 0; b < na; ++b) v = fma(Lx[b][mx] * Ly[b][my], xs[r][b], v);
        acc[q] = v;
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NACC; ++q) {
      const int e = threadIdx.x + q * P2M_WG;
      if (e >= p2 * nr) continue;
      const int m = e % p2, r = e / p2;
      W[((size_t)i * nrhs + r0 + r) * p2 + m] = acc[q];
    }
  }
}

__global__ void k_m2m(const double* __restrict__ E, int p, const double* __restrict__ Wc,
                      double* Wp, int nrhs) {
  const int P = blockIdx.x;
  const int p2 = p * p;
  for (int e = threadIdx.x; e < p2 * nrhs; e += blockDim.x) {
    const int m = e % p2, r = e / p2;
    double acc = 0.0;
    for (int c = 0; c < 4; ++c) {
      const double* Ec = E + (size_t)c * p2 * p2;
      const double* w = Wc + ((size_t)(4 * P + c) * nrhs + r) * p2;
      for (int mm = 0; mm < p2; ++mm) acc = fma(Ec[mm + (size_t)m * p2], w[mm], acc);
    }
    Wp[((size_t)P * nrhs + r) * p2 + m] = acc;
  }
}

// M2L of one level on the matrix cores (FP64): G_i = sum over the far-field
// slots of the 6 x 6 window of T(dx, dy) W_l, with T the node-to-node kernel
// block of offset (dx, dy) = (jx - ix, jy - iy).  One workgroup per 8 x 8
// block of clusters; wave w takes the 16 clusters of parity class
// (w & 1, w >> 1), laid out 4 x 4 with stride 2, so that every slot has the
// same offset for all 16 and the slot is one product (p^2 x p^2) x (p^2 x 16)
// by v_mfma_f64_16x16x4 (A: T read from global memory, L2-resident; B: the
// multipoles of the block's 12 x 12 window, staged in LDS with zeros outside
// the grid).  Output rows are split in 16-row tiles (RT of them), the inner
// dimension in steps of 4.  The A operand of the next far-field slot is
// loaded into a second register set while the current slot's products run
// (DB; for p <= 7, where two sets fit the registers).
template <int P, bool DB>
__device__ inline void m2l_wave(const double* __restrict__ table, const double* __restrict__ win, int px, int py,
                                int c, int kq, md4 (&acc)[(P * P + 15) / 16]) {
  constexpr int P2 = P * P, RT = (P2 + 15) / 16, KS = (P2 + 3) / 4, PS = P2 + 1;
  // this lane's cluster in the window: (2 + px + 2 (c % 4), 2 + py + 2 (c / 4))
  const double* w0 = win + ((2 + py + 2 * (c / 4)) * 12 + (2 + px + 2 * (c % 4))) * PS;
  auto near = [&](int s) {
    const int dx = s / 6 - 2 - px, dy = s % 6 - 2 - py;
    return dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1;
  };
  auto next_far = [&](int s) {  // 36 when none is left
    do ++s;
    while (s < 36 && near(s));
    return s;
  };
  auto load = [&](double (&buf)[RT][KS], int s) {
    const int dx = s / 6 - 2 - px, dy = s % 6 - 2 - py;
    const double* T = table + (size_t)((dx + 3) * 7 + (dy + 3)) * P2 * P2;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int m = 16 * t + c, n = 4 * ks + kq;
        buf[t][ks] = (m < P2 && n < P2) ? T[m + n * P2] : 0.0;
      }
  };
  auto comp = [&](const double (&buf)[RT][KS], int s) {
    const int dx = s / 6 - 2 - px, dy = s % 6 - 2 - py;
    const double* wl = w0 + (dy * 12 + dx) * PS;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int n = 4 * ks + kq;
      const double b = n < P2 ? wl[n] : 0.0;
#pragma unroll
      for (int t = 0; t < RT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(buf[t][ks], b, acc[t], 0, 0, 0);
    }
  };
  int s = next_far(-1);
  if constexpr (DB) {
    double ta[RT][KS], tb[RT][KS];
    load(ta, s);
    while (true) {
      const int s1 = next_far(s);
      load(tb, s1 < 36 ? s1 : s);  // unconditional: no branch between the loads and their use
      comp(ta, s);
      if (s1 >= 36) break;
      const int s2 = next_far(s1);
      load(ta, s2 < 36 ? s2 : s1);
      comp(tb, s1);
      if (s2 >= 36) break;
      s = s2;
    }
  } else {
    for (; s < 36; s = next_far(s)) {
      double ta[RT][KS];
      load(ta, s);
      comp(ta, s);
    }
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_m2l(int k, const double* __restrict__ table,
                                             const double* __restrict__ W, double* __restrict__ G,
                                             int nrhs) {
  constexpr int P2 = P * P, RT = (P2 + 15) / 16, PS = P2 + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  double* win = reinterpret_cast<double*>(smem);  // [12 * 12][PS]
  const int nside = 1 << k;
  const int nbs = nside >= 8 ? nside / 8 : 1;
  const int bx = 8 * ((int)blockIdx.x % nbs), by = 8 * ((int)blockIdx.x / nbs);
  const int lane = threadIdx.x % 64;  // 64-wide waves
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int px = w & 1, py = w >> 1;
  const int c = lane % 16, kq = lane / 16;
  const int ix = bx + px + 2 * (c % 4), iy = by + py + 2 * (c / 4);
  const bool live = ix < nside && iy < nside;
  for (int r = 0; r < nrhs; ++r) {
    if (r) __syncthreads();
    for (int e = threadIdx.x; e < 144 * P2; e += blockDim.x) {
      const int n = e % P2, cell = e / P2;
      const int jx = bx - 2 + cell % 12, jy = by - 2 + cell / 12;
      win[cell * PS + n] = (jx >= 0 && jy >= 0 && jx < nside && jy < nside)
                               ? W[((size_t)morton2(jx, jy) * nrhs + r) * P2 + n] : 0.0;
    }
    __syncthreads();
    md4 acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = md4{0, 0, 0, 0};
    m2l_wave<P, (P <= 7)>(table, win, px, py, c, kq, acc);
    if (live) {
      double* g = G + ((size_t)morton2(ix, iy) * nrhs + r) * P2;
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * t + 4 * v + kq;  // row of output value v of this lane
          if (m < P2) g[m] = acc[t][v];
        }
    }
  }
}

__global__ void k_l2l(const double* __restrict__ E, int p, const double* __restrict__ Gp, double* Gc,
                      int nrhs) {
  const int c = blockIdx.x;  // child index
  const int P = c >> 2, q = c & 3;
  const int p2 = p * p;
  const double* Ec = E + (size_t)q * p2 * p2;
  for (int e = threadIdx.x; e < p2 * nrhs; e += blockDim.x) {
    const int mm = e % p2, r = e / p2;
    const double* g = Gp + ((size_t)P * nrhs + r) * p2;
    double acc = 0.0;
    for (int m = 0; m < p2; ++m) acc = fma(Ec[mm + (size_t)m * p2], g[m], acc);
    Gc[((size_t)c * nrhs + r) * p2 + mm] += acc;
  }
}

__global__ void k_l2p_p2p(const double* __restrict__ pts, const int* __restrict__ start,
                          const int* __restrict__ cnt, const int* __restrict__ nbr9, int kappa,
                          double lox, double loy, double size, int p, KernelFn kf,
                          const double* __restrict__ G, const double* __restrict__ x, int ldx,
                          const double* __restrict__ d, double* y, int ldy, int nrhs) {
  const int i = blockIdx.x;
  const int p2 = p * p;
  const int n = cnt[i];
  double cx, cy, h;
  leaf_box(i, kappa, lox, loy, size, cx, cy, h);
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    const int g = start[i] + a;
    const double xa = pts[2 * g], ya = pts[2 * g + 1];
    double lx[kMaxP], ly[kMaxP];
    lagrange_all(p, (xa - cx) / h, lx);
    lagrange_all(p, (ya - cy) / h, ly);
    for (int r = 0; r < nrhs; ++r) {
      const double* gl = G + ((size_t)i * nrhs + r) * p2;
      double acc = 0.0;
      for (int m = 0; m < p2; ++m) acc = fma(lx[m / p] * ly[m % p], gl[m], acc);
      for (int s = 0; s < 9; ++s) {
        const int j = nbr9[i * 9 + s];
        if (j < 0) continue;
        for (int b = 0; b < cnt[j]; ++b) {
          const int gb = start[j] + b;
          if (gb == g) continue;
          const double dx = xa - pts[2 * gb], dy = ya - pts[2 * gb + 1];
          acc = fma(kval(kf, sqrt(dx * dx + dy * dy)), x[gb + (size_t)r * ldx], acc);
        }
      }
      if (d) acc = fma(d[g], x[g + (size_t)r * ldx], acc);
      y[g + (size_t)r * ldy] = acc;
    }
  }
}

// The same product with the near field read from its stored FP64 blocks
// (k_near): the terms in the same order, the self pairs skipped.
__global__ void k_l2p_near(const double* __restrict__ pts, const int* __restrict__ start,
                           const int* __restrict__ cnt, const int* __restrict__ nbr9, int kappa,
                           double lox, double loy, double size, int p, const double* __restrict__ near,
                           const size_t* __restrict__ near_off, const double* __restrict__ G,
                           const double* __restrict__ x, int ldx, const double* __restrict__ d, double* y,
                           int ldy, int nrhs) {
  const int i = blockIdx.x;
  const int p2 = p * p;
  const int n = cnt[i];
  double cx, cy, h;
  leaf_box(i, kappa, lox, loy, size, cx, cy, h);
  const double* B = near + near_off[i];
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    const int g = start[i] + a;
    const double xa = pts[2 * g], ya = pts[2 * g + 1];
    double lx[kMaxP], ly[kMaxP];
    lagrange_all(p, (xa - cx) / h, lx);
    lagrange_all(p, (ya - cy) / h, ly);
    for (int r = 0; r < nrhs; ++r) {
      const double* gl = G + ((size_t)i * nrhs + r) * p2;
      const double* xr = x + (size_t)r * ldx;
      double acc = 0.0;
      for (int m = 0; m < p2; ++m) acc = fma(lx[m / p] * ly[m % p], gl[m], acc);
      // the stored block holds 0 for the point itself (the diagonal is d);
      // one running sum in column order (the refinement's residual floor
      // depends on this rounding order)
      const double* Ba = B + a;
      for (int s = 0; s < 9; ++s) {
        const int j = nbr9[i * 9 + s];
        if (j < 0) continue;
        const int nj = cnt[j];
        const double* xs = xr + start[j];
        int b = 0;
        for (; b + 8 <= nj; b += 8) {  // eight loads in flight
          double v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = Ba[(size_t)(b + u) * n];
#pragma unroll
          for (int u = 0; u < 8; ++u) acc = fma(v[u], xs[b + u], acc);
        }
        for (; b < nj; ++b) acc = fma(Ba[(size_t)b * n], xs[b], acc);
        Ba += (size_t)nj * n;
      }
      if (d) acc = fma(d[g], xr[g], acc);
      y[g + (size_t)r * ldy] = acc;
    }
  }
}

__global__ void k_gather_rows(const double* __restrict__ src, int ld_src, const int* __restrict__ idx,
                              int n, int nrhs, double* dst, int ld_dst) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * nrhs) return;
  const int i = (int)(e % n), r = (int)(e / n);
  dst[i + (size_t)r * ld_dst] = src[idx[i] + (size_t)r * ld_src];
}

__global__ void k_scatter_rows(const double* __restrict__ src, int ld_src, const int* __restrict__ idx,
                               int n, int nrhs, double* dst, int ld_dst) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * nrhs) return;
  const int i = (int)(e % n), r = (int)(e / n);
  dst[idx[i] + (size_t)r * ld_dst] = src[i + (size_t)r * ld_src];
}

__global__ void k_colnorm2(const double* __restrict__ x, int n, int nrhs, int ld, double* out) {
  __shared__ double red[4];
  const int r = blockIdx.y;
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += (size_t)gridDim.x * blockDim.x) {
    const double v = x[i + (size_t)r * ld];
    s += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out + r, red[0] + red[1] + red[2] + red[3]);
}

}  // namespace

void launch_colnorm2(const double* x, int n, int nrhs, int ld, double* out, hipStream_t s) {
  int nb = (n + 255) / 256;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_colnorm2, dim3(nb, nrhs), dim3(256), 0, s, x, n, nrhs, ld, out);
}

void launch_leaf_interp(const double* pts, const int* leaf_start, const int* leaf_n, int nleaf,
                        int kappa, double lox, double loy, double size, int p, double* dst,
                        size_t stride, int ld, int max_n, hipStream_t s) {
  (void)max_n;
  hipLaunchKernelGGL(k_leaf_interp, dim3(nleaf), dim3(64), 0, s, pts, leaf_start, leaf_n, kappa,
                     lox, loy, size, p, dst, stride, ld);
}

void launch_near_field(const double* pts, const int* leaf_start, const int* leaf_n,
                       const int* nbr9, int nleaf, KernelFn kf, const double* d, void* P, int f32,
                       size_t slot_stride, int ld, int max_n, double* near, const size_t* near_off,
                       hipStream_t s) {
  (void)max_n;
  if (f32)
    hipLaunchKernelGGL(k_near<float>, dim3(nleaf, 9), dim3(256), 0, s, pts, leaf_start, leaf_n, nbr9, kf,
                       d, static_cast<float*>(P), slot_stride, ld, near, near_off);
  else
    hipLaunchKernelGGL(k_near<double>, dim3(nleaf, 9), dim3(256), 0, s, pts, leaf_start, leaf_n, nbr9, kf,
                       d, static_cast<double*>(P), slot_stride, ld, near, near_off);
}

void launch_m2l_table(KernelFn kf, int p, double h, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_m2l_table, dim3(49), dim3(256), 0, s, kf, p, h, dst);
}

void launch_p2m(const double* pts, const int* leaf_start, const int* leaf_n, int nleaf, int kappa,
                double lox, double loy, double size, int p, const double* x, int ldx, int nrhs,
                double* W, hipStream_t s) {
  hipLaunchKernelGGL(k_p2m, dim3(nleaf), dim3(P2M_WG), 0, s, pts, leaf_start, leaf_n, kappa, lox, loy,
                     size, p, x, ldx, nrhs, W);
}

void launch_m2m(const double* E, int p, int nc_parent, const double* Wc, double* Wp, int nrhs,
                hipStream_t s) {
  hipLaunchKernelGGL(k_m2m, dim3(nc_parent), dim3(64), 0, s, E, p, Wc, Wp, nrhs);
}

template <int P>
void m2l_go(int k, const double* table, const double* W, double* G, int nrhs, hipStream_t s) {
  const int nside = 1 << k, nbs = nside >= 8 ? nside / 8 : 1;
  const size_t lds = (size_t)144 * (P * P + 1) * sizeof(double);
  if (lds > 64 * 1024) allow_lds(reinterpret_cast<const void*>(k_m2l<P>));
  hipLaunchKernelGGL(k_m2l<P>, dim3(nbs * nbs), dim3(256), lds, s, k, table, W, G, nrhs);
}

void launch_m2l(int p, int k, const double* table, const double* W, double* G, int nrhs,
                hipStream_t s) {
  if (k < 2 || nrhs <= 0) return;
  switch (p) {
    case 1: m2l_go<1>(k, table, W, G, nrhs, s); break;
    case 2: m2l_go<2>(k, table, W, G, nrhs, s); break;
    case 3: m2l_go<3>(k, table, W, G, nrhs, s); break;
    case 4: m2l_go<4>(k, table, W, G, nrhs, s); break;
    case 5: m2l_go<5>(k, table, W, G, nrhs, s); break;
    case 6: m2l_go<6>(k, table, W, G, nrhs, s); break;
    case 7: m2l_go<7>(k, table, W, G, nrhs, s); break;
    default: m2l_go<8>(k, table, W, G, nrhs, s); break;
  }
}

void launch_l2l(const double* E, int p, int nc_parent, const double* Gp, double* Gc, int nrhs,
                hipStream_t s) {
  hipLaunchKernelGGL(k_l2l, dim3(4 * nc_parent), dim3(64), 0, s, E, p, Gp, Gc, nrhs);
}

void launch_l2p_p2p(const double* pts, const int* leaf_start, const int* leaf_n, const int* nbr9,
                    int nleaf, int kappa, double lox, double loy, double size, int p, KernelFn kf,
                    const double* G, const double* x, int ldx, const double* d, double* y,
                    int ldy, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_l2p_p2p, dim3(nleaf), dim3(64), 0, s, pts, leaf_start, leaf_n, nbr9, kappa,
                     lox, loy, size, p, kf, G, x, ldx, d, y, ldy, nrhs);
}

void launch_l2p_near(const double* pts, const int* leaf_start, const int* leaf_n, const int* nbr9,
                     int nleaf, int kappa, double lox, double loy, double size, int p, const double* near,
                     const size_t* near_off, const double* G, const double* x, int ldx, const double* d,
                     double* y, int ldy, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_l2p_near, dim3(nleaf), dim3(64), 0, s, pts, leaf_start, leaf_n, nbr9, kappa, lox, loy,
                     size, p, near, near_off, G, x, ldx, d, y, ldy, nrhs);
}

void launch_gather_rows(const double* src, int ld_src, const int* idx, int n, int nrhs,
                        double* dst, int ld_dst, hipStream_t s) {
  const size_t tot = (size_t)n * nrhs;
  if (tot == 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src,
                     ld_src, idx, n, nrhs, dst, ld_dst);
}

void launch_scatter_rows(const double* src, int ld_src, const int* idx, int n, int nrhs,
                         double* dst, int ld_dst, hipStream_t s) {
  const size_t tot = (size_t)n * nrhs;
  if (tot == 0) return;
  hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src,
                     ld_src, idx, n, nrhs, dst, ld_dst);
}

}  // namespace ifmm
