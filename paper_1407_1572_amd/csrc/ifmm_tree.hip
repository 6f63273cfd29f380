// Quadtree of the points on gfx950 (Section 2: the hierarchical subdivision of
// the square domain that the FMM and its inverse share).  Every point gets the
// Morton index of its leaf box; a stable radix sort by that index gives the
// tree order (points of one leaf contiguous, original order kept within a
// leaf); a histogram gives the leaf populations.  Validation (finite, inside
// the box, distinct within a leaf for the singular kernel) sets a flag that the
// host reads back with the populations.
#include "ifmm_internal.h"

#include <algorithm>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

namespace ifmm {

namespace {

// key[a] = Morton index of the leaf box of point a, idx[a] = a, leaf_n[key]++.
// A point outside the box or not finite sets *bad and is filed in box 0.
__global__ void __launch_bounds__(256) k_tree_keys(const double* __restrict__ pts, int n, double lox,
                                                   double loy, double size, int nb, int* __restrict__ key,
                                                   int* __restrict__ idx, int* __restrict__ leaf_n,
                                                   int* __restrict__ bad) {
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= n) return;
  const double x = pts[2 * a], y = pts[2 * a + 1];
  int k = 0;
  if (!isfinite(x) || !isfinite(y) || x < lox || y < loy || x > lox + size || y > loy + size) {
    *bad = 1;
  } else {
    int ix = (int)floor((x - lox) / size * nb), iy = (int)floor((y - loy) / size * nb);
    ix = min(max(ix, 0), nb - 1);
    iy = min(max(iy, 0), nb - 1);
    k = morton2(ix, iy);
  }
  key[a] = k;
  idx[a] = a;
  atomicAdd(leaf_n + k, 1);
}

// A non-finite entry of v sets *bad (the caller's diagonal).
__global__ void __launch_bounds__(256) k_check_finite(const double* __restrict__ v, int n, int* __restrict__ bad) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n && !isfinite(v[i])) *bad = 1;
}

// Sorted coordinates: dst[i] = src[perm[i]] for the (x, y) pairs.
__global__ void __launch_bounds__(256) k_tree_gather(const double* __restrict__ src,
                                                     const int* __restrict__ perm, int n,
                                                     double2* __restrict__ dst) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const int a = perm[i];
    dst[i] = make_double2(src[2 * a], src[2 * a + 1]);
  }
}

// Two equal points in one leaf set *bad (the 1/r kernel is singular there).
// One workgroup per leaf, all pairs compared.
__global__ void __launch_bounds__(256) k_tree_distinct(const double2* __restrict__ pts,
                                                       const int* __restrict__ leaf_start,
                                                       const int* __restrict__ leaf_n,
                                                       int* __restrict__ bad) {
  const int i = blockIdx.x, n = leaf_n[i];
  if (n < 2) return;
  const double2* p = pts + leaf_start[i];
  int hit = 0;
  for (int a = threadIdx.x; a < n; a += 256) {
    const double2 u = p[a];
    for (int b = a + 1; b < n; ++b) {
      const double2 v = p[b];
      hit |= (u.x == v.x) & (u.y == v.y);
    }
  }
  if (hit) *bad = 1;
}

// Leaf rows of a tree-order vector (ld ldv, nrhs columns) to / from the
// per-leaf blocks of the solve (leaf i at blk + i bstride, ld ldb).
template <bool kToBlocks>
__global__ void __launch_bounds__(256) k_leaf_copy(double* __restrict__ v, int ldv, double* __restrict__ blk,
                                                   size_t bstride, int ldb, const int* __restrict__ start,
                                                   const int* __restrict__ cnt, int nrhs) {
  const int i = blockIdx.x, n = cnt[i];
  double* b = blk + (size_t)i * bstride;
  double* x = v + start[i];
  for (int e = threadIdx.x; e < n * nrhs; e += 256) {
    const int a = e % n, r = e / n;
    if (kToBlocks) b[a + (size_t)r * ldb] = x[a + (size_t)r * ldv];
    else x[a + (size_t)r * ldv] = b[a + (size_t)r * ldb];
  }
}

__global__ void __launch_bounds__(256) k_fill(double* __restrict__ x, size_t n, double v) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void __launch_bounds__(256) k_add_const(double* __restrict__ x, size_t n, double v) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] += v;
}

}  // namespace

hipError_t tree_scratch_bytes(int n, int nleaf, int bits, size_t* bytes) {
  size_t a = 0, b = 0;
  hipError_t e = rocprim::radix_sort_pairs(nullptr, a, (int*)nullptr, (int*)nullptr, (int*)nullptr, (int*)nullptr,
                                           (size_t)n, 0u, (unsigned)bits);
  if (e != hipSuccess) return e;
  e = rocprim::exclusive_scan(nullptr, b, (int*)nullptr, (int*)nullptr, 0, (size_t)nleaf, rocprim::plus<int>());
  *bytes = a > b ? a : b;
  return e;
}

hipError_t launch_tree_build(const double* pts, int n, double lox, double loy, double size, int kappa,
                       int* key_in, int* key_out, int* idx, int* perm, int* leaf_n, int* leaf_start,
                       int* bad, double* spts, void* tmp, size_t tmp_bytes, hipStream_t s) {
  const int nb = 1 << kappa, nleaf = nb * nb;
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_tree_keys, dim3(g), dim3(256), 0, s, pts, n, lox, loy, size, nb, key_in, idx,
                     leaf_n, bad);
  size_t t = tmp_bytes;
  hipError_t e = rocprim::radix_sort_pairs(tmp, t, key_in, key_out, idx, perm, (size_t)n, 0u, (unsigned)(2 * kappa), s);
  if (e != hipSuccess) return e;
  t = tmp_bytes;
  e = rocprim::exclusive_scan(tmp, t, leaf_n, leaf_start, 0, (size_t)nleaf, rocprim::plus<int>(), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tree_gather, dim3(g), dim3(256), 0, s, pts, perm, n, reinterpret_cast<double2*>(spts));
  return hipGetLastError();
}

void launch_tree_distinct(const double* spts, const int* leaf_start, const int* leaf_n, int nleaf,
                          int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_tree_distinct, dim3(nleaf), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(spts), leaf_start, leaf_n, bad);
}

void launch_leaf_gather(const double* v, int ldv, double* blk, size_t bstride, int ldb, const int* leaf_start,
                        const int* leaf_n, int nleaf, int nrhs, hipStream_t s) {
  if (nleaf <= 0) return;
  hipLaunchKernelGGL(k_leaf_copy<true>, dim3(nleaf), dim3(256), 0, s, const_cast<double*>(v), ldv, blk, bstride,
                     ldb, leaf_start, leaf_n, nrhs);
}

void launch_leaf_scatter(const double* blk, size_t bstride, int ldb, double* v, int ldv, const int* leaf_start,
                         const int* leaf_n, int nleaf, int nrhs, hipStream_t s) {
  if (nleaf <= 0) return;
  hipLaunchKernelGGL(k_leaf_copy<false>, dim3(nleaf), dim3(256), 0, s, v, ldv, const_cast<double*>(blk), bstride,
                     ldb, leaf_start, leaf_n, nrhs);
}

void launch_check_finite(const double* v, int n, int* bad, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, n, bad);
}

// n 32-bit words into pinned host memory (dst: its device address), then a
// system-scope fence: the host reads them once a later event on the stream
// has completed.  One short launch in place of a DMA copy, whose start-up
// would otherwise stall the stream on a read-back the host waits for.
__global__ void __launch_bounds__(256) k_copy_to_host(const unsigned* __restrict__ src, unsigned* dst, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
  __threadfence_system();
}

void launch_copy_to_host(const void* src, void* dst_dev, size_t bytes, hipStream_t s) {
  const int n = (int)(bytes / 4);
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy_to_host, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     static_cast<const unsigned*>(src), static_cast<unsigned*>(dst_dev), n);
}

// bytes from pinned host memory (src: its device address) into device
// memory, 16 bytes per lane and step: an upload that stays on the stream's
// compute queue (a DMA copy between two launches costs the hand-over
// between the copy engine and the compute queue, twice).
__global__ void __launch_bounds__(256) k_copy_from_host(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                        size_t n16, const unsigned char* __restrict__ src_tail,
                                                        unsigned char* __restrict__ dst_tail, int tail) {
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
  if (blockIdx.x == 0 && (int)threadIdx.x < tail) dst_tail[threadIdx.x] = src_tail[threadIdx.x];
}

void launch_copy_from_host(const void* src_dev, void* dst, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  const size_t n16 = bytes / 16;
  const int tail = (int)(bytes % 16);
  const unsigned blocks = (unsigned)std::max<size_t>(1, std::min<size_t>((n16 + 255) / 256, 1024));
  const unsigned char* st = static_cast<const unsigned char*>(src_dev) + n16 * 16;
  unsigned char* dt = static_cast<unsigned char*>(dst) + n16 * 16;
  hipLaunchKernelGGL(k_copy_from_host, dim3(blocks), dim3(256), 0, s, static_cast<const uint4*>(src_dev),
                     static_cast<uint4*>(dst), n16, st, dt, tail);
}

void launch_fill(double* x, size_t n, double v, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, v);
}

void launch_add_const(double* x, size_t n, double v, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_add_const, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, v);
}

}  // namespace ifmm
