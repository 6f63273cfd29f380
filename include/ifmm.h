/*
 * ifmm.h -- C-ABI of the MI355X (gfx950) Inverse Fast Multipole Method.
 *
 * The library factors and solves A x = b where A is an FMM matrix on 2D
 * points: A_ij = K(|x_i - x_j|) for i != j, with the far field represented
 * through nested Chebyshev interpolation (the "FMM matrix" of Ambikasaran &
 * Darve, Section 2.2), and a diagonal chosen by a rule below.  The problem
 * statement follows Section 1 (solve A x = b to a tolerance eps, A an FMM
 * matrix) and the benchmark equation of Section 5 (sigma_i + sum_{j != i}
 * K sigma_j = f_i is the special case diag_mode = CONST, c0 = 1).
 *
 * The factorisation is Algorithm 1 (elimination of the extended sparse system
 * level by level, with fill between well-separated clusters recompressed into
 * the M2L / P2M / L2P operators) and the solve is Algorithm 2 (back
 * substitution in reverse order); factor and solve are decoupled (end of
 * Section 4.2.2), so one factor serves many right-hand sides.
 *
 * Conventions
 *  - All arrays passed in or out are DEVICE pointers on the current HIP
 *    device; the caller owns them (the library never frees them).
 *  - points: [n][2] row-major (x0, y0, x1, y1, ...), FP64.
 *  - b, x, y: [nrhs][n] column-major (leading dimension n), FP64, in the
 *    caller's point order.
 *  - Work is enqueued on `stream` (a hipStream_t, NULL = default stream).
 *    ifmm_factor and ifmm_solve synchronise that stream before returning;
 *    a caller may destroy a stream once the call that used it returned and
 *    use the handle on other streams (ifmm_destroy releases the handle's
 *    blocks on the stream of its last call: that one must still exist).
 *  - Every call returns a status; no exception crosses the ABI.  On error the
 *    outputs are left untouched except where stated.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef IFMM_H_
#define IFMM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ifmm_plan* ifmm_t;

typedef enum {
  IFMM_OK = 0,
  IFMM_EINVAL = 1,     /* invalid argument (sizes, NaN/Inf, points outside the box, duplicates) */
  IFMM_ENOMEM = 2,     /* device or pinned-host allocation failed */
  IFMM_ESINGULAR = 3,  /* a pivot block was exactly singular */
  IFMM_ENOTCONV = 4,   /* refinement did not reach refine_tol (x holds the best iterate) */
  IFMM_EDEVICE = 5,    /* a HIP runtime error */
  IFMM_ESIZE = 6       /* ifmm_matvec_noalloc: the product needs more than its fixed workspace */
} ifmm_status;

typedef enum {
  IFMM_K_INV_R = 0,    /* K(r) = 1/r   (Section 1, Green's functions table) */
  IFMM_K_EXP = 1,      /* K(r) = exp(-r/ell) (Section 1, covariance functions table) */
  /* The three singular kernels of Section 5 (numerical benchmarks), parameter
     a = ell (> 0, != 1), each continuous at r = a with K(a) = 1, K(0) = 0: */
  IFMM_K_LOG_A = 2,    /* (i)   r (log r - 1) / (a (log a - 1)) for r < a, log r / log a else */
  IFMM_K_INV_R_A = 3,  /* (ii)  r / a for r < a, a / r else */
  IFMM_K_R2LOG_A = 4,  /* (iii) r^3 (3 log r - 1) / (a^3 (3 log a - 1)) for r < a,
                                r^2 log r / (a^2 log a) else */
  IFMM_K_EXP_DELL = 5  /* d/d ell exp(-r/ell) = (r / ell^2) exp(-r/ell): entries of dA/d ell
                          of the exp kernel (for ifmm_matvec_kernel) */
} ifmm_kernel_kind;

typedef enum {
  IFMM_DIAG_ROWSUM = 0, /* A_ii = c0 + sum_{j != i} A_ij over the FMM matrix */
  IFMM_DIAG_CONST = 1,  /* A_ii = c0 (e.g. K(0) + sigma^2 for exp, 1 for Section 5) */
  IFMM_DIAG_VECTOR = 2  /* A_ii = diag[i], a caller-supplied device array (c0 unused) */
} ifmm_diag_mode;

typedef struct {
  int kind;            /* ifmm_kernel_kind */
  double ell;          /* length scale of IFMM_K_EXP / _EXP_DELL, parameter a of kinds 2-4 (> 0) */
  int diag_mode;       /* ifmm_diag_mode */
  double c0;
  const double* diag;  /* IFMM_DIAG_VECTOR only: device [n], caller's point order, finite
                          (a non-finite entry gives EINVAL); read during ifmm_factor only,
                          the library keeps its own copy */
} ifmm_kernel;

/*
 * Scalar type of the factor's stored blocks (the off-pivot blocks, bases,
 * M2L operators and fill).  With IFMM_FP32 (the mixed-precision factor) the
 * Schur updates and the fill recompression run in FP32 with FP32
 * accumulation; the pivot-block inverses, the top system, the FMM product,
 * the residuals and every solution vector stay FP64, so refinement recovers
 * an FP64-accurate solution.  The relative compression threshold of an FP32
 * factor is max(eps, 2.5e-7): pivot norms below that are FP32 rounding noise.
 */
typedef enum {
  IFMM_FP64 = 0,
  IFMM_FP32 = 1
} ifmm_precision;

typedef struct {
  int r_max;           /* rank cap of the compressed bases; 0 = 2 p^2; must be >= p^2, <= 128 */
  double refine_tol;   /* 0: plain solve; > 0: FP64 iterative refinement with the FMM product
                          until ||b - A x|| / ||b|| <= refine_tol for every column */
  int refine_maxit;    /* refinement sweeps (0 = 30) */
  double box_lo[2];    /* root box [lo, lo + size]^2 containing every point */
  double box_size;     /* 0 = unit square [0,1]^2 */
  int profile;         /* time batched kernel launches with HIP events (ifmm_stats): 0 off,
                          1 every family, else bit f + 1 set times family f only (the
                          families of ifmm_stats_t.kernel_*; e.g. 1 << 9: elimination steps) */
  int precision;       /* ifmm_precision of the factor (0 = FP64) */
} ifmm_options;

typedef struct {
  int iterations;          /* refinement sweeps done (0 = plain solve) */
  double residual;         /* final max over columns of ||b - A x|| / ||b|| (when refining) */
  double history[32];      /* residual after the direct solve and after each sweep */
  double solve_ms;         /* wall time of this call */
} ifmm_solve_info;

typedef struct {
  int64_t n;
  int kappa;               /* leaf level (levels 2..kappa are eliminated) */
  int p;                   /* Chebyshev nodes per dimension */
  int max_rank;            /* largest rank met (r_m of Section 5) */
  int level_max_rank[16];
  double level_mean_rank[16];
  int top_size;            /* size of the dense level-2 multipole system */
  double assembly_ms;      /* t_a: tree, operators, near field, weights */
  double factor_ms;        /* t_f: Algorithm 1 */
  double last_solve_ms;    /* t_s of the last ifmm_solve (including refinement) */
  double factor_bytes;     /* device bytes held by the factor */
  double factor_flops;     /* counted FP64 flops of the factorisation */
  /* With ifmm_options.profile: per batched-kernel family, accumulated over the
     handle's life.  Slot f + 16 q: family f -- 0 gemm, 1 add/copy, 2 basis
     (unused), 3 Householder QR, 4 column-pivoted QR, 5 basis formation,
     6 stacked R factor, 7 pivot inverse, 8 Schur updates of the
     elimination, 9 basis change of touched clusters, 10 far-field weight
     stacks, 11 solve sweeps, 12 the other elimination steps (pivot build,
     X = D^-1 B, M2L row, fill projection); 13..15 unused -- with
     q = 1 for launches whose blocks are FP32 (gemm: both operands FP32; add:
     FP32 destination).  flops / bytes are the algorithmic counts of the
     launches (bytes at storage size). */
  int64_t kernel_launches[32];
  double kernel_ms[32];
  double kernel_flops[32];
  double kernel_bytes[32];
  int precision;           /* ifmm_precision of the factor */
  int level_cap_hits[16];  /* compressions per level whose rank reached r_max while the
                              cluster had more rows (the cap may have truncated there) */
} ifmm_stats_t;

/*
 * Factor the FMM matrix of `n` points (Algorithm 1).
 *   points     device [n][2], inside the root box (default [0,1]^2)
 *   k          kernel and diagonal rule
 *   eps        relative truncation tolerance of the fill compression (>= 0;
 *              eps = 0 keeps every direction up to the rank cap and needs an
 *              explicit opt->r_max: the default cap would truncate silently)
 *   leaf_size  mean leaf occupancy bound: depth = max(2, ceil(log4(n / leaf_size)))
 *   rank       p^2, the Chebyshev interpolation rank, 1 <= p <= 8
 *   opt        NULL for defaults
 *   out        receives the handle (owns all factor memory; free with ifmm_destroy)
 * Errors: EINVAL (n < 16, rank not a perfect square, p > 8, leaf_size < 1,
 * eps < 0 or NaN, eps = 0 without opt->r_max, kernel parameters, a null or
 * non-finite diagonal vector, unknown precision, non-finite or out-of-box or
 * duplicate points), ENOMEM, ESINGULAR, EDEVICE.
 */
ifmm_status ifmm_factor(const double* points, int64_t n, const ifmm_kernel* k, double eps,
                        int leaf_size, int rank, const ifmm_options* opt, void* stream,
                        ifmm_t* out);

/*
 * Solve A x = b for nrhs columns (Algorithm 2, optionally refined).
 *   b, x  device [nrhs][n]; x may not alias b.
 *   info  optional (host), filled on OK and on ENOTCONV.
 * Errors: EINVAL (null handle/pointers, nrhs < 1 or > 64), ENOTCONV (x holds
 * the best iterate), ENOMEM, EDEVICE.
 */
ifmm_status ifmm_solve(ifmm_t h, const double* b, double* x, int nrhs, void* stream,
                       ifmm_solve_info* info);

/*
 * Batched factorisation of `count` independent problems, each exactly as
 * ifmm_factor(points[i], n[i], &kernels[i], eps, leaf_size, rank, opt, ...)
 * would factor it (uneven sizes and different kernels allowed; Section
 * 4.2.2's decoupling of factor and solve).  `threads` host threads (0 = 4,
 * at most 64) each drive problems in turn on a worker stream of their own
 * (created by the library once per device and worker, kept until the
 * process ends), so the launches of different problems run concurrently on
 * the device (each problem's factorisation reads its new ranks back to the
 * host once per colour phase; concurrent problems fill the device while one
 * waits).  The worker streams overlap best when the process's HIP runtime
 * opens at least `threads` hardware queues (GPU_MAX_HW_QUEUES, read when the
 * runtime starts; its default 4 makes the streams of more threads share 4
 * queues).  The inputs must be ready on `stream`; on return every
 * factorisation is complete and the handles use `stream`.  Results equal
 * those of ifmm_factor bit for bit.  Concurrent batched calls share the
 * worker streams.
 *   out[i], status[i]: host arrays of count entries (out[i] = NULL where
 *   status[i] != IFMM_OK).
 * Returns IFMM_OK if every problem succeeded, else the status of a failed
 * one (EINVAL for null arrays or count < 1, EDEVICE if a worker stream could
 * not be created).
 */
ifmm_status ifmm_factor_batched(int count, const double* const* points, const int64_t* n,
                                const ifmm_kernel* kernels, double eps, int leaf_size, int rank,
                                const ifmm_options* opt, int threads, void* stream, ifmm_t* out,
                                ifmm_status* status);

/*
 * Batched solve: ifmm_solve(h[i], b[i], x[i], nrhs, ...) for i < count,
 * concurrently on `threads` host threads with a stream each (as above).  The
 * handles must be distinct; info (optional) and status are host arrays of
 * count entries.  Returns IFMM_OK if every solve succeeded, else the status
 * of a failed one.
 */
ifmm_status ifmm_solve_batched(int count, const ifmm_t* h, const double* const* b, double* const* x,
                               int nrhs, int threads, void* stream, ifmm_solve_info* info,
                               ifmm_status* status);

/* y = A x with the FMM product in FP64 (the matrix that is factored). */
ifmm_status ifmm_matvec(ifmm_t h, const double* x, double* y, int nrhs, void* stream);

/*
 * y = A_k x: the FMM matrix of another kernel k (with k's own diagonal rule)
 * on the tree and Chebyshev bases of h, in FP64 (near field evaluated, not
 * stored).  The Chebyshev interpolation is linear in the kernel, so with
 * k = IFMM_K_EXP_DELL (ell of the factored exp kernel), IFMM_DIAG_CONST and
 * c0 = 0 this is exactly dA/d ell of the factored matrix exp(-r/ell) +
 * sigma^2 I (the products a gradient with respect to the kernel's
 * hyperparameters needs; Section 1's covariance kernels).
 * Errors: EINVAL (null pointers, nrhs < 1 or > 64, invalid kernel; 1/r on a
 * handle whose kernel is not 1/r: equal points were not ruled out), ENOMEM,
 * EDEVICE.
 */
ifmm_status ifmm_matvec_kernel(ifmm_t h, const ifmm_kernel* k, const double* x, double* y, int nrhs,
                               void* stream);

/*
 * y = A x like ifmm_matvec, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): every intermediate (x and y in tree order, the multipole and
 * local coefficients of every level) lives in a fixed 64 MiB device array
 * that the library holds on each device it runs on until the process ends;
 * no device memory is allocated or freed.  The work is only enqueued on
 * `stream` (no wait).  The fixed array is shared by every call on a device:
 * calls that overlap on one device (different streams, threads or handles)
 * race and must be ordered by the caller.  Nothing in it needs clearing
 * between calls (each pass writes its output before it is read).
 * Needs ifmm_matvec_noalloc_bytes(h, nrhs) <= 64 MiB, i.e.
 * 8 (2 n nrhs + 2 p^2 nrhs sum_{k=2..kappa} 4^k) bytes (n = 2^20, p = 6:
 * 29.4 MB per column, so up to 2 columns).
 * Errors: EINVAL (null handle or pointers, nrhs < 1 or > 64), ESIZE (beyond
 * the fixed workspace), EDEVICE.
 */
ifmm_status ifmm_matvec_noalloc(ifmm_t h, const double* x, double* y, int nrhs, void* stream);

/* Bytes of fixed workspace ifmm_matvec_noalloc needs for nrhs columns (0 for a null handle). */
size_t ifmm_matvec_noalloc_bytes(ifmm_t h, int nrhs);

/* Copy the diagonal of A (caller's point order) into device array d[n]. */
ifmm_status ifmm_diagonal(ifmm_t h, double* d, void* stream);

/* Statistics of the factorisation (host struct). */
ifmm_status ifmm_stats(ifmm_t h, ifmm_stats_t* s);

/* Final rank of every cluster of `level` (Morton order) into host out[4^level]. */
ifmm_status ifmm_ranks(ifmm_t h, int level, int* out, int count);

/* Frees the handle and every device buffer it holds.  The buffers go to a
 * process-wide cache that later ifmm_factor calls reuse (a block serves a
 * request of at least 4/5 of its size; at most 60% of the device memory stays
 * cached; a failed device allocation frees the cache and retries). */
void ifmm_destroy(ifmm_t h);

/* Returns the cached device memory of every device to the HIP runtime. */
void ifmm_release_cached_memory(void);
const char* ifmm_status_string(ifmm_status s);

#ifdef __cplusplus
}
#endif
#endif /* IFMM_H_ */
