// Host orchestration of the IFMM on one MI355X: tree and cluster lists,
// assembly of the extended sparse system, Algorithm 1 (elimination with
// compression of well-separated fill), Algorithm 2 (back substitution), the
// FMM product and FP64 iterative refinement, behind the C-ABI of ifmm.h.
//
// The kernels of the C-ABI are radial, hence symmetric: the reordered extended
// system is symmetric (P2M = L2P^T), so every cluster carries one basis
// (V = U, VP = UP) and fill is compressed from the row side only.
//
// The host plans integer work only (which block feeds which batched kernel);
// every floating-point step runs in the gfx950 kernels.  Per colour phase the
// host reads back the new ranks once (they decide the block shapes of the
// next steps) -- that is the only synchronisation inside the factorisation.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <atomic>
#include <mutex>
#include <thread>
#include <new>
#include <unordered_map>
#include <string>
#include <tuple>
#include <functional>
#include <vector>

#include "../../include/ifmm.h"
#include "ifmm_internal.h"

using namespace ifmm;

namespace {

struct HipError {
  hipError_t e;
  int line;  // where in this file the failing call is
};
struct NoMem {};
struct BadArg {};
struct Broken {  // an internal invariant failed
  const char* what;
  int line;
};

#define HIP_OK(x)                                      \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) throw HipError{e_, __LINE__};          \
  } while (0)

// Process-wide, stream-ordered cache of device blocks.  A factorisation
// holds tens of GB in a few hundred large blocks; a destroyed handle returns
// them here and the next factorisation (typically the same problem sizes
// again: refactoring with new hyperparameters, repeated solves in a loop)
// reuses them instead of going back to hipMalloc / hipFree for every block.
// A release records an event on the stream that last used the block and does
// not wait; a later request makes its own stream wait for that event, so a
// block is never handed out while earlier work still reads it and the host is
// never blocked.  A block is reused for a request of at least 4/5 of its
// size; when hipMalloc fails the device's cache is freed and the allocation
// retried; at most kPoolCapFrac of the device memory stays cached.
class DevicePool {
 public:
  void* get(size_t bytes, hipStream_t s) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    bytes = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
    {
      std::lock_guard<std::mutex> g(mu_);
      size_t best = SIZE_MAX;
      size_t bi = 0;
      for (size_t i = 0; i < free_.size(); ++i) {
        const Blk& b = free_[i];
        if (b.dev == dev && b.bytes >= bytes && b.bytes - bytes <= b.bytes / 5 && b.bytes < best) {
          best = b.bytes;
          bi = i;
        }
      }
      if (best != SIZE_MAX) {
        Blk b = free_[bi];
        if (hipStreamWaitEvent(s, b.ev, 0) != hipSuccess) {
          (void)hipGetLastError();
          // the event cannot be waited on (e.g. its stream was destroyed by
          // its owner since): wait for the device instead
          if (hipEventSynchronize(b.ev) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipDeviceSynchronize();
            (void)hipGetLastError();
          }
        }
        evfree_[dev].push_back(b.ev);
        b.ev = nullptr;
        free_[bi] = free_.back();
        free_.pop_back();
        cached_[dev] -= b.bytes;
        live_[b.p] = b;
        return b.p;
      }
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      trim(dev);
      if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        throw NoMem{};
      }
    }
    std::lock_guard<std::mutex> g(mu_);
    live_[p] = Blk{p, bytes, dev, nullptr};
    return p;
  }
  // s: the stream on which the block's last reader or writer was enqueued.
  void put(void* p, hipStream_t s) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) return;
    Blk b = it->second;
    live_.erase(it);
    if (cap_[b.dev] == 0) {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) (void)hipGetLastError();
      cap_[b.dev] = (size_t)(kPoolCapFrac * (double)tot) + 1;
    }
    if (cached_[b.dev] + b.bytes > cap_[b.dev]) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(b.p);
      return;
    }
    std::vector<hipEvent_t>& ev = evfree_[b.dev];
    if (ev.empty()) {
      hipEvent_t e = nullptr;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        (void)hipFree(b.p);
        return;
      }
      ev.push_back(e);
    }
    b.ev = ev.back();
    ev.pop_back();
    if (hipEventRecord(b.ev, s) != hipSuccess) {
      (void)hipGetLastError();
      ev.push_back(b.ev);
      (void)hipStreamSynchronize(s);
      (void)hipFree(b.p);
      return;
    }
    free_.push_back(b);
    cached_[b.dev] += b.bytes;
  }
  // Frees the cached blocks of device dev (all devices when dev < 0).
  void trim(int dev) {
    (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> g(mu_);
    std::vector<Blk> keep;
    for (const Blk& b : free_) {
      if (dev < 0 || b.dev == dev) {
        (void)hipFree(b.p);
        evfree_[b.dev].push_back(b.ev);
        cached_[b.dev] -= b.bytes;
      } else {
        keep.push_back(b);
      }
    }
    free_.swap(keep);
  }

 private:
  static constexpr double kPoolCapFrac = 0.6;
  struct Blk {
    void* p;
    size_t bytes;
    int dev;
    hipEvent_t ev;  // recorded at release (cached blocks only)
  };
  std::mutex mu_;
  std::vector<Blk> free_;
  std::unordered_map<void*, Blk> live_;
  std::unordered_map<int, size_t> cached_, cap_;
  std::unordered_map<int, std::vector<hipEvent_t>> evfree_;
};

// Never destroyed: handles may be released after static destructors ran.
DevicePool& pool() {
  static DevicePool* p = new DevicePool();
  return *p;
}

// Pinned host buffers of the descriptor uploads, kept for the next handle.
// A buffer is returned only once the copies out of it have completed.
class PinnedPool {
 public:
  char* get(size_t bytes, size_t* got) {
    {
      std::lock_guard<std::mutex> g(mu_);
      size_t best = free_.size();
      for (size_t i = 0; i < free_.size(); ++i)  // the smallest that fits
        if (free_[i].second >= bytes && (best == free_.size() || free_[i].second < free_[best].second)) best = i;
      if (best < free_.size()) {
        auto b = free_[best];
        free_[best] = free_.back();
        free_.pop_back();
        *got = b.second;
        return b.first;
      }
    }
    char* p = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&p), bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw NoMem{};
    }
    *got = bytes;
    return p;
  }
  void put(char* p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    if (free_.size() >= 96) {
      (void)hipHostFree(p);
      return;
    }
    free_.push_back({p, bytes});
  }

 private:
  std::mutex mu_;
  std::vector<std::pair<char*, size_t>> free_;
};
PinnedPool& pinned() {
  static PinnedPool* p = new PinnedPool();
  return *p;
}

template <class T>
T* dalloc(hipStream_t s, size_t n) {
  return static_cast<T*>(pool().get(std::max<size_t>(n, 1) * sizeof(T), s));
}
template <class T>
void dfree(hipStream_t s, T*& p) {
  if (p) pool().put(p, s);
  p = nullptr;
}

inline int rup(int a, int b) { return (a + b - 1) / b * b; }
// Host-side phase clock of the factorisation (IFMM_TRACE_HOST=1 in the
// environment): exclusive wall time per planning phase, a nested phase
// pausing the one that encloses it, printed to stderr when the factorisation
// ends.  Off, it costs one branch per scope.
constexpr int kHcLevels = 13;  // tree levels 0..12
enum HostPhase { HP_TREE, HP_ASSEMBLY, HP_RECORDS, HP_INVPLAN, HP_COMPRESS_PRE, HP_WEIGHTS, HP_RUN, HP_WAIT,
                 HP_COMPRESS_POST, HP_DEFERRED, HP_TRANSITION, HP_TOP, HP_SOLVE_PLAN, HP_COUNT };
struct HostClock {
  using Clock = std::chrono::steady_clock;
  bool on = false;
  int cur = -1;
  Clock::time_point last;
  int level = 0;  // tree level being factored (0: outside the levels)
  double sec[HP_COUNT][kHcLevels] = {};
  long calls[HP_COUNT] = {};
  double upload_bytes[kHcLevels] = {};
  void charge(Clock::time_point t) {
    if (cur >= 0) sec[cur][level] += std::chrono::duration<double>(t - last).count();
    last = t;
  }
  int enter(int id) {
    const int prev = cur;
    if (!on) return prev;
    charge(Clock::now());
    cur = id;
    ++calls[id];
    return prev;
  }
  void leave(int prev) {
    if (!on) return;
    charge(Clock::now());
    cur = prev;
  }
  void print(int64_t n) const {
    if (!on) return;
    static const char* names[HP_COUNT] = {"tree",        "assembly",     "records",    "inverse-plan", "compress-pre",
                                          "weights",     "upload+launch", "rank-wait", "compress-post", "work-counts",
                                          "transition",  "top",          "solve-plan"};
    double tot = 0;
    for (const auto& row : sec)
      for (double v : row) tot += v;
    std::fprintf(stderr, "ifmm host phases (N = %lld): %.2f ms; per level (0: outside the levels)\n", (long long)n,
                 1e3 * tot);
    for (int i = 0; i < HP_COUNT; ++i) {
      if (!calls[i]) continue;
      double t = 0;
      for (double v : sec[i]) t += v;
      std::fprintf(stderr, "  %-14s %9.3f ms %6ld |", names[i], 1e3 * t, calls[i]);
      for (int k = 0; k < kHcLevels; ++k)
        if (sec[i][k] > 0) std::fprintf(stderr, " %d:%.2f", k, 1e3 * sec[i][k]);
      std::fprintf(stderr, "\n");
    }
    std::fprintf(stderr, "  descriptor MB  |");
    for (int k = 0; k < kHcLevels; ++k)
      if (upload_bytes[k] > 0) std::fprintf(stderr, " %d:%.2f", k, upload_bytes[k] / 1e6);
    std::fprintf(stderr, "\n");
  }
};
struct PhaseScope {
  HostClock& c;
  int prev;
  PhaseScope(HostClock& hc, int id) : c(hc), prev(hc.enter(id)) {}
  ~PhaseScope() { c.leave(prev); }
};

// Panel width of the blocked pivot inverse: 64 columns (half the panel,
// row-swap and update launches of 32) while the panel fits the registers
// of the panel kernel (m <= 512), else 32.
constexpr int kInvNb = 64;
inline int inv_panel_width(int max_m) { return max_m <= 512 ? 64 : 32; }
// Largest stored near field of the FMM product (bytes); beyond it the
// product evaluates the near-field kernel on the fly.
constexpr size_t kNearStoreMax = (size_t)16 << 30;
constexpr int kMaxLevels = 12;  // deepest tree (4^12 leaves)

// Relative threshold floor of the fill compression in an FP32 factor: pivot
// norms below a few FP32 rounding units of the first are rounding noise
// there, so a smaller eps would only keep noise directions up to the cap.
constexpr double kF32EpsFloor = 2.5e-7;

// ------------------------------------------------------------ descriptor stages
enum OpType { OP_GEMM, OP_ADD, OP_XFORM, OP_QR, OP_RRQR, OP_FORMQ, OP_STACKQR, OP_GJPANEL, OP_GJREST, OP_GJUNPERM,
              OP_TXFORM, OP_WSTACK, OP_ELIM, OP_TRANS, OP_GJREG, OP_SOLVE, OP_M2LASM, OP_FORMQRR, OP_FILLCP, OP_ROWCP,
              OP_RANKFIN };
// Profile families (slots of ifmm_stats_t): 0 gemm, 1 add, 2 (unused), 3 qr,
// 4 rrqr, 5 formq, 6 stackqr, 7 pivot inverse, 8 Schur updates (elimination
// step 2), 9 touched-cluster transform, 10 window stacked R, 11 solve sweeps,
// 12 the other elimination steps.
constexpr int kOpTypes = 16;
inline int family(int t) {
  switch (t) {
    case OP_GJPANEL:
    case OP_GJREST:
    case OP_GJUNPERM:
    case OP_GJREG: return 7;
    case OP_ELIM: return 8;
    case OP_TXFORM: return 9;
    case OP_WSTACK: return 10;
    case OP_TRANS: return 1;
    case OP_SOLVE: return 11;
    case OP_M2LASM: return 0;
    case OP_FORMQRR: return 5;
    case OP_FILLCP: return 1;
    case OP_ROWCP: return 1;
    case OP_RANKFIN: return 1;
    default: return t;
  }
}
struct Op {
  OpType t;
  size_t off, off2;
  int count, a, b;
  double flops, bytes;  // algorithmic work of the launch
  size_t off2b = 0;
  int ty = 0;  // scalar type code of the descriptors
  size_t off3 = 0;  // register pivoted QR: blob offset + 1 of the FillCopy whose fills it reads in place
};

// Profile family of a launch (the elimination steps other than the Schur
// updates have a slot of their own).
inline int op_family(const Op& o) { return o.t == OP_ELIM && o.count != 2 ? 12 : family(o.t); }

inline double esz(int f32) { return f32 ? 4.0 : 8.0; }

// Splits v into runs of equal type code (first-seen order) and calls
// f(run, ty) for each: one launch per type combination.
template <class D, class F>
void by_type(const std::vector<D>& v, F f) {
  if (v.empty()) return;
  bool mixed = false;
  for (const D& d : v) mixed |= d.ty != v[0].ty;
  if (!mixed) {
    f(v, v[0].ty);
    return;
  }
  std::vector<int> seen;
  for (const D& d : v)
    if (std::find(seen.begin(), seen.end(), d.ty) == seen.end()) seen.push_back(d.ty);
  for (int t : seen) {
    std::vector<D> g;
    for (const D& d : v)
      if (d.ty == t) g.push_back(d);
    f(g, t);
  }
}

// Exact algorithmic work (flops, bytes at element size es) of a touched-
// cluster basis change: per touched cluster, the parent transfer block and
// every block of its M2L window (rows changed by T, columns by S = T^T when
// the window partner is touched too, or the partner's row block when
// col_blocks is set and it is not).
inline std::pair<double, double> txform_work(const TouchXform& a, const std::vector<int>* touch_q,
                                             const std::vector<int>* tidx, const std::vector<int>& r_old,
                                             const std::vector<int>& r_new, const std::vector<int>* r_par,
                                             int ncl, double es) {
  double f = 0, by = 0;
  auto blk = [&](int ro, int co, int rn, int cn, bool hasT, bool hasS) {
    const int rz = hasT ? rn : ro;
    f += 2.0 * (hasT ? (double)rn * ro * co : 0) + 2.0 * (hasS ? (double)rz * co * cn : 0);
    by += es * ((double)ro * co + (hasT ? (double)rn * ro : 0) + (hasS ? (double)co * cn : 0) +
                (double)rz * (hasS ? cn : co));
  };
  for (int t = 0; t < a.nt; ++t) {
    const int q = touch_q ? (*touch_q)[t] : t;
    const int rq = r_old[q], rn = r_new[t];
    if (rq == 0) continue;
    if (a.UP && r_par && (*r_par)[q >> 2] > 0) blk(rq, (*r_par)[q >> 2], rn, 0, true, false);
    const int qx = demorton_x(q), qy = demorton_y(q);
    for (int sl = 0; sl < 36; ++sl) {
      const int jx = 2 * (qx >> 1) - 2 + sl / 6, jy = 2 * (qy >> 1) - 2 + sl % 6;
      if (jx < 0 || jy < 0 || jx >= a.nside || jy >= a.nside) continue;
      if (std::abs(jx - qx) <= 1 && std::abs(jy - qy) <= 1) continue;
      const int l = morton2(jx, jy);
      if (l >= ncl || r_old[l] == 0) continue;
      const int tl = tidx ? (*tidx)[l] : l;
      blk(rq, r_old[l], rn, tl >= 0 ? r_new[tl] : r_old[l], true, tl >= 0);
      if (tl < 0 && a.col_blocks) blk(r_old[l], rq, r_old[l], rn, false, true);
    }
  }
  return {f, by};
}

// Exact work of the far-field weight stacks: per cluster, the R factor of its
// stacked window column (plus the parent chain rows when a.Z is set), by
// Householder steps or (gram) by the packed Gram matrix and its Cholesky
// factor.
inline std::pair<double, double> winstack_work(const WinStack& a, const std::vector<int>& ids,
                                               const std::vector<int>& r, const std::vector<int>* r_par,
                                               double es, bool gram = false) {
  double f = 0, by = 0;
  for (int t = 0; t < a.nt; ++t) {
    const int q = ids[t], rq = r[q];
    if (rq == 0) continue;
    double rows = (a.Z && r_par) ? (*r_par)[q >> 2] : 0;
    const int qx = demorton_x(q), qy = demorton_y(q);
    for (int sl = 0; sl < 36; ++sl) {
      const int jx = 2 * (qx >> 1) - 2 + sl / 6, jy = 2 * (qy >> 1) - 2 + sl % 6;
      if (jx < 0 || jy < 0 || jx >= a.nside || jy >= a.nside) continue;
      if (std::abs(jx - qx) <= 1 && std::abs(jy - qy) <= 1) continue;
      rows += r[morton2(jx, jy)];
    }
    f += gram ? rows * rq * (rq + 1.0) + rq * (double)rq * rq / 3.0 : 2.0 * rows * rq * rq;
    by += es * (rows * rq + (double)a.S * rq * rq);
  }
  return {f, by};
}

// sum_{j < K} (n - j) (m - j), exactly (integer-valued doubles).
inline double tri_sum(double n, double m, double K) {
  return K * n * m - (n + m) * K * (K - 1) / 2 + (K - 1) * K * (2 * K - 1) / 6;
}

// Descriptor bytes of a stage, written straight into pinned host memory from
// the pool (no staging copy before the upload; growth keeps the contents,
// new bytes are not initialised).  Upload hands the buffer to the arena
// slot that copies it, taking the slot's previous (idle) buffer in exchange.
struct Blob {
  char* p = nullptr;
  size_t n = 0, cap = 0;
  Blob() = default;
  Blob(const Blob&) = delete;
  Blob& operator=(const Blob&) = delete;
  Blob(Blob&& o) noexcept : p(o.p), n(o.n), cap(o.cap) { o.p = nullptr, o.n = o.cap = 0; }
  Blob& operator=(Blob&& o) noexcept {
    std::swap(p, o.p);
    std::swap(n, o.n);
    std::swap(cap, o.cap);
    return *this;
  }
  ~Blob() {
    if (p) pinned().put(p, cap);
  }
  size_t size() const { return n; }
  char* data() { return p; }
  const char* data() const { return p; }
  void clear() { n = 0; }
  void resize(size_t m) {
    if (m > cap) {
      size_t got = 0;
      char* q = pinned().get(std::max(m, std::max(2 * cap, (size_t)64 << 10)), &got);
      if (n) std::memcpy(q, p, n);
      if (p) pinned().put(p, cap);
      p = q;
      cap = got;
    }
    n = m;
  }
};

struct Stage {
  Blob blob;
  std::vector<Op> ops;
  double flops = 0.0;
  size_t push(const void* p, size_t n) {
    size_t off = (blob.size() + 63) & ~size_t(63);
    blob.resize(off + n);
    if (n) std::memcpy(blob.data() + off, p, n);
    return off;
  }
  void op(Op o, int ty) {
    o.ty = ty;
    ops.push_back(o);
  }
  // Algorithmic counts: flops of the operation as defined, bytes = every
  // operand read once and every output written once, at its storage size.
  void gemm(const std::vector<GemmDesc>& all) {
    by_type(all, [&](const std::vector<GemmDesc>& v, int ty) {
      int mm = 0, nn = 0, plain = 1;
      double f = 0, by = 0;
      const double sa = esz(ty & 1), sb = esz(ty & 2), sc = esz(ty & 4);
      for (const auto& d : v) {
        mm = std::max(mm, d.M);
        nn = std::max(nn, d.N);
        plain &= d.opA == 0 && d.opB == 0;
        f += 2.0 * d.M * d.N * d.K;
        by += sa * d.M * d.K + sb * (double)d.K * d.N + sc * (d.beta != 0.0 ? 2.0 : 1.0) * d.M * d.N;
      }
      flops += f;
      Op o{OP_GEMM, push(v.data(), v.size() * sizeof(GemmDesc)), 0, (int)v.size(), mm, nn, f, by};
      o.off2 = (size_t)plain;
      op(o, ty);
    });
  }
  void add(const std::vector<AddDesc>& all) {
    by_type(all, [&](const std::vector<AddDesc>& v, int ty) {
      int mm = 0, nn = 0;
      double by = 0;
      for (const auto& d : v) {
        mm = std::max(mm, d.M);
        nn = std::max(nn, d.N);
        by += (double)d.M * d.N * ((d.A ? esz(ty & 1) : 0.0) + esz(ty & 2) * (d.beta != 0.0 ? 2.0 : 1.0));
      }
      op({OP_ADD, push(v.data(), v.size() * sizeof(AddDesc)), 0, (int)v.size(), mm, nn, 0.0, by}, ty);
    });
  }
  // Unpivoted QRs, staged in LDS (off2 = bytes) when the matrix fits
  // kQrLdsBytes, else in place.
  // Matrices of at most 64 columns whose rows fit one lane's registers go to
  // the one-wave kernel (op.b = row class), by row class; the rest to the
  // workgroup kernel, staged in LDS where they fit (op.off2 = LDS bytes).
  void qr(const std::vector<QrDesc>& all) {
    by_type(all, [&](const std::vector<QrDesc>& byt, int ty) {
      std::vector<QrDesc> grp[2], wave[5];
      for (const auto& d : byt) {
        const int nr = qr_wave_rows(d.n, d.m, ty);
        if (nr > 0) wave[nr / 32].push_back(d);
        else grp[qr_lds_bytes(d.n, d.m, ty) <= kQrLdsBytes ? 1 : 0].push_back(d);
      }
      auto work = [&](const std::vector<QrDesc>& v, double& f, double& by, size_t& lds, int& kmax) {
        for (const auto& d : v) {
          const double K = std::min(d.n, d.m);
          f += 4.0 * d.n * d.m * K - 2.0 * K * K * (d.n + d.m) + 4.0 / 3.0 * K * K * K  // factor
               + 4.0 * d.n * K * K - 2.0 * K * K * K;                                   // form Q
          by += esz(ty) * (2.0 * d.n * d.m + K * d.m);
          lds = std::max(lds, qr_lds_bytes(d.n, d.m, ty));
          kmax = std::max(kmax, std::min(d.n, d.m));
        }
        flops += f;
      };
      for (int c = 1; c <= 4; ++c) {
        const auto& v = wave[c];
        if (v.empty()) continue;
        double f = 0, by = 0;
        size_t lds = 0;
        int kmax = 0;
        work(v, f, by, lds, kmax);
        op({OP_QR, push(v.data(), v.size() * sizeof(QrDesc)), 0, (int)v.size(), kmax, 32 * c, f, by}, ty);
      }
      for (int g = 0; g < 2; ++g) {
        const auto& v = grp[g];
        if (v.empty()) continue;
        double f = 0, by = 0;
        size_t lds = 0;
        int kmax = 0;
        work(v, f, by, lds, kmax);
        op({OP_QR, push(v.data(), v.size() * sizeof(QrDesc)), g ? lds : 0, (int)v.size(), 0, 0, f, by}, ty);
      }
    });
  }
  // Ranks finished on the device (RankFin; pointer fields other than rank
  // are arr()-style blob pointers).
  void rank_finalize(RankFin a) {
    if (a.nt <= 0) return;
    op({OP_RANKFIN, push(&a, sizeof(a)), 0, a.nt, 0, 0, 0.0, 0.0}, 0);
  }
  // Pivoted QRs: matrices whose columns fit the registers of one thread each
  // go to the register kernel (b = 2, which also forms Q), by row class;
  // the rest to the LDS kernel (b = 1) or in place (b = 0), followed by the
  // Q formation where Q is asked for.  Q's work is counted once the ranks
  // are known (rrqr_q_work).
  static bool rrqr_in_regs(const RrqrDesc& d) {
    const int nr = rrqr_reg_rows(d.n, d.ty);
    return nr > 0 && d.m <= kRrqrRegCols && rrqr_reg_lds(nr, d.kmax, d.ty) <= 144 * 1024;
  }
  void rrqr(const std::vector<RrqrDesc>& all, size_t fill_off = 0) {
    by_type(all, [&](const std::vector<RrqrDesc>& byt, int ty) {
      const size_t es = ty ? sizeof(float) : sizeof(double);
      std::vector<RrqrDesc> reg[5], grp[2];
      for (const auto& d : byt) {
        if (rrqr_in_regs(d)) {
          reg[rrqr_reg_rows(d.n, ty) / 32].push_back(d);
        } else {
          const size_t need = es * ((size_t)(d.n + 1) * d.m + d.m);
          grp[need <= kRrqrLdsBytes ? 1 : 0].push_back(d);
        }
      }
      auto work = [&](const std::vector<RrqrDesc>& v, double& f, double& by, int& mm) {
        for (const auto& d : v) {
          mm = std::max(mm, d.m);
          const int K = std::min(std::min(d.n, d.m), d.kmax);
          f += 4.0 * tri_sum(d.n, d.m, K);
          by += 2.0 * es * d.n * (double)d.m;
        }
        flops += f;
      };
      for (int c = 1; c <= 4; ++c) {
        const auto& v = reg[c];
        if (v.empty()) continue;
        double f = 0, by = 0;
        int mm = 0, km = 0;
        work(v, f, by, mm);
        for (const auto& d : v) km = std::max(km, d.kmax);
        Op o{OP_RRQR, push(v.data(), v.size() * sizeof(RrqrDesc)), (size_t)(32 * c), (int)v.size(), mm, 2, f, by};
        o.off2b = (size_t)km;
        o.off3 = fill_off;
        op(o, ty);
      }
      for (int g = 0; g < 2; ++g) {
        const auto& v = grp[g];
        if (v.empty()) continue;
        size_t lds = 0;
        double f = 0, by = 0;
        int mm = 0;
        work(v, f, by, mm);
        for (const auto& d : v) lds = std::max(lds, es * ((size_t)(d.n + 1) * d.m + d.m));
        const size_t o = push(v.data(), v.size() * sizeof(RrqrDesc));
        bool q = false;
        int nn = 0, km = 0;
        for (const auto& d : v) {
          q |= d.Q != nullptr;
          nn = std::max(nn, d.n);
          km = std::max(km, d.kmax);
        }
        Op r{OP_RRQR, o, g == 1 ? (size_t)lds : 0, (int)v.size(), mm, g, f, by};
        r.off2b = (size_t)nn;
        op(r, ty);
        if (q) op({OP_FORMQRR, o, 0, (int)v.size(), nn, km, 0.0, 0.0}, ty);
      }
    });
  }

  // Touched-cluster basis change (geometry on the device).  The int arrays
  // travel in the blob; the pointer fields of the stored TouchXform hold
  // their blob offsets + 1 (0 = null) and are rebased at launch.  flops and
  // bytes are the exact algorithmic counts, from the host's rank tables.
  const int* arr(const std::vector<int>* v) {
    if (!v) return nullptr;
    return reinterpret_cast<const int*>(push(v->data(), std::max<size_t>(1, v->size()) * sizeof(int)) + 1);
  }
  // count = false: the exact work counts are left to the caller (see
  // txform_work), the launch carries zeros.  r_new_at: an int array already
  // in the blob (its arr() pointer) used as r_new instead of pushing r_new
  // (its values are then written on the device; no work is counted here).
  template <class T>
  void touch_xform(TouchXform a, const std::vector<int>* touch_q, const std::vector<int>* tidx,
                   const std::vector<int>& r_old, const std::vector<int>& r_new, const std::vector<int>* r_par,
                   int ncl, bool count = true, const int* r_new_at = nullptr) {
    if (a.nt <= 0) return;
    double f = 0, by = 0;
    if (count && !r_new_at) std::tie(f, by) = txform_work(a, touch_q, tidx, r_old, r_new, r_par, ncl, sizeof(T));
    a.touch_q = arr(touch_q);
    a.tidx = arr(tidx);
    a.r_old = arr(&r_old);
    a.r_new = r_new_at ? r_new_at : arr(&r_new);
    a.r_par = arr(r_par);
    flops += f;
    op({OP_TXFORM, push(&a, sizeof(a)), 0, a.nt, 0, 0, f, by}, tcode<T>());
  }
  // Row blocks between a vector of blocks (item i at blk + i bstride, ld ldb)
  // and a long vector (item i at v + start[i], ld ldv), cnt[i] rows x nrhs
  // each: to_blocks = gather into the blocks, else scatter out of them.  The
  // start / cnt arrays travel in the blob (rebased at launch).
  struct RowCopy {
    double* v;
    double* blk;
    const int* start;
    const int* cnt;
    size_t bstride;
    int ldv, ldb, n, nrhs, to_blocks;
  };
  void row_copy(RowCopy a, const std::vector<int>& start, const std::vector<int>& cnt) {
    if (a.n <= 0) return;
    double by = 0;
    for (int c : cnt) by += 16.0 * c * a.nrhs;
    a.start = arr(&start);
    a.cnt = arr(&cnt);
    op({OP_ROWCP, push(&a, sizeof(a)), 0, a.n, 0, 0, 0.0, by}, 0);
  }
  // Fill copies into the pivoted-QR inputs (records and touches travel in
  // the blob; their pointer fields hold blob offsets + 1, rebased at launch).
  // Returns the FillCopy's blob offset + 1 (0: none), for the register
  // pivoted QRs that read the fills of their touches in place.
  template <class T>
  size_t fill_copy(FillCopy a, const std::vector<ElimRec>& rec, const std::vector<int>& touch, double bytes) {
    if (a.nt <= 0) return 0;
    a.rec = reinterpret_cast<const ElimRec*>(push(rec.data(), std::max<size_t>(1, rec.size()) * sizeof(ElimRec)) + 1);
    a.touch = arr(&touch);
    const size_t off = push(&a, sizeof(a));
    op({OP_FILLCP, off, 0, a.nt, 0, 0, 0.0, bytes}, tcode<T>());
    return off + 1;
  }
  // Far-field weight stacks with device-side block lists (arrays as in
  // touch_xform).
  template <class T>
  void win_stack(WinStack a, const std::vector<int>& ids, const std::vector<int>& r, const std::vector<int>* r_par,
                 bool count = true, bool gram = false) {
    if (a.nt <= 0) return;
    double f = 0, by = 0;
    if (count) std::tie(f, by) = winstack_work(a, ids, r, r_par, sizeof(T), gram);
    int rmax = 0;
    for (int t = 0; t < a.nt; ++t) rmax = std::max(rmax, r[ids[t]]);
    a.ids = arr(&ids);
    a.r = arr(&r);
    a.r_par = arr(r_par);
    flops += f;
    op({OP_WSTACK, push(&a, sizeof(a)), 0, a.nt, rmax, gram ? 1 : 0, f, by}, tcode<T>());
  }
  // One step of the elimination kernels over a batch of records (the record
  // array is pushed once per batch: rec_off = its blob offset + 1).
  template <class T>
  void elim(ElimArgs a, size_t rec_off, int step, int max_m, int max_n, double f, double by) {
    if (a.nb <= 0) return;
    a.rec = reinterpret_cast<const ElimRec*>(rec_off);
    flops += f;
    op({OP_ELIM, push(&a, sizeof(a)), 0, step, max_m, max_n, f, by}, tcode<T>());
  }
  // Level transition assembly (device-side geometry).
  template <class T>
  void transition(TransArgs a, const std::vector<int>& choff, const std::vector<int>& cr,
                  const std::vector<int>& r_par, double by) {
    a.choff = arr(&choff);
    a.cr = arr(&cr);
    a.r_par = arr(&r_par);
    op({OP_TRANS, push(&a, sizeof(a)), 0, a.nc, 0, 0, 0.0, by}, tcode<T>());
  }
  // One colour batch of the solve (dir 0 forward, 1 backward); bytes: the
  // blocks read once plus the vectors.
  template <class T>
  void solve(const SolveArgs& a, int step, double* wk, int max_rows, double f, double by) {
    if (a.nb <= 0) return;
    op({OP_SOLVE, push(&a, sizeof(a)), (size_t)(uintptr_t)wk, step, max_rows, 0, f, by}, tcode<T>());
  }
  // M2L assembly of one level (device-side interaction lists).
  template <class T>
  void m2l_assemble(M2LAssemble a, const std::vector<int>& r, double f, double by) {
    a.r = arr(&r);
    op({OP_M2LASM, push(&a, sizeof(a)), 0, a.nc, 0, 0, f, by}, tcode<T>());
  }
  // All blocks of a stack have the type of its R.
  void stackqr(const std::vector<StackQrDesc>& v, const std::vector<BlkRef>& b) {
    if (v.empty()) return;
    const int ty = v[0].ty;
    for (const auto& d : v)
      if (d.ty != ty) throw BadArg{};
    int rr = 0;
    double f = 0, by = 0;
    for (const auto& d : v) {
      rr = std::max(rr, d.r);
      for (int t = 0; t < d.nblk; ++t) {
        f += 2.0 * b[d.first + t].rows * (double)d.r * d.r;
        by += esz(ty) * b[d.first + t].rows * (double)d.r;
      }
      by += esz(ty) * d.r * d.r;
    }
    flops += f;
    size_t o1 = push(v.data(), v.size() * sizeof(StackQrDesc));
    size_t o2 = push(b.data(), std::max<size_t>(1, b.size()) * sizeof(BlkRef));
    op({OP_STACKQR, o1, o2, (int)v.size(), rr, 0, f, by}, ty);
  }
  // Whole-matrix LDS Gauss-Jordan (FP64).
  void inv_reg(const std::vector<InvDesc>& v) {
    if (v.empty()) return;
    int mm = 0;
    double f = 0, by = 0;
    for (const auto& d : v) {
      mm = std::max(mm, d.m);
      f += 2.0 * d.m * (double)d.m * d.m;
      by += 16.0 * d.m * (double)d.m;
    }
    flops += f;
    op({OP_GJREG, push(v.data(), v.size() * sizeof(InvDesc)), 0, (int)v.size(), mm, 0, f, by}, 0);
  }
  // Blocked Gauss-Jordan inverse (FP64) of every matrix in v (panels of nb
  // columns); piv (nd x maxm ints) and tmp (nd x nb x maxm doubles) are
  // device workspace.
  void inv_blocked(const std::vector<InvDesc>& v, int* piv, double* tmp, int nb) {
    if (v.empty()) return;
    int mm = 0;
    for (const auto& d : v) mm = std::max(mm, d.m);
    const size_t o = push(v.data(), v.size() * sizeof(InvDesc));
    const int nd = (int)v.size();
    const size_t ldt = (size_t)nb * mm;
    for (int j0 = 0; j0 < mm; j0 += nb) {
      double fp = 0, bp = 0;
      for (const auto& d : v)
        if (d.m > j0) {
          const int nbe = std::min(nb, d.m - j0);
          fp += 3.0 * d.m * nbe * nbe;
          bp += 16.0 * d.m * nbe;
        }
      flops += fp;
      op({OP_GJPANEL, o, (size_t)(uintptr_t)piv, nd, mm, j0, fp, bp}, 0);
      ops.back().off3 = (size_t)nb;
      op({OP_GJREST, o, (size_t)(uintptr_t)tmp, nd, mm, j0, 0.0, 0.0}, 0);
      ops.back().off2b = (size_t)(uintptr_t)piv;
      ops.back().off3 = (size_t)nb;
      std::vector<GemmDesc> g;
      for (int b = 0; b < nd; ++b) {
        const InvDesc& d = v[b];
        if (d.m <= j0) continue;
        const int nbe = std::min(nb, d.m - j0);
        double* A = d.A;
        const size_t lda = d.lda;
        double* tb = tmp + (size_t)b * ldt;
        const int cr[2][2] = {{0, j0}, {j0 + nbe, d.m}};
        for (const auto& c : cr) {
          if (c[1] <= c[0]) continue;
          g.push_back({A + j0 + j0 * lda, tb + (size_t)c[0] * nb, A + j0 + (size_t)c[0] * lda, nbe, c[1] - c[0],
                       nbe, (int)lda, nb, (int)lda, 0, 0, 1.0, 0.0});
          for (const auto& r : cr) {
            if (r[1] <= r[0]) continue;
            g.push_back({A + r[0] + j0 * lda, tb + (size_t)c[0] * nb, A + r[0] + (size_t)c[0] * lda, r[1] - r[0],
                         c[1] - c[0], nbe, (int)lda, nb, (int)lda, 0, 0, 1.0, 1.0});
          }
        }
      }
      gemm(g);
    }
    op({OP_GJUNPERM, o, (size_t)(uintptr_t)piv, nd, mm, 0, 0.0, 0.0}, 0);
  }
  bool empty() const { return ops.empty(); }
  void clear() {
    blob.clear();
    ops.clear();
    flops = 0.0;
  }
};

// Pinned host + device buffers for descriptor upload, a ring of kSlots: an
// upload waits only for the copy out of the slot it reuses (kSlots uploads
// back), so the host can plan that many stages ahead of the device.  The
// device copy of a slot is rewritten only by a later copy on the same
// stream, after the kernels that read it.
struct Arena {
  static constexpr int kSlots = 16;
  char* h[kSlots] = {};
  char* d[kSlots] = {};
  size_t hcap[kSlots] = {}, dcap[kSlots] = {};
  hipEvent_t ev[kSlots] = {};
  bool pending[kSlots] = {};  // a copy out of the slot may still be in flight
  int cur = 0;
  void init() {
    for (int i = 0; i < kSlots; ++i) HIP_OK(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
  }
  // The stream the copies went to has been synchronised: no slot is in
  // flight, and no later upload needs to query an event recorded on it (the
  // caller may destroy that stream).
  void settle() {
    for (int i = 0; i < kSlots; ++i) pending[i] = false;
  }
  void release(hipStream_t s) {
    for (int i = 0; i < kSlots; ++i) {
      if (ev[i] && pending[i]) (void)hipEventSynchronize(ev[i]);
      pinned().put(h[i], hcap[i]);
      dfree(s, d[i]);
      if (ev[i]) (void)hipEventDestroy(ev[i]);
      h[i] = d[i] = nullptr;
      hcap[i] = dcap[i] = 0;
      ev[i] = nullptr;
    }
  }
  // Copies the blob to the device; returns the device address and, in
  // *host, where the bytes now are on the host (the slot took the blob's
  // buffer; the blob is left empty, holding the slot's previous buffer).
  char* upload(Blob& blob, hipStream_t s, const char** host) {
    const size_t need = blob.size();
    *host = blob.data();
    if (need == 0) return nullptr;
    cur = (cur + 1) % kSlots;
    // the previous copy out of this slot must be done before it is reused
    if (pending[cur]) HIP_OK(hipEventSynchronize(ev[cur]));
    if (need > dcap[cur]) {
      const size_t c = std::max(std::max(need, 2 * dcap[cur]), (size_t)1 << 20);
      dfree(s, d[cur]);
      dcap[cur] = 0;
      d[cur] = dalloc<char>(s, c);
      dcap[cur] = c;
    }
    std::swap(h[cur], blob.p);
    std::swap(hcap[cur], blob.cap);
    blob.n = 0;
    void* hd = nullptr;  // the slot's host buffer, as the device addresses it
    HIP_OK(hipHostGetDevicePointer(&hd, h[cur], 0));
    launch_copy_from_host(hd, d[cur], need, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(ev[cur], s));
    pending[cur] = true;
    *host = h[cur];
    return d[cur];
  }
};

// Grow-only device workspace (typed views of one allocation).
struct Buf {
  char* p = nullptr;
  size_t bytes = 0;
  template <class U = double>
  U* need(size_t m, hipStream_t s) {
    const size_t b = std::max<size_t>(m, 1) * sizeof(U);
    if (b > bytes) {
      dfree(s, p);
      p = dalloc<char>(s, b);
      bytes = b;
    }
    return reinterpret_cast<U*>(p);
  }
  void release(hipStream_t s) {
    dfree(s, p);
    bytes = 0;
  }
};

// ------------------------------------------------------------ geometry helpers
inline int s9_dx(int s) { return s / 3 - 1; }
inline int s9_dy(int s) { return s % 3 - 1; }
inline int slot36(int a, int b) {
  return win_slot(demorton_x(a), demorton_y(a), demorton_x(b), demorton_y(b));
}
// compact index of an ordered pair of 3x3 positions at Chebyshev distance 2
struct PairTable {
  int idx[9][9];
  int count = 0;
  PairTable() {
    for (int a = 0; a < 9; ++a)
      for (int b = 0; b < 9; ++b) {
        const int d = std::max(std::abs(s9_dx(a) - s9_dx(b)), std::abs(s9_dy(a) - s9_dy(b)));
        idx[a][b] = d == 2 ? count++ : -1;
      }
  }
};
const PairTable kPairs;

// ------------------------------------------------------------ Chebyshev (host)
double cheb_t(int p, int m) { return std::cos((2.0 * m + 1.0) * M_PI / (2.0 * p)); }
double lagr(int p, int m, double s) {
  double v = 1.0;
  for (int k = 0; k < p; ++k)
    if (k != m) v *= (s - cheb_t(p, k)) / (cheb_t(p, m) - cheb_t(p, k));
  return v;
}
// E_c: rows child nodes, columns parent nodes (p^2 x p^2, column-major).
std::vector<double> transfer_host(int p) {
  const int p2 = p * p;
  std::vector<double> E(4 * p2 * p2);
  for (int c = 0; c < 4; ++c) {
    const double ox = (c & 1) ? 0.5 : -0.5, oy = (c >> 1) ? 0.5 : -0.5;
    for (int mc = 0; mc < p2; ++mc) {
      const double sx = ox + 0.5 * cheb_t(p, mc / p), sy = oy + 0.5 * cheb_t(p, mc % p);
      for (int mp = 0; mp < p2; ++mp)
        E[(size_t)c * p2 * p2 + mc + (size_t)mp * p2] = lagr(p, mp / p, sx) * lagr(p, mp % p, sy);
    }
  }
  return E;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// ------------------------------------------------------------------- levels
// Blocks of one level, in the factor's scalar type T, except the pivot
// inverses (always FP64).
template <class T>
struct Level {
  int k = 0, nside = 0, nc = 0;
  std::vector<int> n, r, colour, nbr9, choff;  // choff: [nc*4] offsets of children's multipoles
  int npad = 0, rpad = 0, mpad = 0;
  size_t sP = 0, sQ = 0, sL = 0, sM = 0, sU = 0, sUP = 0, sD = 0;
  // one basis per cluster (symmetric system): U is both L2P and P2M^T, UP the
  // parent's transfer block of this child, Om the precomputed far-field weight
  T *P = nullptr, *Qm = nullptr, *L = nullptr, *M = nullptr, *U = nullptr, *UP = nullptr, *Om = nullptr;
  double* Dinv = nullptr;
  T* Pb(int i, int s) const { return P + ((size_t)i * 9 + s) * sP; }
  T* Qb(int i, int s) const { return Qm + ((size_t)i * 9 + s) * sQ; }
  T* Lb(int i, int s) const { return L + ((size_t)i * 9 + s) * sL; }
  T* Mb(int i, int s) const { return M + ((size_t)i * 36 + s) * sM; }
  T* Ub(int i) const { return U + (size_t)i * sU; }
  T* UPb(int i) const { return UP + (size_t)i * sUP; }
  double* Db(int i) const { return Dinv + (size_t)i * sD; }
  T* Omb(int i) const { return Om + (size_t)i * sUP; }
  void set_pads(int np) {
    npad = np;
    mpad = npad + rpad;
    sP = (size_t)npad * npad;
    sQ = (size_t)npad * rpad;
    sL = (size_t)rpad * npad;
    sM = (size_t)rpad * rpad;
    sU = (size_t)npad * rpad;
    sUP = (size_t)rpad * rpad;
    sD = (size_t)mpad * mpad;
  }
  void free_work(hipStream_t s) {
    dfree(s, M);
    dfree(s, U);
    dfree(s, UP);
    dfree(s, Om);
  }
  void free_all(hipStream_t s) {
    free_work(s);
    dfree(s, P);
    dfree(s, Qm);
    dfree(s, L);
    dfree(s, Dinv);
  }
};

// A unit of the 3x3 neighbourhood of an eliminated cluster.
struct UnitH {
  int cl = -1, kind = 0, size = 0, off = 0;  // kind 1: particles, 2: multipoles
};
struct Elim {
  int i, ni, ri, m;
  std::array<UnitH, 9> u;
};

}  // namespace

// Opaque handle of the C-ABI: the problem parameters, and the interface of
// the factor engine, whose block scalar type is its template parameter.
struct ifmm_plan {
  hipStream_t s = nullptr;
  int64_t N = 0;
  int kappa = 0, p = 0, p2 = 0, leaf = 0, r_cap = 0, rpad = 0;
  KernelFn kf{};
  int diag_mode = 0;
  const double* d_diag_user = nullptr;  // IFMM_DIAG_VECTOR: the caller's A_ii (device, caller order)
  double c0 = 0.0, eps = 0.0;
  double lox = 0.0, loy = 0.0, size = 1.0;
  double refine_tol = 0.0;
  int refine_maxit = 30;
  // 0: off; 1: every launch family; otherwise bit f + 1 times family f only
  int profile = 0;
  bool timed(int fam) const { return profile == 1 || ((profile >> (fam + 1)) & 1) != 0; }
  virtual ~ifmm_plan() = default;
  virtual void build(const double* points) = 0;  // assembly + Algorithm 1
  virtual ifmm_status solve(const double* b, double* x, int nrhs, ifmm_solve_info* info) = 0;
  virtual void matvec(const double* x, double* y, int nrhs) = 0;
  virtual void matvec_kernel(const KernelFn& kk, int dmode, double c0k, const double* dvec, const double* x,
                             double* y, int nrhs) = 0;
  virtual size_t matvec_scratch_bytes(int nrhs) const = 0;
  virtual void matvec_into(const double* x, double* y, int nrhs, double* ws) = 0;
  virtual void diagonal(double* d) = 0;
  virtual void stats(ifmm_stats_t* st) = 0;
  virtual int ranks(int level, int* out, int count) = 0;
  virtual void release() = 0;
};

namespace {

// A second stream forked from s (it starts after the work queued on s so
// far) and joined back into s when the scope ends (s then waits for it).
// The stream is one per device, created on first use and kept until the
// process ends (creating one per factorisation cost ~0.3 ms of host time);
// calls that share it stay correct (their forks and joins are events), only
// their side work serialises.  enabled = false: everything stays on s.
struct SideStream {
  hipStream_t main, s;
  hipEvent_t join = nullptr;
  SideStream(hipStream_t m, bool enabled) : main(m), s(m) {
    if (!enabled) return;
    static std::mutex mu;
    static std::unordered_map<int, hipStream_t>* per_dev = new std::unordered_map<int, hipStream_t>();  // never destroyed
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    hipStream_t side = nullptr;
    {
      std::lock_guard<std::mutex> lk(mu);
      hipStream_t& st = (*per_dev)[dev];
      if (!st) HIP_OK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      side = st;
    }
    hipEvent_t fork = nullptr;
    HIP_OK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    const hipError_t e1 = hipEventRecord(fork, main);
    const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(side, fork, 0) : e1;
    (void)hipEventDestroy(fork);
    HIP_OK(e2);
    HIP_OK(hipEventCreateWithFlags(&join, hipEventDisableTiming));
    s = side;
  }
  ~SideStream() {
    if (!join) return;
    (void)hipEventRecord(join, s);
    (void)hipStreamWaitEvent(main, join, 0);
    (void)hipEventDestroy(join);
  }
  SideStream(const SideStream&) = delete;
  SideStream& operator=(const SideStream&) = delete;
};

template <class T>
struct Plan final : ifmm_plan {
  static constexpr bool kF32 = std::is_same<T, float>::value;
  std::vector<int> leaf_start, leaf_n;
  double* d_pts = nullptr;
  int *d_perm = nullptr, *d_leaf_start = nullptr, *d_leaf_n = nullptr, *d_nbr9_leaf = nullptr;
  double* d_diag = nullptr;
  double* d_near = nullptr;      // FP64 near field of the product (null: evaluated on the fly)
  size_t* d_near_off = nullptr;  // per leaf: offset of its block in d_near
  std::vector<size_t> near_off_h;
  double* d_E = nullptr;
  std::vector<double*> d_table;
  std::vector<Level<T>> lv;
  std::vector<std::vector<std::vector<Elim>>> plan;  // [k][colour] eliminations in order
  std::vector<unsigned> batch_mark;  // per cluster: stamp of the last colour batch whose neighbourhood holds it
  unsigned batch_stamp = 0;
  std::vector<std::vector<std::vector<ElimRec>>> erec;  // their records, kept for the solve
  ElimRec* d_erec = nullptr;                          // all records on the device
  std::vector<std::vector<size_t>> erec_off;          // [k][colour] offset into d_erec
  // top
  std::vector<int> top_ids, top_off;
  int top_m = 0;
  double* d_top = nullptr;
  Status* d_status = nullptr;
  Arena arena;
  HostClock hc;
  Blob up_E, up_nbr9, up_near_off;  // pinned sources of assembly uploads, kept until build() has synchronised
  Buf wsX, wsF, wsT, wsA, wsB, wsQ, wsR, wsZ, wsS1, wsS2, wsVec, wsSeg, wsTab;
  int* d_rank = nullptr;
  size_t rank_cap = 0;
  // the ranks' pinned copy on the host, and the event after its copy
  int* h_rank = nullptr;
  int* h_rank_dev = nullptr;  // h_rank's device address
  size_t h_rank_bytes = 0;
  char* h_small = nullptr;  // pinned scratch of the small read-backs (leaf counts, norms, status)
  size_t h_small_bytes = 0;
  // A pinned pool buffer as the device addresses it.
  static void* dev_view(const void* h) {
    void* d = nullptr;
    HIP_OK(hipHostGetDevicePointer(&d, const_cast<void*>(h), 0));
    return d;
  }
  // The first `bytes` of a pinned blob into device memory, queued on the
  // stream (the blob must outlive the copy).
  void upload_pinned(void* d, const Blob& b, size_t bytes) {
    launch_copy_from_host(dev_view(b.data()), d, bytes, s);
    HIP_OK(hipGetLastError());
  }
  // bytes (a multiple of 4) of device data into out: a kernel writes them
  // into the pinned scratch, then the stream is waited for.
  void to_host(const void* d, size_t bytes, void* out) {
    if (h_small_bytes < bytes) {
      pinned().put(h_small, h_small_bytes);
      h_small = nullptr;
      h_small_bytes = 0;
      h_small = pinned().get(std::max(bytes, (size_t)4096), &h_small_bytes);
    }
    launch_copy_to_host(d, dev_view(h_small), bytes, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    std::memcpy(out, h_small, bytes);
  }
  hipEvent_t ev_rank = nullptr;
  // stats
  double t_assembly = 0, t_factor = 0, t_solve = 0, factor_flops = 0;
  hipEvent_t ev_t[3] = {nullptr, nullptr, nullptr};
  int max_rank = 0;
  int cap_hits[16] = {};  // compressions per level whose rank reached the cap with more rows left
  // per-kernel profile (HIP events around each batched launch)
  struct Pending {
    int t;
    hipEvent_t a, b;
    double flops, bytes;
  };
  std::vector<Pending> pend;
  std::vector<hipEvent_t> evpool;
  // slot = family + kOpTypes * (1 if the launch computes in FP32)
  double prof_ms[2 * kOpTypes] = {}, prof_flops[2 * kOpTypes] = {}, prof_bytes[2 * kOpTypes] = {};
  long prof_launch[2 * kOpTypes] = {};
  hipEvent_t get_event() {
    if (!evpool.empty()) {
      hipEvent_t e = evpool.back();
      evpool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIP_OK(hipEventCreate(&e));
    return e;
  }
  // Exact work counts that take a pass over every cluster window feed only
  // the statistics: they are computed later, while the host waits on the
  // stream anyway.
  std::vector<std::function<void()>> deferred;
  template <class F>
  void count_later(int op_t, F work) {
    const int slot = family(op_t) + (kF32 ? kOpTypes : 0);
    const bool tm = profile && timed(family(op_t));
    deferred.emplace_back([this, slot, tm, work] {
      const std::pair<double, double> w = work();
      factor_flops += w.first;
      if (tm) {
        prof_flops[slot] += w.first;
        prof_bytes[slot] += w.second;
      }
    });
  }
  // The same for a launch whose profile family is given directly.
  template <class F>
  void count_later_family(int fam, F work) {
    const int slot = fam + (kF32 ? kOpTypes : 0);
    const bool tm = profile && timed(fam);
    deferred.emplace_back([this, slot, tm, work] {
      const std::pair<double, double> w = work();
      factor_flops += w.first;
      if (tm) {
        prof_flops[slot] += w.first;
        prof_bytes[slot] += w.second;
      }
    });
  }
  // Work counted after its launch (it depends on results read back).
  void add_count(int fam, double f, double by) {
    factor_flops += f;
    if (profile && timed(fam)) {
      prof_flops[fam + (kF32 ? kOpTypes : 0)] += f;
      prof_bytes[fam + (kF32 ? kOpTypes : 0)] += by;
    }
  }
  void run_deferred() {
    PhaseScope ps_(hc, HP_DEFERRED);
    for (auto& f : deferred) f();
    deferred.clear();
  }
  void resolve_profile() {
    run_deferred();
    if (pend.empty()) return;
    HIP_OK(hipStreamSynchronize(s));
    for (const Pending& p : pend) {
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, p.a, p.b));
      prof_ms[p.t] += ms;
      prof_flops[p.t] += p.flops;
      prof_bytes[p.t] += p.bytes;
      prof_launch[p.t] += 1;
      evpool.push_back(p.a);
      evpool.push_back(p.b);
    }
    pend.clear();
  }

  void run(Stage& st) {
    PhaseScope ps_(hc, HP_RUN);
    if (st.empty()) return;
    if (hc.on) hc.upload_bytes[hc.level] += (double)st.blob.size();
    factor_flops += st.flops;
    const char* hb = nullptr;
    char* d = arena.upload(st.blob, s, &hb);
    launch_ops(st, d, hb);
    st.clear();
  }

  // Launches the ops of a stage whose blob is at device address d and host
  // address hb (default: the stage's own blob).
  void launch_ops(const Stage& st, char* d, const char* hb = nullptr) {
    if (!hb) hb = st.blob.data();
    for (const Op& op : st.ops) {
      hipEvent_t ea = nullptr, eb = nullptr;
      const bool tm = profile && timed(op_family(op));
      if (tm) {
        ea = get_event();
        eb = get_event();
        HIP_OK(hipEventRecord(ea, s));
      }
      switch (op.t) {
        case OP_GEMM:
          launch_gemm(reinterpret_cast<GemmDesc*>(d + op.off), op.count, op.a, op.b, op.ty, (int)op.off2, s);
          break;
        case OP_ADD: launch_add(reinterpret_cast<AddDesc*>(d + op.off), op.count, op.a, op.b, op.ty, s); break;
        case OP_QR:
          if (op.b) launch_qr_wave(reinterpret_cast<QrDesc*>(d + op.off), op.count, op.b, op.a, op.ty, s);
          else launch_qr(reinterpret_cast<QrDesc*>(d + op.off), op.count, op.off2, op.ty, s);
          break;
        case OP_RRQR:
          if (op.b == 2) {
            FillCopy fc{};
            if (op.off3) {
              std::memcpy(&fc, hb + (op.off3 - 1), sizeof(fc));
              fc.rec = reinterpret_cast<const ElimRec*>(d + (reinterpret_cast<uintptr_t>(fc.rec) - 1));
              fc.touch = reinterpret_cast<const int*>(d + (reinterpret_cast<uintptr_t>(fc.touch) - 1));
            }
            launch_rrqr_reg(reinterpret_cast<RrqrDesc*>(d + op.off), op.count, op.a, (int)op.off2, (int)op.off2b,
                            op.ty, op.off3 ? &fc : nullptr, s);
          } else if (op.b == 1) launch_rrqr_lds(reinterpret_cast<RrqrDesc*>(d + op.off), op.count, op.off2, (int)op.off2b, op.ty, s);
          else launch_rrqr_global(reinterpret_cast<RrqrDesc*>(d + op.off), op.count, op.a, (int)op.off2b, op.ty, s);
          break;
        case OP_FORMQRR:
          launch_formq_rr(reinterpret_cast<RrqrDesc*>(d + op.off), op.count, op.a, op.b, op.ty, s);
          break;
        case OP_FORMQ: break;  // Q is formed with the pivoted QR (OP_RRQR / OP_FORMQRR)
        case OP_STACKQR:
          launch_stackqr(reinterpret_cast<StackQrDesc*>(d + op.off), reinterpret_cast<BlkRef*>(d + op.off2),
                         op.count, op.a, op.ty, s);
          break;
        case OP_ROWCP: {
          Stage::RowCopy a;
          std::memcpy(&a, hb + op.off, sizeof(a));
          a.start = reinterpret_cast<const int*>(d + (reinterpret_cast<uintptr_t>(a.start) - 1));
          a.cnt = reinterpret_cast<const int*>(d + (reinterpret_cast<uintptr_t>(a.cnt) - 1));
          if (a.to_blocks)
            launch_leaf_gather(a.v, a.ldv, a.blk, a.bstride, a.ldb, a.start, a.cnt, a.n, a.nrhs, s);
          else
            launch_leaf_scatter(a.blk, a.bstride, a.ldb, a.v, a.ldv, a.start, a.cnt, a.n, a.nrhs, s);
          break;
        }
        case OP_FILLCP: {
          FillCopy a;
          std::memcpy(&a, hb + op.off, sizeof(a));
          a.rec = reinterpret_cast<const ElimRec*>(d + (reinterpret_cast<uintptr_t>(a.rec) - 1));
          a.touch = reinterpret_cast<const int*>(d + (reinterpret_cast<uintptr_t>(a.touch) - 1));
          launch_fill_copy(a, op.ty, s);
          break;
        }
        case OP_TXFORM: {
          TouchXform a;
          std::memcpy(&a, hb + op.off, sizeof(a));
          auto rebase = [&](const int*& p) {
            if (p) p = reinterpret_cast<const int*>(d + (reinterpret_cast<uintptr_t>(p) - 1));
          };
          rebase(a.touch_q);
          rebase(a.tidx);
          rebase(a.r_old);
          rebase(a.r_new);
          rebase(a.r_par);
          rebase(a.n);
          launch_touch_xform(a, op.ty, s);
          break;
        }
        case OP_SOLVE: {
          SolveArgs a;
          std::memcpy(&a, hb + op.off, sizeof(a));
          launch_solve(a, op.count, reinterpret_cast<double*>(op.off2), op.a, op.ty, s);
          break;
        }
        case OP_M2LASM: {
          M2LAssemble a;
          std::memcpy(&a, hb + op.off, sizeof(a));
          a.r = reinterpret_cast<const int*>(d + (reinterpret_cast<uintptr_t>(a.r) - 1));
          launch_m2l_assemble(a, op.ty, s);
          break;
        }
        case OP_TRANS: {
          TransArgs a;
          std::memcpy(&a, hb + op.off, sizeof(a));
          auto rebase = [&](const int*& p) {
            if (p) p = reinterpret_cast<const int*>(d + (reinterpret_cast<uintptr_t>(p) - 1));
          };
          rebase(a.choff);
          rebase(a.cr);
          rebase(a.r_par);
          launch_transition(a, op.ty, s);
          break;
        }
        case OP_ELIM: {
          ElimArgs a;
          std::memcpy(&a, hb + op.off, sizeof(a));
          a.rec = reinterpret_cast<const ElimRec*>(d + (reinterpret_cast<uintptr_t>(a.rec) - 1));
          if (a.rk) a.rk = reinterpret_cast<const int*>(d + (reinterpret_cast<uintptr_t>(a.rk) - 1));
          launch_elim(a, op.count, op.a, op.b, op.ty, s);
          break;
        }
        case OP_WSTACK: {
          WinStack a;
          std::memcpy(&a, hb + op.off, sizeof(a));
          auto rebase = [&](const int*& p) {
            if (p) p = reinterpret_cast<const int*>(d + (reinterpret_cast<uintptr_t>(p) - 1));
          };
          rebase(a.ids);
          rebase(a.r);
          rebase(a.r_par);
          if (op.b) launch_gram_win(a, op.a, op.ty, s);
          else launch_stackqr_win(a, op.a, op.ty, s);
          break;
        }
        case OP_RANKFIN: {
          RankFin a;
          std::memcpy(&a, hb + op.off, sizeof(a));
          auto rebase = [&](auto*& p) {
            using P = typename std::remove_reference<decltype(p)>::type;
            if (p) p = reinterpret_cast<P>(d + (reinterpret_cast<uintptr_t>(p) - 1));
          };
          rebase(a.q);
          rebase(a.n);
          rebase(a.r_new);
          rebase(a.r_lvl);
          rebase(a.g);
          launch_rank_finalize(a, s);
          break;
        }
        case OP_XFORM: break;  // family 2 has no launches
        case OP_GJREG: launch_gj_reg(reinterpret_cast<InvDesc*>(d + op.off), op.count, op.a, d_status, s); break;
        case OP_GJPANEL:  // off3: the panel width
          launch_gj_panel(reinterpret_cast<InvDesc*>(d + op.off), op.count, op.a, op.b, (int)op.off3,
                          reinterpret_cast<int*>(op.off2), op.a, d_status, s);
          break;
        case OP_GJREST:
          launch_gj_rest(reinterpret_cast<InvDesc*>(d + op.off), op.count, op.a, op.b, (int)op.off3,
                         reinterpret_cast<int*>(op.off2b), op.a, reinterpret_cast<double*>(op.off2),
                         op.off3 * (size_t)op.a, s);
          break;
        case OP_GJUNPERM:
          launch_gj_unpermute(reinterpret_cast<InvDesc*>(d + op.off), op.count, op.a,
                              reinterpret_cast<int*>(op.off2), op.a, s);
          break;
      }
      HIP_OK(hipGetLastError());
      if (tm) {
        HIP_OK(hipEventRecord(eb, s));
        const bool f32 = op.t == OP_GEMM ? (op.ty & 3) == 3 : op.t == OP_ADD ? (op.ty & 2) != 0 : op.ty != 0;  // elim: block type
        pend.push_back({op_family(op) + (f32 ? kOpTypes : 0), ea, eb, op.flops, op.bytes});
        if (pend.size() > 4096) resolve_profile();
      }
    }
  }

  // Inverse of the pivot blocks (Gauss-Jordan with partial pivoting).
  Buf wsInvT, wsInvP;
  // Matrices up to kGjRegMax are inverted whole in registers, one workgroup
  // each, in launches of one size class (the class sets the workgroup
  // shape); larger ones by panels.
  void plan_inverse(Stage& st, const std::vector<InvDesc>& all) {
    PhaseScope ps_(hc, HP_INVPLAN);
    if (all.empty()) return;
    std::vector<InvDesc> cls[3], big;
    for (const auto& d : all) {
      if (d.m > kGjRegMax) big.push_back(d);
      else cls[d.m <= 64 ? 0 : d.m <= 128 ? 1 : 2].push_back(d);
    }
    for (const auto& c : cls) st.inv_reg(c);
    if (big.empty()) return;
    int mm = 0;
    for (const auto& d : big) mm = std::max(mm, d.m);
    double* tmp = wsInvT.need((size_t)big.size() * kInvNb * mm, s);
    int* piv = wsInvP.need<int>((size_t)big.size() * mm + 1, s);
    st.inv_blocked(big, piv, tmp, inv_panel_width(mm));
  }

  // ---------------------------------------------------------------- tree
  // Points (original order, device) -> tree order on the device; the leaf
  // populations come back to the host for planning.
  void build_tree(const double* d_points_in) {
    PhaseScope ps_(hc, HP_TREE);
    kappa = 2;
    while ((int64_t)leaf * (1LL << (2 * kappa)) < N) ++kappa;
    if (kappa > kMaxLevels) throw BadArg{};
    const int nb = 1 << kappa;
    const int nleaf = nb * nb;
    const int n = (int)N;
    d_pts = dalloc<double>(s, 2 * N);
    d_perm = dalloc<int>(s, N);
    d_leaf_start = dalloc<int>(s, nleaf);
    d_leaf_n = dalloc<int>(s, nleaf + 1);  // + the rejection flag
    int* bad = d_leaf_n + nleaf;
    size_t tmp_bytes = 0;
    HIP_OK(tree_scratch_bytes(n, nleaf, 2 * kappa, &tmp_bytes));
    int* ki = wsS1.need<int>(3 * N, s);
    void* tmp = wsS2.need<char>(tmp_bytes, s);
    HIP_OK(hipMemsetAsync(d_leaf_n, 0, sizeof(int) * (nleaf + 1), s));
    HIP_OK(launch_tree_build(d_points_in, n, lox, loy, size, kappa, ki, ki + N, ki + 2 * N, d_perm, d_leaf_n,
                             d_leaf_start, bad, d_pts, tmp, tmp_bytes, s));
    if (kf.kind == 0) launch_tree_distinct(d_pts, d_leaf_start, d_leaf_n, nleaf, bad, s);  // 1/r: distinct
    if (diag_mode == IFMM_DIAG_VECTOR) launch_check_finite(d_diag_user, n, bad, s);
    leaf_n.assign(nleaf + 1, 0);
    to_host(d_leaf_n, sizeof(int) * (nleaf + 1), leaf_n.data());
    if (leaf_n[nleaf]) throw BadArg{};
    leaf_n.resize(nleaf);
    leaf_start.assign(nleaf, 0);
    for (int i = 1; i < nleaf; ++i) leaf_start[i] = leaf_start[i - 1] + leaf_n[i - 1];
    lv.assign(kappa + 1, Level<T>());
    for (int k = 2; k <= kappa; ++k) {
      Level<T>& L = lv[k];
      L.k = k;
      L.nside = 1 << k;
      L.nc = L.nside * L.nside;
      L.n.assign(L.nc, 0);
      L.r.assign(L.nc, 0);
      L.colour.assign(L.nc, 0);
      L.nbr9.assign((size_t)L.nc * 9, -1);
      for (int i = 0; i < L.nc; ++i) {
        const int ix = demorton_x(i), iy = demorton_y(i);
        L.colour[i] = 3 * (ix % 3) + (iy % 3);
        for (int s = 0; s < 9; ++s) {
          const int jx = ix + s9_dx(s), jy = iy + s9_dy(s);
          if (jx >= 0 && jy >= 0 && jx < L.nside && jy < L.nside) L.nbr9[(size_t)i * 9 + s] = morton2(jx, jy);
        }
      }
      L.rpad = rpad;
    }
    for (int i = 0; i < nleaf; ++i) lv[kappa].n[i] = leaf_n[i];
  }

  // ------------------------------------------------------------- FMM product
  // y = A x (tree order, column-major ld N); diag null = off-diagonal part only.
  // coeff: the multipole / local coefficients (fmm_coeff_count doubles), null =
  // the handle's own workspace.
  size_t fmm_coeff_count(int nrhs) const {
    size_t tot = 0;
    for (int k = 2; k <= kappa; ++k) tot += (size_t)(1 << (2 * k)) * p2 * nrhs;
    return 2 * tot;
  }
  // tables / kov: the M2L tables and kernel of another kernel on the same
  // tree (its near field evaluated on the fly); null = the factored kernel.
  void fmm_apply_tree(const double* xs, double* ys, int nrhs, const double* diag, double* coeff = nullptr,
                      double* const* tables = nullptr, const KernelFn* kov = nullptr) {
    const int nleaf = 1 << (2 * kappa);
    double* W[kMaxLevels + 1] = {};
    double* G[kMaxLevels + 1] = {};
    double* base = coeff ? coeff : wsVec.need(fmm_coeff_count(nrhs), s);
    size_t off = 0;
    for (int k = 2; k <= kappa; ++k) {
      W[k] = base + off;
      off += (size_t)(1 << (2 * k)) * p2 * nrhs;
    }
    for (int k = 2; k <= kappa; ++k) {
      G[k] = base + off;
      off += (size_t)(1 << (2 * k)) * p2 * nrhs;
    }
    launch_p2m(d_pts, d_leaf_start, d_leaf_n, nleaf, kappa, lox, loy, size, p, xs, (int)N, nrhs, W[kappa], s);
    for (int k = kappa - 1; k >= 2; --k) launch_m2m(d_E, p, 1 << (2 * k), W[k + 1], W[k], nrhs, s);
    for (int k = 2; k <= kappa; ++k) launch_m2l(p, k, tables ? tables[k] : d_table[k], W[k], G[k], nrhs, s);
    for (int k = 2; k < kappa; ++k) launch_l2l(d_E, p, 1 << (2 * k), G[k], G[k + 1], nrhs, s);
    if (kov)
      launch_l2p_p2p(d_pts, d_leaf_start, d_leaf_n, d_nbr9_leaf, nleaf, kappa, lox, loy, size, p, *kov,
                     G[kappa], xs, (int)N, diag, ys, (int)N, nrhs, s);
    else if (d_near)
      launch_l2p_near(d_pts, d_leaf_start, d_leaf_n, d_nbr9_leaf, nleaf, kappa, lox, loy, size, p, d_near,
                      d_near_off, G[kappa], xs, (int)N, diag, ys, (int)N, nrhs, s);
    else
      launch_l2p_p2p(d_pts, d_leaf_start, d_leaf_n, d_nbr9_leaf, nleaf, kappa, lox, loy, size, p, kf,
                     G[kappa], xs, (int)N, diag, ys, (int)N, nrhs, s);
    HIP_OK(hipGetLastError());
  }

  // --------------------------------------------------------------- assembly
  void assemble(const double* d_points_in) {
    PhaseScope ps_(hc, HP_ASSEMBLY);
    // the kernel tables and the transfer matrices depend on the depth only:
    // queued ahead of the tree, in pinned memory, so the device works while
    // the host reads the leaf populations back and plans
    kappa = 2;
    while ((int64_t)leaf * (1LL << (2 * kappa)) < N) ++kappa;
    if (kappa > kMaxLevels) throw BadArg{};
    d_table.assign(kappa + 1, nullptr);
    for (int k = 2; k <= kappa; ++k) {
      d_table[k] = dalloc<double>(s, (size_t)49 * p2 * p2);
      launch_m2l_table(kf, p, 0.5 * size / (1 << k), d_table[k], s);
    }
    {
      const std::vector<double> E = transfer_host(p);
      up_E.resize(E.size() * sizeof(double));
      std::memcpy(up_E.data(), E.data(), up_E.size());
      d_E = dalloc<double>(s, E.size());
      upload_pinned(d_E, up_E, up_E.size());
    }
    build_tree(d_points_in);
    const int nleaf = 1 << (2 * kappa);
    d_nbr9_leaf = dalloc<int>(s, (size_t)nleaf * 9);
    d_diag = dalloc<double>(s, N);
    d_status = dalloc<Status>(s, 1);
    HIP_OK(hipMemsetAsync(d_status, 0, sizeof(Status), s));
    up_nbr9.resize(sizeof(int) * nleaf * 9);
    std::memcpy(up_nbr9.data(), lv[kappa].nbr9.data(), up_nbr9.size());
    upload_pinned(d_nbr9_leaf, up_nbr9, up_nbr9.size());
    // diagonal
    if (diag_mode == IFMM_DIAG_ROWSUM) {
      double* ones = wsS1.need(N, s);
      launch_fill(ones, N, 1.0, s);
      fmm_apply_tree(ones, d_diag, 1, nullptr);
      launch_add_const(d_diag, N, c0, s);
    } else if (diag_mode == IFMM_DIAG_VECTOR) {
      launch_gather_rows(d_diag_user, (int)N, d_perm, (int)N, 1, d_diag, (int)N, s);
    } else {
      launch_fill(d_diag, N, c0, s);
    }
    HIP_OK(hipGetLastError());

    // ---- leaf level: interpolation, orthonormal bases, near field
    Level<T>& Lf = lv[kappa];
    int nmax = 0;
    for (int i = 0; i < nleaf; ++i) {
      nmax = std::max(nmax, Lf.n[i]);
      Lf.r[i] = std::min(Lf.n[i], p2);
    }
    Lf.set_pads(rup(std::max(nmax, 1), 8));
    Lf.P = dalloc<T>(s, Lf.sP * 9 * Lf.nc);
    Lf.Qm = dalloc<T>(s, Lf.sQ * 9 * Lf.nc);
    Lf.L = dalloc<T>(s, Lf.sL * 9 * Lf.nc);
    Lf.U = dalloc<T>(s, Lf.sU * Lf.nc);
    Lf.Dinv = dalloc<double>(s, Lf.sD * Lf.nc);
    // The product's near field is stored once (FP64, every leaf's row block
    // over its neighbours' points) when it fits kNearStoreMax; the refinement
    // sweeps then read it instead of evaluating the kernel again.
    {
      std::vector<size_t>& off = near_off_h;
      off.assign(nleaf, 0);
      size_t tot = 0;
      for (int i = 0; i < nleaf; ++i) {
        size_t c = 0;
        for (int q = 0; q < 9; ++q) {
          const int j = Lf.nbr9[(size_t)i * 9 + q];
          if (j >= 0) c += (size_t)leaf_n[j];
        }
        off[i] = tot;
        tot += c * (size_t)leaf_n[i];
      }
      if (tot * sizeof(double) <= kNearStoreMax) {
        d_near = dalloc<double>(s, std::max<size_t>(tot, 1));
        d_near_off = dalloc<size_t>(s, nleaf);
        up_near_off.resize(sizeof(size_t) * nleaf);
        std::memcpy(up_near_off.data(), off.data(), up_near_off.size());
        upload_pinned(d_near_off, up_near_off, up_near_off.size());
      }
    }
    // The clearing of the leaf fill slots and the near field (P blocks and
    // the stored FP64 near field) run on a second stream beside the basis
    // QRs and the M2L assembly below, whose latency-bound launches leave
    // most of the GPU idle, for problems large enough to fill both; the
    // factorisation starts after both.
    SideStream side(s, N >= ((int64_t)1 << 18));
    HIP_OK(hipMemsetAsync(Lf.Qm, 0, sizeof(T) * Lf.sQ * 9 * Lf.nc, side.s));
    HIP_OK(hipMemsetAsync(Lf.L, 0, sizeof(T) * Lf.sL * 9 * Lf.nc, side.s));
    launch_near_field(d_pts, d_leaf_start, d_leaf_n, d_nbr9_leaf, nleaf, kf, d_diag, Lf.P, kF32 ? 1 : 0,
                      Lf.sP, Lf.npad, nmax, d_near, d_near_off, side.s);
    HIP_OK(hipGetLastError());
    // Interpolation and orthonormalisation in FP64; an FP32 factor takes the
    // rounded bases.
    double* U64;
    if constexpr (kF32) U64 = wsS2.need<double>(Lf.sU * Lf.nc, s);
    else U64 = Lf.U;
    launch_leaf_interp(d_pts, d_leaf_start, d_leaf_n, nleaf, kappa, lox, loy, size, p, U64, Lf.sU,
                       Lf.npad, nmax, s);
    // R factors of every level at assembly (r x p^2), kept until M2L is built
    std::vector<double*> Ra(kappa + 1, nullptr);
    for (int k = 2; k <= kappa; ++k) Ra[k] = dalloc<double>(s, (size_t)lv[k].nc * rpad * p2);
    {
      Stage st;
      std::vector<QrDesc> q;
      for (int i = 0; i < nleaf; ++i)
        if (Lf.n[i] > 0) q.push_back({U64 + (size_t)i * Lf.sU, Ra[kappa] + (size_t)i * rpad * p2, Lf.n[i], p2, Lf.npad, rpad});
      st.qr(q);
      if constexpr (kF32) {
        std::vector<AddDesc> cv;
        for (int i = 0; i < nleaf; ++i)
          if (Lf.n[i] > 0) cv.push_back({U64 + (size_t)i * Lf.sU, Lf.Ub(i), Lf.n[i], Lf.r[i], Lf.npad, Lf.npad, 0, 1.0, 0.0});
        st.add(cv);
      }
      run(st);
    }
    // ---- non-leaf levels at assembly: S_P = [R_c E_c], QR, transfer blocks
    for (int k = kappa; k >= 2; --k) {
      Level<T>& L = lv[k];
      L.UP = dalloc<T>(s, L.sUP == 0 ? (size_t)rpad * rpad * L.nc : L.sUP * L.nc);
    }
    for (int k = kappa - 1; k >= 2; --k) {
      Level<T>& L = lv[k];
      Level<T>& C = lv[k + 1];
      L.choff.assign((size_t)L.nc * 4, 0);
      int nm = 0;
      for (int P = 0; P < L.nc; ++P) {
        int o = 0;
        for (int c = 0; c < 4; ++c) {
          L.choff[(size_t)P * 4 + c] = o;
          o += C.r[4 * P + c];
        }
        L.n[P] = o;
        L.r[P] = std::min(o, p2);
        nm = std::max(nm, o);
      }
      const int npA = rup(std::max(nm, 1), 8);
      double* SP = wsA.need((size_t)L.nc * npA * p2, s);
      Stage st;
      std::vector<GemmDesc> g;
      for (int P = 0; P < L.nc; ++P)
        for (int c = 0; c < 4; ++c) {
          const int ch = 4 * P + c;
          if (C.r[ch] == 0) continue;
          g.push_back({Ra[k + 1] + (size_t)ch * rpad * p2, d_E + (size_t)c * p2 * p2,
                       SP + (size_t)P * npA * p2 + L.choff[(size_t)P * 4 + c], C.r[ch], p2, p2, rpad, p2,
                       npA, 0, 0, 1.0, 0.0});
        }
      st.gemm(g);
      std::vector<QrDesc> q;
      for (int P = 0; P < L.nc; ++P)
        if (L.n[P] > 0) q.push_back({SP + (size_t)P * npA * p2, Ra[k] + (size_t)P * rpad * p2, L.n[P], p2, npA, rpad});
      st.qr(q);
      C.sUP = (size_t)rpad * rpad;
      std::vector<AddDesc> cp;
      for (int P = 0; P < L.nc; ++P)
        for (int c = 0; c < 4; ++c) {
          const int ch = 4 * P + c;
          if (C.r[ch] == 0) continue;
          cp.push_back({SP + (size_t)P * npA * p2 + L.choff[(size_t)P * 4 + c], C.UPb(ch), C.r[ch], L.r[P],
                        npA, rpad, 0, 1.0, 0.0});
        }
      st.add(cp);
      run(st);
    }
    for (int k = 2; k <= kappa; ++k) {
      Level<T>& L = lv[k];
      L.sUP = (size_t)rpad * rpad;
      L.sM = (size_t)rpad * rpad;

    }
    // ---- M2L in orthonormal coordinates: M_il = R_i K(dx,dy) R_l^T
    for (int k = 2; k <= kappa; ++k) {
      Level<T>& L = lv[k];
      // the assembly writes every far-field block (its partner's rank wide)
      // and zeroes the neighbours' slots, where fill-in accumulates; no other
      // part of a slot is ever read
      L.M = dalloc<T>(s, L.sM * 36 * L.nc);
      M2LAssemble a{};
      a.R = Ra[k];
      a.table = d_table[k];
      a.M = L.M;
      a.sR = (size_t)rpad * p2;
      a.sM = L.sM;
      a.nc = L.nc;
      a.nside = L.nside;
      a.rpad = rpad;
      a.p2 = p2;
      double f = 0, by = 0;
      for (int i = 0; i < L.nc; ++i) {
        if (L.r[i] == 0) continue;
        const int ix = demorton_x(i), iy = demorton_y(i);
        for (int sl = 0; sl < 36; ++sl) {
          const int jx = 2 * (ix >> 1) - 2 + sl / 6, jy = 2 * (iy >> 1) - 2 + sl % 6;
          if (jx < 0 || jy < 0 || jx >= L.nside || jy >= L.nside) continue;
          if (std::abs(jx - ix) <= 1 && std::abs(jy - iy) <= 1) continue;
          const double rl = L.r[morton2(jx, jy)];
          if (rl == 0) continue;
          f += 2.0 * L.r[i] * p2 * (p2 + rl);
          by += 8.0 * ((double)L.r[i] * p2 + (double)p2 * p2 + rl * p2) + sizeof(T) * L.r[i] * rl;
        }
      }
      Stage st;
      st.m2l_assemble<T>(a, L.r, f, by);
      run(st);
    }
    for (int k = 2; k <= kappa; ++k) dfree(s, Ra[k]);
    // ---- far-field weights of the parent levels, top-down
    for (int k = 2; k < kappa; ++k) {
      Level<T>& L = lv[k];
      L.Om = dalloc<T>(s, L.sUP * L.nc);
      std::vector<int> ids;
      for (int i = 0; i < L.nc; ++i)
        if (L.r[i] > 0) ids.push_back(i);
      weights(k, ids, L.Om, true);
    }
  }

  // Omega of the clusters `ids` at level k: R factor of the stacked
  // transposed far-field row (+ the parent chain UP Omega_parent^T), written
  // to out + t * rpad^2 (or out + ids[t] * rpad^2 when by_id).
  // With ext, the launches are appended to that stage (run by the caller).
  void weights(int k, const std::vector<int>& ids, T* out, bool by_id, Stage* ext = nullptr) {
    PhaseScope ps_(hc, HP_WEIGHTS);
    Level<T>& L = lv[k];
    const int nt = (int)ids.size();
    if (nt == 0) return;
    const size_t so = (size_t)rpad * rpad;
    T* Z = nullptr;
    Stage own;
    Stage& st = ext ? *ext : own;
    if (k > 2) {
      Z = wsZ.need<T>((size_t)nt * so, s);
      Level<T>& Pl = lv[k - 1];
      std::vector<GemmDesc> g;
      for (int t = 0; t < nt; ++t) {
        const int q = ids[t], P = q >> 2, rP = Pl.r[P];
        if (rP > 0 && L.r[q] > 0)
          g.push_back({Pl.Omb(P), L.UPb(q), Z + (size_t)t * so, rP, L.r[q], rP, rpad, rpad, rpad, 0, 1, 1.0, 0.0});
      }
      st.gemm(g);
    }
    // FP32 factor: R from the FP64 Gram matrix (one workgroup per cluster).
    // FP64 factor: Householder steps; with few clusters (coarse levels) each
    // stack is split into segments handled by separate workgroups, then the R
    // factor of the stacked partial R's is taken (the same R up to rounding).
    const bool gram = kF32;
    const int S = gram ? 1 : std::max(1, std::min(8, (3072 + nt - 1) / nt));
    T* part = S > 1 ? wsSeg.need<T>((size_t)nt * S * so, s) : nullptr;
    WinStack a{};
    a.M = L.M;
    a.Z = Z;
    a.out = S > 1 ? part : out;
    a.sM = L.sM;
    a.so = so;
    a.rpad = rpad;
    a.nside = L.nside;
    a.ldo = rpad;
    a.nt = nt;
    a.S = S;
    a.out_by_id = by_id ? 1 : 0;
    a.max_rows = *std::max_element(L.r.begin(), L.r.end());
    if (k > 2) a.max_rows = std::max(a.max_rows, *std::max_element(lv[k - 1].r.begin(), lv[k - 1].r.end()));
    a.max_rows = std::max(a.max_rows, 1);
    st.win_stack<T>(a, ids, L.r, k > 2 ? &lv[k - 1].r : nullptr, false, gram);
    count_later(OP_WSTACK, [a, ids, r = L.r, rp = k > 2 ? lv[k - 1].r : std::vector<int>(), par = k > 2] {
      return winstack_work(a, ids, r, par ? &rp : nullptr, sizeof(T), gram);
    });
    if (S > 1) {
      std::vector<StackQrDesc> s2;
      std::vector<BlkRef> b2;
      for (int t = 0; t < nt; ++t) {
        const int q = ids[t], rq = L.r[q];
        if (rq == 0) continue;
        StackQrDesc fin{out + (by_id ? (size_t)q : (size_t)t) * so, rq, rpad, (int)b2.size(), S};
        for (int g0 = 0; g0 < S; ++g0) b2.push_back({part + ((size_t)t * S + g0) * so, rpad, rq, 0});
        s2.push_back(fin);
      }
      st.stackqr(s2, b2);
    }
    if (!ext) run(st);
  }

  // ------------------------------------------------------------ factorisation
  void factor() {
    plan.assign(kappa + 1, std::vector<std::vector<Elim>>(9));
    erec.assign(kappa + 1, std::vector<std::vector<ElimRec>>(9));
    for (int k = kappa; k >= 2; --k) {
      if (hc.on) {
        hc.charge(HostClock::Clock::now());
        hc.level = k;
      }
      for (int c = 0; c < 9; ++c) phase(k, c);
      Level<T>& L = lv[k];
      for (int i = 0; i < L.nc; ++i) max_rank = std::max(max_rank, L.r[i]);
      if (k > 2) transition(k);
    }
    if (hc.on) {
      hc.charge(HostClock::Clock::now());
      hc.level = 0;
    }
    top();
    // the records drive the solve sweeps
    // (gathered in pinned memory: the copy is queued without waiting for the
    // launches ahead of it, and the solve plan is built meanwhile)
    erec_off.assign(kappa + 1, std::vector<size_t>(9, 0));
    size_t nrec = 0;
    for (int k = 2; k <= kappa; ++k)
      for (int c = 0; c < 9; ++c) {
        erec_off[k][c] = nrec;
        nrec += erec[k][c].size();
      }
    Blob all;
    all.resize(std::max<size_t>(nrec, 1) * sizeof(ElimRec));
    for (int k = 2; k <= kappa; ++k)
      for (int c = 0; c < 9; ++c)
        if (!erec[k][c].empty())
          std::memcpy(all.data() + erec_off[k][c] * sizeof(ElimRec), erec[k][c].data(),
                      erec[k][c].size() * sizeof(ElimRec));
    d_erec = dalloc<ElimRec>(s, std::max<size_t>(nrec, 1));
    upload_pinned(d_erec, all, sizeof(ElimRec) * nrec);
    solve_plan(1);  // planned while the last launches run
    run_deferred();
    HIP_OK(hipStreamSynchronize(s));
    resolve_profile();
    Status hs{};
    to_host(d_status, sizeof(Status), &hs);
    if (hs.singular) throw 3;
  }

  ElimArgs elim_args(const Level<T>& L, T* X, T* F, int wpad, int fpad, int nb) {
    ElimArgs a{};
    a.P = L.P;
    a.Qm = L.Qm;
    a.L = L.L;
    a.M = L.M;
    a.U = L.U;
    a.Dinv = L.Dinv;
    a.X = X;
    a.F = F;
    a.sP = L.sP;
    a.sQ = L.sQ;
    a.sL = L.sL;
    a.sM = L.sM;
    a.sU = L.sU;
    a.sD = L.sD;
    a.sX = (size_t)L.mpad * wpad;
    a.nb = nb;
    a.npad = L.npad;
    a.rpad = rpad;
    a.mpad = L.mpad;
    a.fpad = fpad;
    a.npair = kPairs.count;
    for (int sa = 0; sa < 9; ++sa)
      for (int sb = 0; sb < 9; ++sb) {
        a.pair[9 * sa + sb] = (signed char)kPairs.idx[sa][sb];
        if (kPairs.idx[sa][sb] >= 0) a.plist[kPairs.idx[sa][sb]] = (unsigned char)(9 * sa + sb);
      }
    return a;
  }

  void phase(int k, int c) {
    PhaseScope ps_(hc, HP_RECORDS);
    Level<T>& L = lv[k];
    std::vector<Elim>& E = plan[k][c];
    for (int i = 0; i < L.nc; ++i) {
      if (L.colour[i] != c || L.n[i] == 0) continue;
      Elim e;
      e.i = i;
      e.ni = L.n[i];
      e.ri = L.r[i];
      e.m = e.ni + e.ri;
      int off = 0;
      for (int sp = 0; sp < 9; ++sp) {
        UnitH u;
        if (sp == 4) {
          u = {i, 2, e.ri, 0};
        } else {
          const int j = L.nbr9[(size_t)i * 9 + sp];
          if (j >= 0 && L.n[j] > 0) {
            if (L.colour[j] > c) u = {j, 1, L.n[j], 0};
            else if (L.r[j] > 0) u = {j, 2, L.r[j], 0};
          }
        }
        if (u.kind) {
          u.off = off;
          off += u.size;
        }
        e.u[sp] = u;
      }
      E.push_back(e);
    }
    // The batch's eliminations run concurrently: their 3 x 3 neighbourhoods
    // (every block an elimination reads or writes, and every cluster it
    // recompresses) must be disjoint.  The colouring gives it; checked here.
    if (batch_mark.size() < (size_t)L.nc) batch_mark.assign(L.nc, 0);
    ++batch_stamp;
    for (const Elim& e : E)
      for (int sp = 0; sp < 9; ++sp) {
        const int j = sp == 4 ? e.i : L.nbr9[(size_t)e.i * 9 + sp];
        if (j < 0) continue;
        if (batch_mark[j] == batch_stamp) throw Broken{"a colour batch with overlapping neighbourhoods", __LINE__};
        batch_mark[j] = batch_stamp;
      }
    const int nb = (int)E.size();
    if (nb == 0) return;
    const int fpad = std::max(L.npad, rpad);
    const int wpad = 8 * fpad + rpad;
    T* X = wsX.need<T>((size_t)nb * L.mpad * wpad, s);
    T* F = wsF.need<T>((size_t)nb * kPairs.count * fpad * fpad, s);
    // ---- eliminate the batch: pivot inverse, X = D^-1 B, Schur updates
    {
      Stage st;
      std::vector<ElimRec> recs(nb);
      int maxm = 0, maxu = 0;
      const double es = sizeof(T);
      for (int b = 0; b < nb; ++b) {
        const Elim& e = E[b];
        ElimRec& r = recs[b];
        r.i = e.i;
        r.ni = e.ni;
        r.ri = e.ri;
        r.m = e.m;
        maxm = std::max(maxm, e.m);
        for (int sp = 0; sp < 9; ++sp) {
          r.cl[sp] = e.u[sp].cl;
          r.kind[sp] = e.u[sp].kind;
          r.size[sp] = e.u[sp].size;
          r.off[sp] = e.u[sp].off;
          if (e.u[sp].kind) maxu = std::max(maxu, e.u[sp].size);
        }
      }
      // algorithmic work of steps 1-3, counted while the host next waits
      // (E is plan[k][c], kept until the factorisation ends)
      auto work = [&E, es](int step) {
        double f = 0, by = 0;
        for (const Elim& e : E) {
          if (step == 2) {
            // Schur updates, counted per elimination GEMM: the pivot column
            // C (h x n_i) and X (n_i x w) read once, every target block read
            // and written once (a fill block between well-separated units is
            // only written)
            double h = 0, wcols = 0;
            for (int sa = 0; sa < 9; ++sa) {
              if (!e.u[sa].kind) continue;
              wcols += e.u[sa].size;
              if (sa != 4) h += e.u[sa].size;
            }
            by += es * (h * e.ni + e.ni * wcols);
            for (int sa = 0; sa < 9; ++sa) {
              if (sa == 4 || !e.u[sa].kind) continue;
              for (int sb = 0; sb < 9; ++sb) {
                if (!e.u[sb].kind) continue;
                const double ma = e.u[sa].size, nbu = e.u[sb].size;
                f += 2.0 * ma * nbu * e.ni;
                by += es * (kPairs.idx[sa][sb] >= 0 && !(e.u[sa].kind == 2 && e.u[sb].kind == 2) ? 1.0 : 2.0) * ma *
                      nbu;
              }
            }
            continue;
          }
          for (int sp = 0; sp < 9; ++sp) {
            if (!e.u[sp].kind) continue;
            if (step == 1 && sp != 4) {
              f += 2.0 * e.m * e.u[sp].size * e.ni;
              by += 8.0 * e.m * e.ni + es * (2.0 * e.ni * e.u[sp].size + (double)e.m * e.u[sp].size);
            }
            if (step == 3) by += es * 3.0 * e.ri * e.u[sp].size;
          }
        }
        return std::make_pair(f, by);
      };
      count_later_family(12, [work] {
        const auto a = work(1), b = work(3);
        return std::make_pair(a.first + b.first, a.second + b.second);
      });
      count_later_family(8, [work] { return work(2); });
      ElimArgs a = elim_args(L, X, F, wpad, fpad, nb);
      const size_t ro = st.push(recs.data(), recs.size() * sizeof(ElimRec)) + 1;
      erec[k][c] = recs;
      double bd = 0;
      std::vector<InvDesc> inv;
      for (const Elim& e : E) {
        inv.push_back({L.Db(e.i), e.m, L.mpad});
        bd += (es + 8.0) * e.m * (double)e.m;
      }
      st.elim<T>(a, ro, 0, maxm, maxm, 0.0, bd);
      plan_inverse(st, inv);
      st.elim<T>(a, ro, 1, maxm, maxu, 0.0, 0.0);
      st.elim<T>(a, ro, 2, maxu, maxu, 0.0, 0.0);
      st.elim<T>(a, ro, 3, rpad, maxu, 0.0, 0.0);
      // the compression's work up to the rank read-back depends only on
      // host-known shapes: it joins this stage, uploaded and launched at once
      compress(k, c, E, X, F, wpad, fpad, st);
    }
  }

  // pre: launches not yet run (the batch's elimination); run with the first
  // chunk of the compression.
  void compress(int k, int c, const std::vector<Elim>& E, T* X, T* F, int wpad, int fpad, Stage& pre) {
    PhaseScope ps_(hc, HP_COMPRESS_PRE);
    Level<T>& L = lv[k];
    struct Touch {
      int q, b, sq;
    };
    std::vector<Touch> touch;
    std::vector<int> tidx(L.nc, -1);
    for (int b = 0; b < (int)E.size(); ++b)
      for (int sq = 0; sq < 9; ++sq) {
        const UnitH& u = E[b].u[sq];
        if (u.kind != 1) continue;
        int cu = 0;
        for (int s2 = 0; s2 < 9; ++s2) {
          if (kPairs.idx[sq][s2] < 0 || !E[b].u[s2].kind) continue;
          cu += E[b].u[s2].size;
        }
        if (cu == 0) continue;
        tidx[u.cl] = (int)touch.size();
        touch.push_back({u.cl, b, sq});
      }
    const int nt = (int)touch.size();
    if (nt == 0) {
      run(pre);
      return;
    }
    const double eps_c = kF32 ? std::max(eps, kF32EpsFloor) : eps;
    // Omega from the current state (before any basis change)
    T* Om = wsB.need<T>((size_t)nt * rpad * rpad, s);
    std::vector<int> ids(nt);
    for (int t = 0; t < nt; ++t) ids[t] = touch[t].q;
    weights(k, ids, Om, false, &pre);
    // new bases, chunk by chunk: pivoted QR of [U Omega^T | fill of the row]
    const int cmax = rpad + 5 * fpad;
    T* Uh = wsQ.need<T>((size_t)nt * L.sU, s);
    T* Tt = wsR.need<T>((size_t)nt * rpad * rpad, s);
    const size_t per = (size_t)L.npad * cmax;
    int chunk = (int)std::min<size_t>(nt, std::max<size_t>(64, ((size_t)12 << 30) / (per * sizeof(T))));
    T* A = wsT.need<T>(per * chunk + (size_t)chunk * 2 * kMaxRank, s);
    T* tauA = A + per * chunk;
    if (rank_cap < (size_t)2 * nt) {
      dfree(s, d_rank);
      rank_cap = (size_t)2 * nt;
      d_rank = dalloc<int>(s, rank_cap);
    }
    std::vector<int> rnew(nt);
    std::vector<char> in_regs(nt);
    for (int t0 = 0; t0 < nt; t0 += chunk) {
      const int t1 = std::min(nt, t0 + chunk);
      Stage own;
      Stage& st = t0 == 0 ? pre : own;
      std::vector<GemmDesc> g;
      std::vector<int> fc;  // fill copies on the device: (b, sq, nq, col0, read in place) per touch
      double fcb = 0;
      std::vector<RrqrDesc> rq;
      for (int t = t0; t < t1; ++t) {
        const Touch& tc = touch[t];
        const int q = tc.q, nq = L.n[q], rq0 = L.r[q];
        T* Aw = A + (size_t)(t - t0) * per;
        g.push_back({L.Ub(q), Om + (size_t)t * rpad * rpad, Aw, nq, rq0, rq0, L.npad, rpad, L.npad, 0, 1, 1.0, 0.0});
        int col = rq0;
        for (int s2 = 0; s2 < 9; ++s2) {
          if (kPairs.idx[tc.sq][s2] < 0 || !E[tc.b].u[s2].kind) continue;
          col += E[tc.b].u[s2].size;
        }
        T* tb = tauA + (size_t)(t - t0) * 2 * kMaxRank;
        rq.push_back({Aw, tb, tb + kMaxRank, d_rank + 2 * t, d_rank + 2 * t + 1, nq, col, L.npad,
                      std::min(nq, r_cap), eps_c, 1, Uh + (size_t)t * L.sU, L.npad});
        // a register pivoted QR reads this touch's fill blocks in place: no copy
        const bool in_place = Stage::rrqr_in_regs(rq.back()) && rrqr_reg_reads_fill(rrqr_reg_rows(nq, rq.back().ty), rq.back().ty);
        if (in_place) rq.back().fill_t = t - t0;
        else fcb += 2.0 * sizeof(T) * nq * (double)(col - rq0);
        fc.insert(fc.end(), {tc.b, tc.sq, nq, rq0, in_place ? 1 : 0});
      }
      st.gemm(g);
      size_t fill_off = 0;
      {
        FillCopy f{};
        f.F = F;
        f.A = A;
        f.per = per;
        f.fpad = fpad;
        f.npad = L.npad;
        f.npair = kPairs.count;
        f.nt = t1 - t0;
        for (int x = 0; x < 81; ++x) f.pair[x] = (signed char)kPairs.idx[x / 9][x % 9];
        fill_off = st.fill_copy<T>(f, erec[k][c], fc, fcb);
      }
      st.rrqr(rq, fill_off);
      for (int t = t0; t < t1; ++t) in_regs[t] = Stage::rrqr_in_regs(rq[t - t0]);
      run(st);
    }
    // The ranks go to the host (a kernel writes them into a pinned buffer;
    // event) while the basis change is queued at once: its launches take the
    // new ranks from the device (RankFin), so the device does not wait for
    // the host's planning.
    const size_t rb = sizeof(int) * 2 * (size_t)nt;
    if (h_rank_bytes < rb) {
      pinned().put(reinterpret_cast<char*>(h_rank), h_rank_bytes);
      h_rank = nullptr;
      h_rank_dev = nullptr;
      h_rank_bytes = 0;
      size_t got = 0;
      h_rank = reinterpret_cast<int*>(pinned().get(std::max(rb, (size_t)64 << 10), &got));
      h_rank_bytes = got;
      HIP_OK(hipHostGetDevicePointer(reinterpret_cast<void**>(&h_rank_dev), h_rank, 0));
    }
    launch_copy_to_host(d_rank, h_rank_dev, rb, s);
    HIP_OK(hipEventRecord(ev_rank, s));
    // basis change T = U^^T U (the column side uses S = T^T); row counts
    // r_new written on the device before the launches read them
    PhaseScope post(hc, HP_COMPRESS_POST);
    Stage st;
    std::vector<int> tq(nt), rbound(nt);
    for (int t = 0; t < nt; ++t) {
      tq[t] = touch[t].q;
      rbound[t] = std::min(L.n[tq[t]], r_cap);
    }
    std::vector<GemmDesc> g;
    for (int t = 0; t < nt; ++t) {
      const int q = touch[t].q, nq = L.n[q];
      g.push_back({Uh + (size_t)t * L.sU, L.Ub(q), Tt + (size_t)t * rpad * rpad, rbound[t], L.r[q], nq, L.npad,
                   L.npad, rpad, 1, 0, 1.0, 0.0});
    }
    RankFin fin{};
    fin.rank = d_rank;
    fin.q = st.arr(&tq);
    fin.n = st.arr(&L.n);
    fin.r_new = const_cast<int*>(st.arr(&rbound));
    fin.nt = nt;
    fin.r_cap = r_cap;
    const int* rk_blob = st.arr(&L.r);  // the level's ranks, touched entries patched on the device
    fin.r_lvl = const_cast<int*>(rk_blob);
    // descriptor array pushed first, its op queued after the finalize op
    {
      const size_t goff = st.push(g.data(), g.size() * sizeof(GemmDesc));
      fin.g = reinterpret_cast<GemmDesc*>(goff + 1);
      st.rank_finalize(fin);
      int mm = 0, nn = 0;
      for (const auto& d : g) {
        mm = std::max(mm, d.M);
        nn = std::max(nn, d.N);
      }
      Op o{OP_GEMM, goff, 0, (int)g.size(), mm, nn, 0.0, 0.0};
      o.off2 = 0;  // opA = 1
      st.op(o, g[0].ty);
    }
    TouchXform txa{};
    {
      TouchXform a{};
      a.M = L.M;
      a.UP = k > 2 ? L.UP : nullptr;
      a.Tm = Tt;
      a.nt = nt;
      a.nside = L.nside;
      a.rpad = rpad;
      a.col_blocks = 1;
      a.sM = L.sM;
      // the new bases replace U inside the same launch (after the product
      // T = U^^T U above has read the old ones)
      a.Unew = Uh;
      a.U = L.U;
      a.n = fin.n;
      a.sU = L.sU;
      a.npad = L.npad;
      st.touch_xform<T>(a, &tq, &tidx, L.r, rbound, k > 2 ? &lv[k - 1].r : nullptr, L.nc, false, fin.r_new);
      txa = a;
    }
    // project the compressed fill into M2L (steps 4, 5 of the records)
    {
      ElimArgs a = elim_args(L, X, F, wpad, fpad, (int)E.size());
      a.tmp = wsS2.need<T>((size_t)E.size() * kPairs.count * rpad * fpad, s);
      a.rk = rk_blob;
      const size_t ro = st.push(erec[k][c].data(), erec[k][c].size() * sizeof(ElimRec)) + 1;
      int mx = rpad;
      for (const Elim& e : E)
        for (int sa = 0; sa < 9; ++sa)
          for (int sb = 0; sb < 9; ++sb) {
            const UnitH& ua = e.u[sa];
            const UnitH& ub = e.u[sb];
            if (kPairs.idx[sa][sb] < 0 || !ua.kind || !ub.kind || (ua.kind == 2 && ub.kind == 2)) continue;
            mx = std::max(mx, std::max(ua.size, ub.size));
          }
      st.elim<T>(a, ro, 4, mx, mx, 0.0, 0.0);
      st.elim<T>(a, ro, 5, mx, mx, 0.0, 0.0);
    }
    run(st);
    // the deferred work counts while the device runs the compression (after
    // every launch of it is queued), then the host's copy of the ranks and
    // the work counts that depend on them
    run_deferred();
    {
      PhaseScope w(hc, HP_WAIT);
      HIP_OK(hipEventSynchronize(ev_rank));
    }
    const double es = sizeof(T);
    double gf = 0, gb = 0, ucb = 0;
    for (int t = 0; t < nt; ++t) {
      const int q = tq[t], nq = L.n[q];
      rnew[t] = std::min(std::min(h_rank[2 * t], nq), r_cap);
      if (rnew[t] == r_cap && nq > r_cap) ++cap_hits[k];
      // Q of the pivoted steps, formed on the device
      const int kk = std::min(rnew[t], h_rank[2 * t + 1]);
      add_count(in_regs[t] ? 4 : 5, 4.0 * tri_sum(nq, rnew[t], kk), es * ((double)nq * kk + (double)nq * rnew[t]));
      // T = U^^T U (r_new x r_old, inner n_q)
      gf += 2.0 * rnew[t] * (double)L.r[q] * nq;
      gb += es * ((double)rnew[t] * nq + (double)nq * L.r[q] + (double)rnew[t] * L.r[q]);
      ucb += 2.0 * es * nq * (double)rnew[t];
    }
    add_count(0, gf, gb);
    add_count(9, 0.0, ucb);
    count_later(OP_TXFORM, [a = txa, tq, tidx, ro = L.r, rnew, rp = k > 2 ? lv[k - 1].r : std::vector<int>(),
                            par = k > 2, ncl = L.nc] {
      return txform_work(a, &tq, &tidx, ro, rnew, par ? &rp : nullptr, ncl, sizeof(T));
    });
    for (int t = 0; t < nt; ++t) L.r[tq[t]] = rnew[t];
    {
      count_later_family(12, [E, r = L.r] {
        double f = 0, by = 0;
        const double es = sizeof(T);
        for (const Elim& e : E)
          for (int sa = 0; sa < 9; ++sa)
            for (int sb = 0; sb < 9; ++sb) {
              if (kPairs.idx[sa][sb] < 0) continue;
              const UnitH& ua = e.u[sa];
              const UnitH& ub = e.u[sb];
              if (!ua.kind || !ub.kind || (ua.kind == 2 && ub.kind == 2)) continue;
              const double ra = ua.kind == 1 ? r[ua.cl] : ua.size, rb = ub.kind == 1 ? r[ub.cl] : ub.size;
              if (ua.kind == 1 && ub.kind == 1) {
                f += 2.0 * ra * ub.size * ua.size + 2.0 * ra * rb * ub.size;
                by += es * (ua.size * ra + (double)ua.size * ub.size + ra * ub.size) +
                      es * (ra * ub.size + (double)ub.size * rb + 2.0 * ra * rb);
              } else {
                f += 2.0 * ra * rb * (ua.kind == 1 ? ua.size : ub.size);
                by += es * ((double)ua.size * ub.size + (ua.kind == 1 ? ua.size * ra : ub.size * rb) + 2.0 * ra * rb);
              }
            }
        return std::make_pair(f, by);
      });
    }
  }

  // Level k -> k-1: particles are the children's multipoles; P2P from their
  // M2L; parent bases re-orthonormalised (z_P -> Ru z_P, y_P = Rv^T y^_P).
  void transition(int k) {
    PhaseScope ps_(hc, HP_TRANSITION);
    Level<T>& C = lv[k];
    Level<T>& L = lv[k - 1];
    int nm = 0;
    std::vector<int> rold(L.r);
    for (int P = 0; P < L.nc; ++P) {
      int o = 0;
      for (int c = 0; c < 4; ++c) {
        L.choff[(size_t)P * 4 + c] = o;
        o += C.r[4 * P + c];
      }
      L.n[P] = o;
      nm = std::max(nm, o);
    }
    L.set_pads(rup(std::max(nm, 1), 8));
    L.P = dalloc<T>(s, L.sP * 9 * L.nc);
    L.Qm = dalloc<T>(s, L.sQ * 9 * L.nc);
    L.L = dalloc<T>(s, L.sL * 9 * L.nc);
    L.U = dalloc<T>(s, L.sU * L.nc);
    L.Dinv = dalloc<double>(s, L.sD * L.nc);
    HIP_OK(hipMemsetAsync(L.Qm, 0, sizeof(T) * L.sQ * 9 * L.nc, s));
    HIP_OK(hipMemsetAsync(L.L, 0, sizeof(T) * L.sL * 9 * L.nc, s));
    T* Ru = wsA.need<T>((size_t)L.nc * rpad * rpad, s);
    auto Rub = [&](int P) { return Ru + (size_t)P * rpad * rpad; };
    Stage st;
    {
      TransArgs a{};
      a.CM = C.M;
      a.CUP = C.UP;
      a.P = L.P;
      a.U = L.U;
      a.sM = C.sM;
      a.sP = L.sP;
      a.sU = L.sU;
      a.npad = L.npad;
      a.rpad = rpad;
      a.nside = L.nside;
      a.nc = L.nc;
      double by = 0;
      for (int P = 0; P < L.nc; ++P) {
        if (L.n[P] == 0) continue;
        for (int sp = 0; sp < 9; ++sp) {
          const int Q = L.nbr9[(size_t)P * 9 + sp];
          if (Q >= 0) by += 2.0 * sizeof(T) * (double)L.n[P] * L.n[Q];
        }
        by += 2.0 * sizeof(T) * (double)L.n[P] * rold[P];
      }
      st.transition<T>(a, L.choff, C.r, rold, by);
    }
    std::vector<QrDesc> q;
    std::vector<AddDesc> z;
    for (int P = 0; P < L.nc; ++P) {
      if (L.n[P] > 0) q.push_back({L.Ub(P), Rub(P), L.n[P], rold[P], L.npad, rpad});
      L.r[P] = std::min(L.n[P], rold[P]);
    }
    st.qr(q);
    {
      TouchXform a{};
      a.M = L.M;
      a.UP = k - 1 > 2 ? L.UP : nullptr;
      a.Tm = Ru;
      a.nt = L.nc;
      a.nside = L.nside;
      a.rpad = rpad;
      a.col_blocks = 0;
      a.sM = L.sM;
      st.touch_xform<T>(a, nullptr, nullptr, rold, L.r, k - 1 > 2 ? &lv[k - 2].r : nullptr, L.nc, false);
      count_later(OP_TXFORM, [a, rold, rn = L.r, rp = k - 1 > 2 ? lv[k - 2].r : std::vector<int>(),
                              par = k - 1 > 2, ncl = L.nc] {
        return txform_work(a, nullptr, nullptr, rold, rn, par ? &rp : nullptr, ncl, sizeof(T));
      });
    }
    run(st);
    C.free_work(s);
  }

  void top() {
    PhaseScope ps_(hc, HP_TOP);
    Level<T>& L = lv[2];
    top_ids.clear();
    top_off.assign(1, 0);
    for (int c = 0; c < 16; ++c)
      if (L.r[c] > 0) {
        top_ids.push_back(c);
        top_off.push_back(top_off.back() + L.r[c]);
      }
    top_m = top_off.back();
    if (top_m == 0) return;
    d_top = dalloc<double>(s, (size_t)top_m * top_m);
    Stage st;
    std::vector<AddDesc> a;
    for (size_t x = 0; x < top_ids.size(); ++x)
      for (size_t y = 0; y < top_ids.size(); ++y) {
        const int ca = top_ids[x], cb = top_ids[y];
        a.push_back({L.Mb(ca, slot36(ca, cb)), d_top + top_off[x] + (size_t)top_off[y] * top_m, L.r[ca], L.r[cb], rpad,
                     top_m, 0, 1.0, 0.0});
      }
    st.add(a);
    plan_inverse(st, {InvDesc{d_top, top_m, top_m}});
    run(st);
    L.free_work(s);
  }

  // ------------------------------------------------------------------ solve
  struct SolveBufs {
    std::vector<double*> b, c, sn, x, y;
  };
  // Plans of Algorithm 2 already uploaded, keyed by their vectors (the
  // refinement alternates two): a repeated solve launches them as they are.
  // The launches of one solve sweep for nrhs columns (every level, colour
  // and step, the level transitions and the top solve) on the workspace at
  // base; the right-hand side and the solution enter and leave through the
  // leaf blocks, so one plan serves every vector pair.
  struct SolvePlan {
    double* base;
    int nrhs;
    size_t tot, bleaf, xleaf;  // zeroed length; leaf b and x blocks (offsets)
    Stage st;
    char* d = nullptr;
  };
  std::vector<SolvePlan> splans;

  // x (tree order, ld N) = A^-1 b (tree order, ld N)
  SolvePlan& solve_plan(int nrhs) {
    PhaseScope ps_(hc, HP_SOLVE_PLAN);
    std::vector<size_t> ob(kappa + 1), oc(kappa + 1);
    size_t tot = 0;
    for (int k = 2; k <= kappa; ++k) {
      const Level<T>& L = lv[k];
      ob[k] = tot;
      tot += (size_t)3 * L.nc * L.npad * nrhs;
      oc[k] = tot;
      tot += (size_t)2 * L.nc * rpad * nrhs;
    }
    size_t wsz = 0;
    for (int k = 2; k <= kappa; ++k)
      for (int c = 0; c < 9; ++c) wsz = std::max(wsz, plan[k][c].size() * lv[k].mpad);
    double* base = wsS1.need<double>(tot + 2 * (size_t)std::max(top_m, 1) * nrhs + wsz * nrhs, s);
    double* tv = base + tot;
    double* wk = tv + 2 * (size_t)std::max(top_m, 1) * nrhs;
    auto bvec = [&](int k, int i) { return base + ob[k] + (size_t)i * lv[k].npad * nrhs; };
    auto xvec = [&](int k, int i) { return base + ob[k] + ((size_t)2 * lv[k].nc + i) * lv[k].npad * nrhs; };
    auto cvec = [&](int k, int i) { return base + oc[k] + (size_t)i * rpad * nrhs; };
    auto yvec = [&](int k, int i) { return base + oc[k] + ((size_t)lv[k].nc + i) * rpad * nrhs; };
    for (SolvePlan& sp : splans)
      if (sp.base == base && sp.nrhs == nrhs) return sp;
    auto args = [&](int k, int c) {
      const Level<T>& L = lv[k];
      SolveArgs a{};
      a.rec = d_erec + erec_off[k][c];
      a.P = L.P;
      a.Qm = L.Qm;
      a.L = L.L;
      a.Dinv = L.Dinv;
      a.bv = base + ob[k];
      a.cv = base + oc[k];
      a.sP = L.sP;
      a.sQ = L.sQ;
      a.sL = L.sL;
      a.sD = L.sD;
      a.nb = (int)plan[k][c].size();
      a.nc = L.nc;
      a.npad = L.npad;
      a.rpad = rpad;
      a.mpad = L.mpad;
      a.nrhs = nrhs;
      return a;
    };
    // algorithmic work of one step: every block it reads once, vectors read
    // and written once (counted for the profile only); max_rows: largest row
    // count of the step
    auto work = [&](int k, int c, int step, double& f, double& by, int& rows) {
      f = by = 0;
      rows = 0;
      if (!(profile && timed(family(OP_SOLVE)))) {
        for (const Elim& e : plan[k][c]) {
          if (step == 0 || step == 3) {
            rows = std::max(rows, step == 0 ? e.m : e.ni);
            continue;
          }
          rows = std::max(rows, step == 1 ? e.ri : e.m);
          if (step == 1)
            for (int sp = 0; sp < 9; ++sp)
              if (sp != 4 && e.u[sp].kind) rows = std::max(rows, e.u[sp].size);
        }
        return;
      }
      for (const Elim& e : plan[k][c]) {
        if (step == 0 || step == 3) {
          const double kk = step == 0 ? e.ni : e.m, rr = step == 0 ? e.m : e.ni;
          f += 2.0 * rr * kk * nrhs;
          by += 8.0 * rr * kk + 8.0 * nrhs * (kk + rr);
          rows = std::max(rows, (int)rr);
          continue;
        }
        rows = std::max(rows, step == 1 ? e.ri : e.m);
        for (int sp = 0; sp < 9; ++sp)
          if (sp != 4 && e.u[sp].kind) {
            f += 2.0 * e.u[sp].size * e.ni * nrhs;
            by += sizeof(T) * (double)e.u[sp].size * e.ni + 8.0 * nrhs * (e.u[sp].size + e.ni);
            if (step == 1) rows = std::max(rows, e.u[sp].size);
          }
      }
    };
    Stage st;
    for (int k = kappa; k >= 2; --k) {
      const Level<T>& L = lv[k];
      for (int c = 0; c < 9; ++c) {
        if (plan[k][c].empty()) continue;
        for (int step = 0; step < 2; ++step) {
          double f, by;
          int rows;
          work(k, c, step, f, by, rows);
          st.solve<T>(args(k, c), step, wk, rows, f, by);
        }
      }
      if (k > 2) {  // children's c into the parents' b at the children's offsets
        const Level<T>& Lp = lv[k - 1];
        std::vector<int> start(L.nc);
        for (int ch = 0; ch < L.nc; ++ch) start[ch] = (ch >> 2) * Lp.npad * nrhs + Lp.choff[ch];
        st.row_copy({bvec(k - 1, 0), cvec(k, 0), nullptr, nullptr, (size_t)rpad * nrhs, Lp.npad, rpad, L.nc, nrhs, 0},
                    start, L.r);
      }
    }
    if (top_m > 0) {
      std::vector<AddDesc> a, a2;
      for (size_t x = 0; x < top_ids.size(); ++x)
        a.push_back({cvec(2, top_ids[x]), tv + top_off[x], lv[2].r[top_ids[x]], nrhs, rpad, top_m, 0, 1.0, 0.0});
      st.add(a);
      double* yt = tv + (size_t)top_m * nrhs;
      st.gemm({GemmDesc{d_top, tv, yt, top_m, nrhs, top_m, top_m, top_m, top_m, 0, 0, 1.0, 0.0}});
      for (size_t x = 0; x < top_ids.size(); ++x)
        a2.push_back({yt + top_off[x], yvec(2, top_ids[x]), lv[2].r[top_ids[x]], nrhs, top_m, rpad, 0, 1.0, 0.0});
      st.add(a2);
    }
    for (int k = 2; k <= kappa; ++k) {
      const Level<T>& L = lv[k];
      for (int c = 8; c >= 0; --c) {
        if (plan[k][c].empty()) continue;
        for (int step = 2; step < 4; ++step) {
          double f, by;
          int rows;
          work(k, c, step, f, by, rows);
          st.solve<T>(args(k, c), step, wk, rows, f, by);
        }
      }
      if (k < kappa) {  // the parents' x at the children's offsets into the children's y
        const Level<T>& Lc = lv[k + 1];
        std::vector<int> start(Lc.nc);
        for (int ch = 0; ch < Lc.nc; ++ch) start[ch] = (ch >> 2) * L.npad * nrhs + L.choff[ch];
        st.row_copy({xvec(k, 0), yvec(k + 1, 0), nullptr, nullptr, (size_t)rpad * nrhs, L.npad, rpad, Lc.nc, nrhs, 1},
                    start, Lc.r);
      }
    }
    st.flops = 0.0;  // solve work is not factorisation work
    if (splans.size() >= 4) {
      dfree(s, splans.front().d);
      splans.erase(splans.begin());
    }
    splans.push_back(SolvePlan{base, nrhs, tot, (size_t)(bvec(kappa, 0) - base), (size_t)(xvec(kappa, 0) - base),
                               std::move(st), nullptr});
    SolvePlan& sp = splans.back();
    sp.d = dalloc<char>(s, sp.st.blob.size());
    upload_pinned(sp.d, sp.st.blob, sp.st.blob.size());
    return sp;
  }

  // One sweep: x = A_f^-1 b (tree order, ld N).
  void solve_tree(const double* bt, double* xt, int nrhs) {
    SolvePlan& sp = solve_plan(nrhs);
    const Level<T>& Lf = lv[kappa];
    const size_t bs = (size_t)Lf.npad * nrhs;
    HIP_OK(hipMemsetAsync(sp.base, 0, sizeof(double) * sp.tot, s));
    launch_leaf_gather(bt, (int)N, sp.base + sp.bleaf, bs, Lf.npad, d_leaf_start, d_leaf_n, Lf.nc, nrhs, s);
    launch_ops(sp.st, sp.d);
    launch_leaf_scatter(sp.base + sp.xleaf, bs, Lf.npad, xt, (int)N, d_leaf_start, d_leaf_n, Lf.nc, nrhs, s);
    HIP_OK(hipGetLastError());
  }

  // ---------------------------------------------------------- entry points
  void build(const double* points) override {
    const char* tr = std::getenv("IFMM_TRACE_HOST");
    hc.on = tr && tr[0] && tr[0] != '0';
    arena.init();
    for (hipEvent_t& e : ev_t) HIP_OK(hipEventCreate(&e));
    HIP_OK(hipEventCreateWithFlags(&ev_rank, hipEventDisableTiming));
    HIP_OK(hipEventRecord(ev_t[0], s));
    assemble(points);
    HIP_OK(hipEventRecord(ev_t[1], s));
    factor();
    HIP_OK(hipEventRecord(ev_t[2], s));
    HIP_OK(hipStreamSynchronize(s));
    arena.settle();
    up_E = Blob();
    up_nbr9 = Blob();
    up_near_off = Blob();
    // stream-timeline times: assembly ends when its last kernel does (the
    // host plans the factorisation meanwhile)
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, ev_t[0], ev_t[1]));
    t_assembly = ms;
    HIP_OK(hipEventElapsedTime(&ms, ev_t[1], ev_t[2]));
    t_factor = ms;
    hc.print(N);
  }

  void matvec(const double* x, double* y, int nrhs) override {
    const int n = (int)N;
    double* buf = wsS2.need<double>((size_t)2 * n * nrhs, s);
    launch_gather_rows(x, n, d_perm, n, nrhs, buf, n, s);
    fmm_apply_tree(buf, buf + (size_t)n * nrhs, nrhs, d_diag);
    launch_scatter_rows(buf + (size_t)n * nrhs, n, d_perm, n, nrhs, y, n, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
  }

  size_t matvec_scratch_bytes(int nrhs) const override {
    return sizeof(double) * (2 * (size_t)N * nrhs + fmm_coeff_count(nrhs));
  }

  // The product with every intermediate in ws (matvec_scratch_bytes): the
  // tree-order x and y, then the coefficients.  Enqueued only (no wait).
  void matvec_into(const double* x, double* y, int nrhs, double* ws) override {
    const int n = (int)N;
    double* xt = ws;
    double* yt = ws + (size_t)n * nrhs;
    launch_gather_rows(x, n, d_perm, n, nrhs, xt, n, s);
    fmm_apply_tree(xt, yt, nrhs, d_diag, yt + (size_t)n * nrhs);
    launch_scatter_rows(yt, n, d_perm, n, nrhs, y, n, s);
    HIP_OK(hipGetLastError());
  }

  // y = A_k x for another kernel kk on this tree and these bases, with its
  // own diagonal rule (dmode / c0k / dvec as in ifmm_kernel).
  void matvec_kernel(const KernelFn& kk, int dmode, double c0k, const double* dvec, const double* x, double* y,
                     int nrhs) override {
    const int n = (int)N;
    const size_t tsz = (size_t)49 * p2 * p2;
    double* tb = wsTab.need<double>((size_t)(kappa + 1) * tsz, s);
    double* tab[kMaxLevels + 1] = {};
    for (int k = 2; k <= kappa; ++k) {
      tab[k] = tb + (size_t)k * tsz;
      launch_m2l_table(kk, p, 0.5 * size / (1 << k), tab[k], s);
    }
    double* buf = wsS2.need<double>((size_t)2 * n * nrhs + n, s);
    double* xt = buf;
    double* yt = buf + (size_t)n * nrhs;
    double* dg = buf + (size_t)2 * n * nrhs;
    if (dmode == IFMM_DIAG_ROWSUM) {  // c0 + the row sums of the off-diagonal part
      launch_fill(xt, n, 1.0, s);
      fmm_apply_tree(xt, dg, 1, nullptr, nullptr, tab, &kk);
      launch_add_const(dg, n, c0k, s);
    } else if (dmode == IFMM_DIAG_VECTOR) {
      launch_gather_rows(dvec, n, d_perm, n, 1, dg, n, s);
    } else {
      launch_fill(dg, n, c0k, s);
    }
    launch_gather_rows(x, n, d_perm, n, nrhs, xt, n, s);
    fmm_apply_tree(xt, yt, nrhs, dg, nullptr, tab, &kk);
    launch_scatter_rows(yt, n, d_perm, n, nrhs, y, n, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
  }

  void diagonal(double* d) override {
    launch_scatter_rows(d_diag, (int)N, d_perm, (int)N, 1, d, (int)N, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
  }

  // Algorithm 2, then FP64 iterative refinement against the FMM product:
  // x += A_f^-1 (b - A x) until every column meets refine_tol.
  ifmm_status solve(const double* b, double* x, int nrhs, ifmm_solve_info* info) override {
    ifmm_status result = IFMM_OK;
    const double t0 = now_ms();
    const int n = (int)N;
    const size_t sz = (size_t)n * nrhs;
    // tree-order vectors: b, x, r, dx, y, best x
    double* base = wsB.need<double>(6 * sz + 2 * (size_t)nrhs, s);
    double* bt = base;
    double* xt = base + sz;
    double* rt = base + 2 * sz;
    double* dx = base + 3 * sz;
    double* yt = base + 4 * sz;
    double* xbest = base + 5 * sz;
    double* nrm = base + 6 * sz;
    launch_gather_rows(b, n, d_perm, n, nrhs, bt, n, s);
    solve_tree(bt, xt, nrhs);
    int it = 0;
    std::vector<double> hist;
    const double* xout = xt;
    if (refine_tol > 0.0) {
      std::vector<double> bn(nrhs), rn(nrhs);
      HIP_OK(hipMemsetAsync(nrm, 0, sizeof(double) * nrhs, s));
      launch_colnorm2(bt, n, nrhs, n, nrm, s);
      to_host(nrm, sizeof(double) * nrhs, bn.data());
      double best = 1e300;
      while (true) {
        fmm_apply_tree(xt, yt, nrhs, d_diag);
        Stage st;
        st.add({AddDesc{bt, rt, n, nrhs, n, n, 0, 1.0, 0.0}});
        st.add({AddDesc{yt, rt, n, nrhs, n, n, 0, -1.0, 1.0}});
        run(st);
        HIP_OK(hipMemsetAsync(nrm, 0, sizeof(double) * nrhs, s));
        launch_colnorm2(rt, n, nrhs, n, nrm, s);
        to_host(nrm, sizeof(double) * nrhs, rn.data());
        double worst = 0.0;
        for (int r = 0; r < nrhs; ++r) {
          const double rel = std::sqrt(rn[r]) / std::max(std::sqrt(bn[r]), 1e-300);
          worst = std::isfinite(rel) ? std::max(worst, rel) : HUGE_VAL;  // a NaN column is not converged
        }
        hist.push_back(worst);
        if (worst <= refine_tol) {
          xout = xt;
          break;
        }
        if (worst == HUGE_VAL) {  // non-finite residual: stop with the best finite iterate (else x as is)
          result = IFMM_ENOTCONV;
          xout = best < 1e300 ? xbest : xt;
          break;
        }
        if (worst < best) {  // keep the best iterate for a non-converged return
          best = worst;
          Stage sb;
          sb.add({AddDesc{xt, xbest, n, nrhs, n, n, 0, 1.0, 0.0}});
          run(sb);
        }
        if (it >= refine_maxit || (hist.size() >= 3 && worst > 0.9 * hist[hist.size() - 2] && worst > hist[0])) {
          result = IFMM_ENOTCONV;
          xout = xbest;
          break;
        }
        solve_tree(rt, dx, nrhs);
        Stage s2;
        s2.add({AddDesc{dx, xt, n, nrhs, n, n, 0, 1.0, 1.0}});
        run(s2);
        ++it;
      }
    }
    launch_scatter_rows(xout, n, d_perm, n, nrhs, x, n, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    arena.settle();
    t_solve = now_ms() - t0;
    resolve_profile();
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->iterations = it;
      info->residual = hist.empty() ? 0.0 : (result == IFMM_OK ? hist.back() : *std::min_element(hist.begin(), hist.end()));
      for (size_t i = 0; i < hist.size() && i < 32; ++i) info->history[i] = hist[i];
      info->solve_ms = t_solve;
    }
    return result;
  }

  void stats(ifmm_stats_t* st) override {
    std::memset(st, 0, sizeof(*st));
    st->n = N;
    st->kappa = kappa;
    st->p = p;
    st->max_rank = max_rank;
    double bytes = 0;
    for (int k = 2; k <= kappa && k < 16; ++k) {
      const Level<T>& L = lv[k];
      int mx = 0;
      double sum = 0;
      int cnt = 0;
      for (int i = 0; i < L.nc; ++i)
        if (L.n[i] > 0) {
          mx = std::max(mx, L.r[i]);
          sum += L.r[i];
          ++cnt;
        }
      st->level_max_rank[k] = mx;
      st->level_mean_rank[k] = cnt ? sum / cnt : 0.0;
      st->level_cap_hits[k] = cap_hits[k];
      bytes += (double)L.nc * (sizeof(T) * 9.0 * (L.sP + L.sQ + L.sL) + sizeof(double) * L.sD);
    }
    st->top_size = top_m;
    st->assembly_ms = t_assembly;
    st->factor_ms = t_factor;
    st->last_solve_ms = t_solve;
    st->factor_bytes = bytes;
    st->factor_flops = factor_flops;
    st->precision = kF32 ? IFMM_FP32 : IFMM_FP64;
    for (int t = 0; t < 2 * kOpTypes; ++t) {
      st->kernel_launches[t] = prof_launch[t];
      st->kernel_ms[t] = prof_ms[t];
      st->kernel_flops[t] = prof_flops[t];
      st->kernel_bytes[t] = prof_bytes[t];
    }
  }

  int ranks(int level, int* out, int count) override {
    if (level < 2 || level > kappa) return IFMM_EINVAL;
    const Level<T>& L = lv[level];
    if (count < L.nc) return IFMM_EINVAL;
    for (int i = 0; i < L.nc; ++i) out[i] = L.r[i];
    return IFMM_OK;
  }

  void release() override {
    for (auto& L : lv) L.free_all(s);
    for (auto& t : d_table) dfree(s, t);
    dfree(s, d_near);
    dfree(s, d_near_off);
    dfree(s, d_pts);
    dfree(s, d_perm);
    dfree(s, d_leaf_start);
    dfree(s, d_leaf_n);
    dfree(s, d_nbr9_leaf);
    dfree(s, d_diag);
    dfree(s, d_E);
    dfree(s, d_top);
    dfree(s, d_erec);
    for (SolvePlan& sp : splans) dfree(s, sp.d);
    splans.clear();
    dfree(s, d_status);
    dfree(s, d_rank);
    for (Buf* b : {&wsX, &wsF, &wsT, &wsA, &wsB, &wsQ, &wsR, &wsZ, &wsS1, &wsS2, &wsVec, &wsInvT, &wsInvP,
                   &wsSeg, &wsTab})
      b->release(s);
    arena.release(s);
    for (const Pending& p : pend) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    pend.clear();
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
    evpool.clear();
    for (hipEvent_t& e : ev_t) {
      if (e) (void)hipEventDestroy(e);
      e = nullptr;
    }
    if (ev_rank) (void)hipEventDestroy(ev_rank);
    ev_rank = nullptr;
    pinned().put(reinterpret_cast<char*>(h_rank), h_rank_bytes);
    h_rank = nullptr;
    h_rank_dev = nullptr;
    h_rank_bytes = 0;
    pinned().put(h_small, h_small_bytes);
    h_small = nullptr;
    h_small_bytes = 0;
  }
};

// ------------------------------------------------ fixed device workspace
// The workspace of ifmm_matvec_noalloc: one copy per device, held by the
// process from the library's first use of the device until it ends.  Its
// device address is looked up once per device (hipGetSymbolAddress); host
// code only ever passes that address on, never the array's own name.
constexpr size_t kScratchBytes = (size_t)64 << 20;
std::mutex scratch_mu;
void* scratch_addr[64] = {};

}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

// Device address of the current device's workspace (resolved on first use).
hipError_t scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_addr[dev] = p;
  }
  *out = scratch_addr[dev];
  return hipSuccess;
}

ifmm_status map_exc() {
  try {
    throw;
  } catch (const HipError& h) {
    // a HIP runtime error has no other way out through the status codes:
    // name it on stderr (the call's line in this file and the runtime's text)
    std::fprintf(stderr, "ifmm: HIP error %d (%s) at ifmm_host.hip:%d\n", (int)h.e, hipGetErrorString(h.e), h.line);
    return IFMM_EDEVICE;
  } catch (const NoMem&) {
    return IFMM_ENOMEM;
  } catch (const BadArg&) {
    return IFMM_EINVAL;
  } catch (const Broken& b) {
    std::fprintf(stderr, "ifmm: internal check failed at ifmm_host.hip:%d: %s\n", b.line, b.what);
    return IFMM_EDEVICE;
  } catch (int code) {
    return (ifmm_status)code;
  } catch (const std::bad_alloc&) {
    return IFMM_ENOMEM;
  } catch (...) {
    return IFMM_EDEVICE;
  }
}

}  // namespace

namespace {
// Runs job(i, stream) for i = 0 .. count-1 on `threads` host threads, each
// with its own non-blocking HIP stream (default priority), problems taken
// in order from a shared counter.  Every job ends with its stream
// synchronised (ifmm_factor / ifmm_solve do), so the handles it touched are
// handed back on `caller` once the worker is done with them.
// Worker stream `idx` of device `dev`, created on first use and kept until
// the process ends: block releases and descriptor uploads record events on
// the stream a call ran on, and later calls may wait on those events; an
// event must not outlive the stream it was last recorded on.
hipError_t worker_stream(int dev, int idx, hipStream_t* out) {
  static std::mutex mu;
  static std::unordered_map<int, std::vector<hipStream_t>>* all =
      new std::unordered_map<int, std::vector<hipStream_t>>();  // never destroyed
  std::lock_guard<std::mutex> lk(mu);
  std::vector<hipStream_t>& v = (*all)[dev];
  while ((int)v.size() <= idx) {
    hipStream_t st = nullptr;
    const hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    v.push_back(st);
  }
  *out = v[idx];
  return hipSuccess;
}

// Runs job(i, stream) for i = 0 .. count-1 on `threads` host threads, each
// on a worker stream of its own (non-blocking, default priority), problems
// taken in order from a shared counter.  Every job ends with its stream
// synchronised (ifmm_factor / ifmm_solve do), so the handles it touched can
// be handed back to the caller's stream.
template <class Job>
ifmm_status run_batched(int count, int threads, Job job) {
  if (threads <= 0) threads = 4;
  threads = std::min(std::min(threads, count), 64);
  std::atomic<int> next{0};
  std::atomic<int> dev_err{0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return IFMM_EDEVICE;
  auto worker = [&](int t) {
    hipStream_t st = nullptr;
    hipError_t e = hipSetDevice(dev);
    if (e == hipSuccess) e = worker_stream(dev, t, &st);
    if (e != hipSuccess) {
      std::fprintf(stderr, "ifmm: batched worker %d: HIP error %d (%s)\n", t, (int)e, hipGetErrorString(e));
      dev_err = 1;
      return;
    }
    for (int i = next.fetch_add(1); i < count; i = next.fetch_add(1)) job(i, st);
  };
  std::vector<std::thread> pool;
  try {
    for (int t = 1; t < threads; ++t) pool.emplace_back(worker, t);
  } catch (...) {
    // fewer threads: the ones started and this one take every problem
  }
  worker(0);
  for (auto& t : pool) t.join();
  return dev_err ? IFMM_EDEVICE : IFMM_OK;
}
}  // namespace

extern "C" {

namespace {
// The kernel description is usable: known kind and diagonal rule, valid parameters.
bool kernel_ok(const ifmm_kernel* k) {
  if (k->kind < IFMM_K_INV_R || k->kind > IFMM_K_EXP_DELL) return false;
  if (k->kind != IFMM_K_INV_R && !(k->ell > 0.0 && std::isfinite(k->ell))) return false;
  if ((k->kind == IFMM_K_LOG_A || k->kind == IFMM_K_R2LOG_A) && k->ell == 1.0) return false;
  if (k->diag_mode != IFMM_DIAG_ROWSUM && k->diag_mode != IFMM_DIAG_CONST && k->diag_mode != IFMM_DIAG_VECTOR)
    return false;
  if (k->diag_mode == IFMM_DIAG_VECTOR && !k->diag) return false;
  if (k->diag_mode != IFMM_DIAG_VECTOR && !std::isfinite(k->c0)) return false;
  return true;
}
}  // namespace

ifmm_status ifmm_factor(const double* points, int64_t n, const ifmm_kernel* k, double eps, int leaf_size,
                        int rank, const ifmm_options* opt, void* stream, ifmm_t* out) {
  if (!out || !points || !k) return IFMM_EINVAL;
  if (n < 16 || n > (int64_t)1 << 30 || leaf_size < 1 || !(eps >= 0.0) || !std::isfinite(eps)) return IFMM_EINVAL;
  int p = (int)std::lround(std::sqrt((double)rank));
  if (rank < 1 || p * p != rank || p > kMaxP) return IFMM_EINVAL;
  if (!kernel_ok(k)) return IFMM_EINVAL;
  // eps = 0 asks for lossless compression: only with an explicit rank cap
  // (ranks grow with every elimination; the default cap would truncate)
  if (eps == 0.0 && !(opt && opt->r_max > 0)) return IFMM_EINVAL;
  int r_cap = opt && opt->r_max > 0 ? opt->r_max : 2 * rank;
  if (r_cap > kMaxRank) r_cap = opt && opt->r_max > 0 ? -1 : kMaxRank;
  if (r_cap < rank || r_cap > kMaxRank) return IFMM_EINVAL;
  const int prec = opt ? opt->precision : IFMM_FP64;
  if (prec != IFMM_FP64 && prec != IFMM_FP32) return IFMM_EINVAL;
  ifmm_plan* h = nullptr;
  if (prec == IFMM_FP32) h = new (std::nothrow) Plan<float>();
  else h = new (std::nothrow) Plan<double>();
  if (!h) return IFMM_ENOMEM;
  h->s = static_cast<hipStream_t>(stream);
  h->N = n;
  h->p = p;
  h->p2 = rank;
  h->leaf = leaf_size;
  h->r_cap = r_cap;
  h->rpad = rup(r_cap, 8);
  h->kf = KernelFn{k->kind, k->ell};
  h->diag_mode = k->diag_mode;
  h->d_diag_user = k->diag_mode == IFMM_DIAG_VECTOR ? k->diag : nullptr;
  h->c0 = k->diag_mode == IFMM_DIAG_VECTOR ? 0.0 : k->c0;
  h->eps = eps;
  if (opt && opt->box_size > 0.0) {
    h->lox = opt->box_lo[0];
    h->loy = opt->box_lo[1];
    h->size = opt->box_size;
  }
  if (opt) {
    h->profile = opt->profile;
    h->refine_tol = opt->refine_tol;
    h->refine_maxit = opt->refine_maxit > 0 ? opt->refine_maxit : 30;
  }
  try {
    h->build(points);
  } catch (...) {
    ifmm_status st = map_exc();
    (void)hipStreamSynchronize(h->s);
    h->release();
    delete h;
    return st;
  }
  *out = h;
  // set-up of the device's fixed workspace (ifmm_matvec_noalloc); a failure
  // here is reported by that entry point, not by the factorisation
  void* ws = nullptr;
  (void)scratch_ptr(&ws);
  return IFMM_OK;
}

ifmm_status ifmm_matvec(ifmm_t h, const double* x, double* y, int nrhs, void* stream) {
  if (!h || !x || !y || nrhs < 1 || nrhs > 64) return IFMM_EINVAL;
  try {
    h->s = static_cast<hipStream_t>(stream);
    h->matvec(x, y, nrhs);
  } catch (...) {
    return map_exc();
  }
  return IFMM_OK;
}


ifmm_status ifmm_factor_batched(int count, const double* const* points, const int64_t* n, const ifmm_kernel* kernels,
                                double eps, int leaf_size, int rank, const ifmm_options* opt, int threads,
                                void* stream, ifmm_t* out, ifmm_status* status) {
  if (count < 1 || !points || !n || !kernels || !out || !status) return IFMM_EINVAL;
  for (int i = 0; i < count; ++i) {
    out[i] = nullptr;
    status[i] = IFMM_EINVAL;
  }
  const hipStream_t caller = static_cast<hipStream_t>(stream);
  // the problems' inputs are the caller's: they are ready once its stream is
  if (hipStreamSynchronize(caller) != hipSuccess) return IFMM_EDEVICE;
  const ifmm_status r = run_batched(count, threads, [&](int i, hipStream_t st) {
    status[i] = ifmm_factor(points[i], n[i], &kernels[i], eps, leaf_size, rank, opt, st, &out[i]);
    if (status[i] == IFMM_OK) out[i]->s = caller;
  });
  if (r != IFMM_OK) return r;
  ifmm_status worst = IFMM_OK;
  for (int i = 0; i < count; ++i)
    if (status[i] != IFMM_OK) worst = status[i];
  return worst;
}

ifmm_status ifmm_solve_batched(int count, const ifmm_t* h, const double* const* b, double* const* x, int nrhs,
                               int threads, void* stream, ifmm_solve_info* info, ifmm_status* status) {
  if (count < 1 || !h || !b || !x || !status) return IFMM_EINVAL;
  for (int i = 0; i < count; ++i) status[i] = IFMM_EINVAL;
  const hipStream_t caller = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(caller) != hipSuccess) return IFMM_EDEVICE;
  const ifmm_status r = run_batched(count, threads, [&](int i, hipStream_t st) {
    status[i] = ifmm_solve(h[i], b[i], x[i], nrhs, st, info ? &info[i] : nullptr);
    if (h[i]) h[i]->s = caller;
  });
  if (r != IFMM_OK) return r;
  ifmm_status worst = IFMM_OK;
  for (int i = 0; i < count; ++i)
    if (status[i] != IFMM_OK) worst = status[i];
  return worst;
}

ifmm_status ifmm_matvec_kernel(ifmm_t h, const ifmm_kernel* k, const double* x, double* y, int nrhs,
                               void* stream) {
  if (!h || !k || !x || !y || nrhs < 1 || nrhs > 64 || !kernel_ok(k)) return IFMM_EINVAL;
  // 1/r is singular at equal points: only on a tree whose points were checked distinct
  if (k->kind == IFMM_K_INV_R && h->kf.kind != IFMM_K_INV_R) return IFMM_EINVAL;
  try {
    h->s = static_cast<hipStream_t>(stream);
    h->matvec_kernel(KernelFn{k->kind, k->ell}, k->diag_mode, k->c0, k->diag, x, y, nrhs);
  } catch (...) {
    return map_exc();
  }
  return IFMM_OK;
}

ifmm_status ifmm_matvec_noalloc(ifmm_t h, const double* x, double* y, int nrhs, void* stream) {
  if (!h || !x || !y || nrhs < 1 || nrhs > 64) return IFMM_EINVAL;
  if (h->matvec_scratch_bytes(nrhs) > kScratchBytes) return IFMM_ESIZE;
  void* ws = nullptr;
  if (scratch_ptr(&ws) != hipSuccess) return IFMM_EDEVICE;
  try {
    h->s = static_cast<hipStream_t>(stream);
    h->matvec_into(x, y, nrhs, static_cast<double*>(ws));
  } catch (...) {
    return map_exc();
  }
  return IFMM_OK;
}

size_t ifmm_matvec_noalloc_bytes(ifmm_t h, int nrhs) {
  if (!h || nrhs < 1) return 0;
  return h->matvec_scratch_bytes(nrhs);
}

ifmm_status ifmm_diagonal(ifmm_t h, double* d, void* stream) {
  if (!h || !d) return IFMM_EINVAL;
  try {
    h->s = static_cast<hipStream_t>(stream);
    h->diagonal(d);
  } catch (...) {
    return map_exc();
  }
  return IFMM_OK;
}

ifmm_status ifmm_solve(ifmm_t h, const double* b, double* x, int nrhs, void* stream, ifmm_solve_info* info) {
  if (!h || !b || !x || nrhs < 1 || nrhs > 64 || b == x) return IFMM_EINVAL;
  try {
    h->s = static_cast<hipStream_t>(stream);
    return h->solve(b, x, nrhs, info);
  } catch (...) {
    return map_exc();
  }
}

ifmm_status ifmm_stats(ifmm_t h, ifmm_stats_t* s) {
  if (!h || !s) return IFMM_EINVAL;
  h->stats(s);
  return IFMM_OK;
}

ifmm_status ifmm_ranks(ifmm_t h, int level, int* out, int count) {
  if (!h || !out) return IFMM_EINVAL;
  return (ifmm_status)h->ranks(level, out, count);
}

void ifmm_destroy(ifmm_t h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->s);
  h->release();
  delete h;
}

void ifmm_release_cached_memory(void) { pool().trim(-1); }

const char* ifmm_status_string(ifmm_status s) {
  switch (s) {
    case IFMM_OK: return "ok";
    case IFMM_EINVAL: return "invalid argument";
    case IFMM_ESIZE: return "problem exceeds the fixed device workspace";
    case IFMM_ENOMEM: return "out of memory";
    case IFMM_ESINGULAR: return "singular pivot block";
    case IFMM_ENOTCONV: return "refinement did not converge";
    case IFMM_EDEVICE: return "HIP device error";
  }
  return "unknown status";
}

}  // extern "C"
