// Host driver and C ABI of the space-time Sylvester solver.
//
// Galerkin projection (Sec. 4) onto an extended Krylov space in the operator
// A = Mx^{-1} Kx started from Mx^{-1} F1 (the rational Krylov space of Sec. 4
// with the poles 0 and infinity):
//   V_1     = orth_M([Mx^{-1} F1, Kx^{-1} F1])
//   V_{j+1} = orth_M([Mx^{-1} Kx V_j^+, Kx^{-1} Mx V_j^-])   against V_1..V_j
// (V_j^+ / V_j^- are the block's columns descended from the positive /
// negative powers).  Because Mx^{-1} F1 lies in the space and V is
// Mx-orthonormal, F1 = Mx V beta with beta = V^T F1, and the Arnoldi-type
// relation A V_m = V_{m+1} T gives the residual of the Galerkin solution in
// closed form: R = -(Mx V_new)(tau Y Mt^T) with tau = V_new^T Kx V_m, so
// ||R||_F = ||L^T tau Y Mt^T||_F where L L^T = (Mx V_new)^T (Mx V_new).  This
// projected residual is monitored; success is confirmed with the exact
// residual ||F1 F2^T - (Kx V) Y Mt^T - (Mx V) Y Dt^T||_F, evaluated without
// forming the Nh x Nt product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sts_internal.h"

namespace sts {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

thread_local Profiler* g_profiler = nullptr;

Profiler* active_profiler() { return g_profiler; }
void set_active_profiler(Profiler* p) { g_profiler = p; }

Profiler::~Profiler() {
  for (auto e : pool) (void)hipEventDestroy(e);
}

void Profiler::reset() {
  ids.clear();
  bytes.clear();
  collected = false;
}

void Profiler::next(int kid, double b, hipEvent_t* s, hipEvent_t* e) {
  const size_t i = ids.size();
  while (pool.size() < 2 * (i + 1)) {
    hipEvent_t ev;
    STS_HIP(hipEventCreate(&ev));
    pool.push_back(ev);
  }
  *s = pool[2 * i];
  *e = pool[2 * i + 1];
  ids.push_back(kid);
  bytes.push_back(b);
}

void Profiler::collect() {
  if (collected) return;
  for (int k = 0; k < STS_K_COUNT; ++k) {
    sec[k] = byt[k] = 0.0;
    cnt[k] = 0;
  }
  for (size_t i = 0; i < ids.size(); ++i) {
    STS_HIP(hipEventSynchronize(pool[2 * i + 1]));
    float ms = 0.0f;
    STS_HIP(hipEventElapsedTime(&ms, pool[2 * i], pool[2 * i + 1]));
    sec[ids[i]] += 1e-3 * ms;
    cnt[ids[i]] += 1;
    byt[ids[i]] += bytes[i];
  }
  collected = true;
}

// ---------------------------------------------------------------------------
// spatial operators
// ---------------------------------------------------------------------------

void validate_space(const sts_space* s) {
  STS_REQUIRE(s != nullptr, STS_E_INVALID, "space is NULL");
  STS_REQUIRE(s->kind == STS_FE_P1_1D || s->kind == STS_FE_P1_2D || s->kind == STS_FE_Q1_3D_7PT,
              STS_E_INVALID, "unsupported space kind");
  STS_REQUIRE(std::isfinite(s->mu) && s->mu > 0.0, STS_E_INVALID, "mu must be finite and > 0");
  const int dim = s->kind;
  for (int d = 0; d < 3; ++d) {
    if (d < dim) {
      STS_REQUIRE(s->n[d] >= 1 && s->n[d] <= (int64_t)1 << 30, STS_E_INVALID,
                  "grid size out of range");
      STS_REQUIRE(s->n[d] == s->n[0], STS_E_INVALID, "grid must be isotropic (equal n[d])");
    } else {
      STS_REQUIRE(s->n[d] == 1 || s->n[d] == 0, STS_E_INVALID, "unused directions need n[d] = 1");
    }
  }
  int64_t nh = 1;
  for (int d = 0; d < dim; ++d) nh *= s->n[d];
  STS_REQUIRE(nh <= ((int64_t)1 << 34), STS_E_INVALID, "too many grid nodes");
}

Grid make_grid(const sts_space& s) {
  Grid g;
  g.dim = s.kind;
  g.nx = (int)s.n[0];
  g.ny = g.dim >= 2 ? (int)s.n[1] : 1;
  g.nz = g.dim >= 3 ? (int)s.n[2] : 1;
  g.nh = (int64_t)g.nx * g.ny * g.nz;
  return g;
}

static inline int sidx(int dx, int dy, int dz) { return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1); }

Stencil make_stencil(const sts_space& s, int op) {
  Stencil st{};
  const Grid g = make_grid(s);
  st.dim = g.dim;
  st.nx = g.nx;
  st.ny = g.ny;
  st.nz = g.nz;
  const double h = 1.0 / (double)(s.n[0] + 1);
  const double mu = s.mu;
  if (s.kind == STS_FE_P1_1D) {
    if (op == STS_OP_K) {
      st.c[sidx(-1, 0, 0)] = -mu / h;
      st.c[sidx(0, 0, 0)] = 2.0 * mu / h;
      st.c[sidx(1, 0, 0)] = -mu / h;
    } else {
      st.c[sidx(-1, 0, 0)] = h / 6.0;
      st.c[sidx(0, 0, 0)] = 4.0 * h / 6.0;
      st.c[sidx(1, 0, 0)] = h / 6.0;
    }
  } else if (s.kind == STS_FE_P1_2D) {
    if (op == STS_OP_K) {
      st.c[sidx(0, 0, 0)] = 4.0 * mu;
      st.c[sidx(1, 0, 0)] = st.c[sidx(-1, 0, 0)] = -mu;
      st.c[sidx(0, 1, 0)] = st.c[sidx(0, -1, 0)] = -mu;
    } else {
      const double w = h * h / 12.0;
      st.c[sidx(0, 0, 0)] = 6.0 * w;
      st.c[sidx(1, 0, 0)] = st.c[sidx(-1, 0, 0)] = w;
      st.c[sidx(0, 1, 0)] = st.c[sidx(0, -1, 0)] = w;
      st.c[sidx(1, 1, 0)] = st.c[sidx(-1, -1, 0)] = w;
    }
  } else {
    if (op == STS_OP_K) {
      st.c[sidx(0, 0, 0)] = 6.0 * mu * h;
      st.c[sidx(1, 0, 0)] = st.c[sidx(-1, 0, 0)] = -mu * h;
      st.c[sidx(0, 1, 0)] = st.c[sidx(0, -1, 0)] = -mu * h;
      st.c[sidx(0, 0, 1)] = st.c[sidx(0, 0, -1)] = -mu * h;
    } else {
      const double w1[3] = {1.0, 4.0, 1.0};
      const double sc = (h / 6.0) * (h / 6.0) * (h / 6.0);
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx)
            st.c[sidx(dx, dy, dz)] = sc * w1[dx + 1] * w1[dy + 1] * w1[dz + 1];
    }
  }
  return st;
}

// ---------------------------------------------------------------------------
// device memory helpers
// ---------------------------------------------------------------------------

// Device block cache.  Allocating and freeing blocks of gigabytes through the
// driver takes from milliseconds to seconds (a 95^3 request's basis growth
// measured 0.1 to 2.9 s per step, with 0.5 s frees), which bounded serving.
// Blocks of kCacheMin bytes and more are therefore rounded up to one of
// eight sizes per power of two and, when released, kept per device for a
// later allocation that fits (best fit, at most a quarter larger) instead of
// being returned; a failed hipMalloc returns the idle blocks to the driver
// and retries.  Callers release a block only when no queued work uses it:
// the problem's stream is synchronised before teardown, before the basis
// grows and before any other reallocation of a live buffer; a release while
// an exception unwinds goes to hipFree.  Idle blocks above kCacheMaxIdle go
// back to the driver, largest first.  The cache lives until the process ends.
constexpr size_t kCacheMin = size_t(16) << 20;
constexpr size_t kCacheMaxIdle = size_t(32) << 30;

struct BlockCache {
  std::mutex mu;
  std::multimap<size_t, std::pair<int, void*>> idle;   // bytes -> (device, block)
  size_t idle_bytes = 0;
};

BlockCache& block_cache() {
  static BlockCache* c = new BlockCache;   // never destroyed: no frees after runtime teardown
  return *c;
}

size_t cache_class(size_t n) {
  if (n < kCacheMin) return n;
  const int e = 63 - __builtin_clzll((unsigned long long)n);
  const size_t step = size_t(1) << (e - 3);
  return (n + step - 1) / step * step;
}

void cache_trim(int dev) {
  BlockCache& c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (auto it = c.idle.begin(); it != c.idle.end();) {
    if (dev >= 0 && it->second.first != dev) {
      ++it;
      continue;
    }
    (void)hipFree(it->second.second);
    c.idle_bytes -= it->first;
    it = c.idle.erase(it);
  }
}

// A block of at least n bytes on the current device; *got receives its size.
void* dev_alloc(size_t n, size_t* got, int* dev_out) {
  int dev = 0;
  STS_HIP(hipGetDevice(&dev));
  *dev_out = dev;
  const size_t cls = cache_class(std::max<size_t>(n, 8));
  if (cls >= kCacheMin) {
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    for (auto it = c.idle.lower_bound(cls); it != c.idle.end() && it->first <= cls + cls / 4;
         ++it) {
      if (it->second.first != dev) continue;
      void* p = it->second.second;
      *got = it->first;
      c.idle_bytes -= it->first;
      c.idle.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, cls) != hipSuccess) {
    (void)hipGetLastError();
    cache_trim(dev);
    if (hipMalloc(&p, cls) != hipSuccess) {
      (void)hipGetLastError();
      throw Error{STS_E_NOMEM, "hipMalloc of " + std::to_string(cls) + " bytes failed"};
    }
  }
  *got = cls;
  return p;
}

void dev_free(void* p, size_t bytes, int dev) {
  if (!p) return;
  if (bytes < kCacheMin || std::uncaught_exceptions() > 0) {
    (void)hipFree(p);
    return;
  }
  BlockCache& c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.idle.emplace(bytes, std::make_pair(dev, p));
  c.idle_bytes += bytes;
  while (c.idle_bytes > kCacheMaxIdle && !c.idle.empty()) {
    auto it = std::prev(c.idle.end());
    (void)hipFree(it->second.second);
    c.idle_bytes -= it->first;
    c.idle.erase(it);
  }
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int dev = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    dev_free(p, bytes, dev);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t n) {
    release();
    p = dev_alloc(n == 0 ? 8 : n, &bytes, &dev);
  }
  double* d() const { return static_cast<double*>(p); }
};

// A device array that grows: a larger allocation replaces the old one and a
// kernel copies the kept prefix across.  Old and new coexist for the copy.
struct GrowBuf {
  char* base = nullptr;
  size_t bytes = 0;
  int dev = 0;

  GrowBuf() = default;
  GrowBuf(const GrowBuf&) = delete;
  GrowBuf& operator=(const GrowBuf&) = delete;
  ~GrowBuf() { release(); }

  void release() {
    dev_free(base, bytes, dev);
    base = nullptr;
    bytes = 0;
  }
  double* d() const { return reinterpret_cast<double*>(base); }

  // Make `need` bytes usable; the first `keep` bytes (a multiple of 8) keep
  // their contents.
  void ensure(size_t need, size_t keep, hipStream_t st) {
    if (need <= bytes) return;
    size_t got = 0;
    int ndev = 0;
    void* p = dev_alloc(need, &got, &ndev);
    if (base && keep)
      copy_cols((int64_t)(std::min(keep, bytes) / 8), 1, reinterpret_cast<const double*>(base), 0,
                static_cast<double*>(p), 0, st);
    STS_HIP(hipStreamSynchronize(st));
    release();
    base = static_cast<char*>(p);
    bytes = got;
    dev = ndev;
  }
};

static inline int64_t pad_ld(int64_t n) { return ((n + 31) / 32) * 32; }

// Basis columns added per growth step, in blocks of 2p columns.
constexpr int kGrowBlocks = 8;

// Bytes of the k-dependent buffers for a basis capacity of kc columns
// (leading dimension ld): V, Mx V, Kx V (and V's FP32 copy in the mixed-
// precision solve), the reduced matrices and beta, the
// eigensolver's Q and workspace, Z, Y and the refinement scratch, and the time
// factor of the exact residual.
int64_t basis_capacity_bytes(int64_t ld, int64_t nt, int p, int64_t kc, bool v32) {
  return 3 * ld * kc * 8 + (v32 ? ld * kc * 4 : 0) + 2 * kc * kc * 8 + kc * p * 8 + kc * kc * 8 +
         eig_work_doubles((int)std::min<int64_t>(kc, kEigMaxK)) * 8 + kc * 8 * 3 +
         3 * kc * nt * 8 + nt * (p + 2 * kc) * 8;
}

// The first capacity sts_solve allocates: kGrowBlocks blocks, or the whole
// max_outer + 2 blocks if fewer.
int64_t initial_capacity(int p, int max_outer) {
  return 2LL * p * std::min<int64_t>(kGrowBlocks, (int64_t)max_outer + 2);
}

// Scratch of the step-level calls: freed when the call returns.
struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  T* get(size_t count) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(count * sizeof(T), 8));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error{STS_E_NOMEM, "hipMalloc failed in step-level call"};
    }
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
};

// ---------------------------------------------------------------------------
// block Gram-Schmidt in the Mx inner product
// ---------------------------------------------------------------------------

// Below this independence ratio of the block the Cholesky-QR step amplifies
// the O(eps) components along V left by CGS2 beyond 1e-14.
constexpr double kThirdPassRatio = 1e-2;

int orthonormalize_block(const Grid& g, const Stencil& K, const Stencil& M, const double* V,
                         const double* MV, int64_t ldv, int64_t k, double* W, double* MW,
                         int64_t ldw, int ncols, double defl, OrthScratch& s, int* idx,
                         hipStream_t st, double* KW, bool first_done) {
  const int64_t nh = g.nh;
  int opsM[16];
  for (int c = 0; c < 16; ++c) opsM[c] = STS_OP_M;
  s.cgs_passes = 0;
  s.cgs32_passes = 0;
  auto cgs = [&](int nc) {
    if (k <= 0) return;
    ++s.cgs_passes;
    gemm_tn(nh, (int)k, nc, MV, ldv, W, ldw, s.C, s.ldc, s.part, st);   // C = V^T Mx W
    gemm_nn_sub(nh, (int)k, nc, V, ldv, s.C, s.ldc, W, ldw, st);        // W -= V C
  };
  // mixed precision: the first pass takes its coefficients from the FP32
  // copy of V contracted with Mx W (rounded to FP32) in FP32, and removes
  // them with the FP64 basis, so the new block stays in the span of W and V
  // exactly (an update with the rounded basis would add the rounding of V,
  // which lies outside that span, to every block); the FP64 pass after it
  // re-orthogonalises
  auto cgs32 = [&](int nc) {
    if (k <= 0) return;
    ++s.cgs32_passes;
    gemm_tn32(nh, (int)k, nc, s.V32, ldv, MW, ldw, s.C, s.ldc, reinterpret_cast<float*>(s.part),
              st);                                                         // C = V^T (Mx W)
    gemm_nn_sub(nh, (int)k, nc, V, ldv, s.C, s.ldc, W, ldw, st);           // W -= V C
  };
  auto fetch_info = [&]() {
    STS_HIP(hipMemcpyAsync(s.host, s.info, sizeof(CholInfo), hipMemcpyDeviceToHost, st));
    STS_HIP(hipStreamSynchronize(st));
    return *s.host;
  };
  // Mx-norms on entry: the reference for "already in the span of V" (with
  // first_done the caller has formed them and the first pass)
  if (!first_done) {
    stencil_apply(g, K, M, opsM, ncols, W, ldw, MW, ldw, st);
    gemm_tn(nh, ncols, ncols, W, ldw, MW, ldw, s.G, 16, s.part, st);
    copy_cols(1, ncols, s.G, 17, s.norm0, 1, st);
  }
  // the second pass with the reduced-matrix columns of the previous block in
  // the same read of V: [C | Kred | Mred] = V^T [Mx W, Kx V_p, Mx V_p] (the
  // coefficients from Mx W, formed by the stencil, rather than from the
  // stored Mx V)
  auto cgs_fused = [&](int nc) {
    ++s.cgs_passes;
    stencil_apply(g, K, M, opsM, nc, W, ldw, MW, ldw, st);
    const double* B[3] = {MW, s.pend_K, s.pend_M};
    const int nb[3] = {nc, s.pend_n, s.pend_n};
    double* C[3] = {s.C, s.pend_Kout, s.pend_Mout};
    const int64_t ldc[3] = {s.ldc, s.pend_ldc, s.pend_ldc};
    gemm_tn_segs(nh, (int)k, V, ldv, 3, B, nb, ldw, C, ldc, s.part, st);
    gemm_nn_sub(nh, (int)k, nc, V, ldv, s.C, s.ldc, W, ldw, st);        // W -= V C
    s.pend_done = true;
  };
  // classical Gram-Schmidt against V, twice
  s.pend_done = false;
  if (first_done) {
  } else if (s.V32) {
    cgs32(ncols);
  } else {
    cgs(ncols);
  }
  if (s.pend_n > 0 && k > 0) cgs_fused(ncols);
  else cgs(ncols);
  // Cholesky-QR of the block with deflation
  stencil_apply(g, K, M, opsM, ncols, W, ldw, MW, ldw, st);
  gemm_tn(nh, ncols, ncols, W, ldw, MW, ldw, s.G, 16, s.part, st);
  chol_deflate(ncols, s.G, 16, s.norm0, defl, kBlockDefl, s.Rinv, s.info, st);
  apply_rinv(nh, ncols, s.info, s.Rinv, W, nullptr, ldw, nullptr, st);
  CholInfo h = fetch_info();
  const int kept = h.kept;
  for (int j = 0; j < kept; ++j) idx[j] = h.idx[j];
  if (kept == 0) return 0;
  // A small pivot above amplifies the rounding left along V (by 1 / rmin)
  // and within the block: then one more pass against V restores the
  // former; a second Cholesky-QR always restores the latter.
  if (h.rmin < kThirdPassRatio) cgs(kept);
  stencil_apply(g, K, M, opsM, kept, W, ldw, MW, ldw, st);
  gemm_tn(nh, kept, kept, W, ldw, MW, ldw, s.G, 16, s.part, st);
  chol_deflate(kept, s.G, 16, nullptr, 0.0, kBlockDefl, s.Rinv, s.info, st);
  apply_rinv(nh, kept, s.info, s.Rinv, W, nullptr, ldw, nullptr, st);
  h = fetch_info();
  STS_REQUIRE(h.kept == kept, STS_E_NUMERIC, "block lost rank in the second Cholesky-QR pass");
  if (KW) stencil_apply_km(g, K, M, kept, W, ldw, KW, ldw, MW, ldw, st);   // exact images
  else stencil_apply(g, K, M, opsM, kept, W, ldw, MW, ldw, st);            // exact Mx image
  return kept;
}

// ---------------------------------------------------------------------------
// Iteration loop with asynchronous polling (plain CG and multigrid PCG)
// ---------------------------------------------------------------------------

// Launches iterations in chunks until every column has stopped.  After each
// chunk the newest state slot is copied to pinned memory behind an event.
// Pipelined: the next chunk is queued before the host waits for the copy of
// the previous one (the GPU never idles; suits long runs of short launches).
// Not pipelined: the host waits for the chunk it just queued (suits short
// runs whose length is known well in advance).
struct PollLoop {
  CGScal* host_scal = nullptr;   // pinned, 2 * kMaxCols
  hipEvent_t ev[2] = {nullptr, nullptr};
  int64_t poll_restarts = 0;

  PollLoop() = default;
  PollLoop(const PollLoop&) = delete;
  PollLoop& operator=(const PollLoop&) = delete;
  ~PollLoop() {
    if (host_scal) (void)hipHostFree(host_scal);
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  void init() {
    if (host_scal) return;
    STS_HIP(hipHostMalloc(reinterpret_cast<void**>(&host_scal), sizeof(CGScal) * 2 * kMaxCols,
                          hipHostMallocDefault));
    STS_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    STS_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  }

  // iterate(parity, cols, nl) queues one iteration writing state slot
  // `parity`; the set-up has initialised both slots.  Iteration i (from 1)
  // has parity i & 1.  Final states of columns < ncols go to out.
  template <class F>
  void run(F&& iterate, const CGScal* dev_scal, int ncols, int chunk, int chunk_cap,
           bool pipelined, CGScal* out, hipStream_t st) {
    for (int q = 0; q < 2 * kMaxCols; ++q) {
      host_scal[q] = CGScal{};
      host_scal[q].active = 1;   // never read as "stopped" before a copy lands
    }
    int64_t iters = 0;
    int cols[kMaxCols], nl = 0;
    for (int c = 0; c < ncols; ++c) cols[nl++] = c;
    int slot = 0;
    bool done = false;
    while (!done) {
      bool pending = false;
      for (;;) {
        for (int i = 0; i < chunk; ++i) {
          ++iters;
          iterate((int)(iters & 1), cols, nl);
        }
        // state written by the last iteration of the chunk
        STS_HIP(hipMemcpyAsync(host_scal + slot * kMaxCols, dev_scal + (iters & 1) * kMaxCols,
                               sizeof(CGScal) * kMaxCols, hipMemcpyDeviceToHost, st));
        STS_HIP(hipEventRecord(ev[slot], st));
        if (pipelined && !pending) {
          pending = true;
          slot ^= 1;
          chunk = std::min(chunk * 2, chunk_cap);
          continue;
        }
        const int look = pipelined ? slot ^ 1 : slot;
        STS_HIP(hipEventSynchronize(ev[look]));
        int n2 = 0;
        for (int c = 0; c < ncols; ++c)
          if (host_scal[look * kMaxCols + c].active) cols[n2++] = c;
        if (n2 == 0) {
          if (!pipelined) {
            // the copy followed every queued iteration: it is the final state
            for (int c = 0; c < ncols; ++c) out[c] = host_scal[look * kMaxCols + c];
            done = true;
          }
          break;
        }
        nl = n2;
        slot ^= 1;
        chunk = pipelined ? std::min(chunk * 2, chunk_cap) : chunk_cap;
      }
      if (done) break;
      // confirm with a fully synchronised read of the newest state
      STS_HIP(hipStreamSynchronize(st));
      STS_HIP(hipMemcpy(out, dev_scal + (iters & 1) * kMaxCols, sizeof(CGScal) * kMaxCols,
                        hipMemcpyDeviceToHost));
      int n2 = 0;
      for (int c = 0; c < ncols; ++c)
        if (out[c].active) cols[n2++] = c;
      if (n2 == 0) break;
      ++poll_restarts;   // the polled copy was not current: keep iterating
      nl = n2;
      chunk = pipelined ? 8 : chunk_cap;
    }
  }
};

// Plain CG on a batch of columns (Kx or Mx per column).
struct CGRunner {
  Grid g;
  Stencil K, M;
  CGWork w;
  PollLoop poll;
  // iterations the last batch of each kind needed (0 = none yet): batches
  // with only Mx columns converge in a nearly fixed count, so the first chunk
  // is sized from it and the host waits once instead of doubling chunks
  int expect[2] = {0, 0};

  // Solve A_c x_c = b_c for c < ncols; x_c written to w.x + c * w.ld.
  void run(const int* ops, int ncols, const double* const* b, double rtol, int maxit,
           CGScal* out, hipStream_t st) {
    // initial state (read by the set-up, launch 0, and by launch 1)
    cg_init_state(w, ncols, rtol, maxit, st);
    for (int c = 0; c < ncols; ++c) w.b[c] = b[c];
    cg_setup(g, K, M, ops, ncols, w, st);
    int kind = 0;   // 1 if any column is Kx
    for (int c = 0; c < ncols; ++c) kind |= ops[c] == STS_OP_K ? 1 : 0;
    auto iterate = [&](int parity, const int* cols, int nl) {
      cg_iterate(g, K, M, ops, ncols, w, parity, cols, nl, st);
    };
    const int ex = expect[kind];
    if (ex > 0)
      poll.run(iterate, w.scal, ncols, std::min(ex, maxit + 1), std::max(2, ex / 16), false, out,
               st);
    else
      poll.run(iterate, w.scal, ncols, 8, 256, true, out, st);
    int most = 0;
    for (int c = 0; c < ncols; ++c) most = std::max(most, out[c].iters);
    expect[kind] = most + 1;   // the launch after the last update detects convergence
  }
};

// Multigrid-preconditioned CG on Kx columns, with its level buffers.
struct MGRunner {
  MGWork w{};
  PollLoop poll;
  DevBuf levels, vecs, scal, parts, dst;
  int expect = 12;          // iterations the last run needed (first chunk length)
  int expect_shifted = 12;  // the same for the shifted operator Kx + s Mx
  int expect32 = 6;         // the same for one FP32 round of a mixed-precision solve
  DevBuf corr, defect, norms;   // mixed precision: correction, FP64 residual, (r, r)

  // Allocate for the plan; x / ldx are set per run.
  void setup(const MGPlan& plan) {
    w.plan = plan;
    const bool d3 = plan.dim == 3;
    auto nodes = [&](int l) {
      const int64_t n = plan.n[l];
      return d3 ? n * n * n : n * n;
    };
    for (int l = 0; l <= plan.nlev; ++l) w.ld[l] = pad_ld(nodes(l));
    // per smoothed level l >= 1: b, e, the pre-smoothed iterate and, in 3-D,
    // the two post-smoothing buffers; the exact level: b, e and temporaries
    int64_t tot = 0;
    for (int l = 1; l <= plan.nlev; ++l) {
      tot += 2 * w.ld[l] * kMaxCols;
      if (l < plan.nlev) tot += (d3 ? 3 : 1) * w.ld[l] * kMaxCols;
    }
    const int ntmp = d3 ? 1 : (plan.exact > kMGCoarseMax ? 2 : 0);
    tot += ntmp * w.ld[plan.nlev] * kMaxCols;
    levels.alloc(std::max<int64_t>(tot, 1) * 8);
    vecs.alloc((d3 ? 7 : 6) * w.ld[0] * kMaxCols * 8);
    double* q = levels.d();
    for (int l = 1; l <= plan.nlev; ++l) {
      w.b[l] = q;
      w.e[l] = q + w.ld[l] * kMaxCols;
      q += 2 * w.ld[l] * kMaxCols;
      if (l < plan.nlev) {
        w.xp[l] = q;
        q += w.ld[l] * kMaxCols;
        if (d3) {
          w.u1[l] = q;
          w.d0[l] = q + w.ld[l] * kMaxCols;
          q += 2 * w.ld[l] * kMaxCols;
        }
      }
    }
    if (ntmp > 0) w.t1 = q;
    if (ntmp > 1) w.t2 = q + w.ld[plan.nlev] * kMaxCols;
    double* v = vecs.d();
    w.b[0] = v;
    w.e[0] = v + 1 * w.ld[0] * kMaxCols;
    w.p[0] = v + 2 * w.ld[0] * kMaxCols;
    w.p[1] = v + 3 * w.ld[0] * kMaxCols;
    w.q = v + 4 * w.ld[0] * kMaxCols;
    w.xp[0] = v + 5 * w.ld[0] * kMaxCols;
    if (d3) {
      // q is free while the V-cycle runs (the iteration's A launch rewrites it)
      w.u1[0] = w.q;
      w.d0[0] = v + 6 * w.ld[0] * kMaxCols;
    }
    w.max_tiles = mg_max_tiles(plan);
    scal.alloc(sizeof(CGScal) * 2 * kMaxCols);
    w.scal = static_cast<CGScal*>(scal.p);
    parts.alloc((size_t)(3 * w.max_tiles + 4) * kMaxCols * 8);
    w.part_rr = parts.d();
    w.part_rz = w.part_rr + (size_t)w.max_tiles * kMaxCols;
    w.part_pq = w.part_rz + (size_t)w.max_tiles * kMaxCols;
    w.alpha = w.part_pq + (size_t)w.max_tiles * kMaxCols;
    w.tot = w.alpha + kMaxCols;
    const int m = plan.exact;
    std::vector<double> tab(mg_dst_table_size(m));
    mg_dst_table(m, tab.data());
    dst.alloc(tab.size() * 8);
    STS_HIP(hipMemcpy(dst.p, tab.data(), tab.size() * 8, hipMemcpyHostToDevice));
    w.dst = dst.d();
    poll.init();
  }

  // Algorithmic bytes of one column-iteration per fine node: each level's
  // down reads b_l and writes b_{l+1} and the pre-smoothed iterate, its up
  // reads b_l, that iterate and e_{l+1} and writes e_l, the coarse launch reads b_L and writes e_L, A reads z, p and
  // writes p, q, B reads x, p, r, q and writes x, r.
  double bytes_per_node() const {
    if (w.plan.dim == 3) return mg3_bytes_per_node(w.plan);
    const double n0 = (double)w.plan.n[0] * w.plan.n[0];
    double b = 80.0 * n0;
    for (int l = 0; l < w.plan.nlev; ++l) {
      const double nf = (double)w.plan.n[l] * w.plan.n[l];
      const double nc = (double)w.plan.n[l + 1] * w.plan.n[l + 1];
      b += 8.0 * (2.0 * nf + nc) + 8.0 * (3.0 * nf + nc);
    }
    const double nL = (double)w.plan.n[w.plan.nlev] * w.plan.n[w.plan.nlev];
    b += 16.0 * nL;
    return b / n0;
  }

  // K x_c = b_c for c < ncols, x_c at x + c * ldx.  With replace_every > 0
  // (the FP32 PCG with x in FP64) the residual is replaced by b - K x before
  // every replace_every-th iteration.
  void run(double* x, int64_t ldx, int ncols, const double* const* b, double rtol, int maxit,
           CGScal* out, hipStream_t st, int replace_every = 0) {
    w.x = x;
    w.ldx = ldx;
    int cols[kMaxCols];
    for (int c = 0; c < ncols; ++c) {
      cols[c] = c;
      w.rhs[c] = b[c];
    }
    pcg_setup(w, b, cols, ncols, ncols, rtol, maxit, st);
    int it = 0;
    poll.run(
        [&](int parity, const int* cl, int nl) {
          if (replace_every > 0 && it > 0 && it % replace_every == 0) mg3_replace(w, cl, nl, st);
          ++it;
          pcg_iterate(w, parity, cl, nl, ncols, st);
        },
        w.scal, ncols, std::max(1, std::min(expect, maxit + 1)), 2, false, out, st);
    int most = 0;
    for (int c = 0; c < ncols; ++c) most = std::max(most, out[c].iters);
    expect = most + 1;   // the iteration after the last update detects convergence
  }
};

}  // namespace sts

using namespace sts;

// ---------------------------------------------------------------------------
// the problem object
// ---------------------------------------------------------------------------

struct sts_problem {
  sts_space space{};
  Grid grid{};
  Stencil K{}, M{};
  int64_t nh = 0, nt = 0, ldv = 0;
  int p = 0;
  hipStream_t stream = nullptr;
  double fnorm = 0.0;
  double floor_coef = 0.0;   // residual_floor() / ||U||_F / kFloorFactor

  std::vector<double> h_td, h_ts, h_md, h_ms;
  DevBuf F1, F2, tdv;   // tdv: d (nt) | e (nt) | m (nt) | n (nt)

  // basis and reduced matrices
  int64_t kcap = 0;
  int64_t k = 0;          // columns in V (including a pending new block)
  int64_t k_sol = 0;      // columns of the current Galerkin solution
  // reduced-matrix columns of the newest block not yet formed: the next
  // block's re-orthogonalisation pass forms them in its read of V
  int64_t pend_start = 0, pend_size = 0;
  int64_t blk_start = 0, blk_size = 0;
  // lagged re-orthogonalisation: a block orthogonalised once and normalised
  // provisionally, at V[:, k .. k + prov) with its exact images in KV, MV; the
  // next block is expanded from it, and its second pass comes with the next
  // block's first (prov_norm0: its entry norms, the deflation reference)
  int64_t prov = 0;
  DevBuf prov_norm0;
  std::vector<int> tags;  // 0: positive power, 1: negative power (final and provisional columns)
  GrowBuf V, MV, KV;      // basis and its images, grown with the space
  GrowBuf V32;            // mixed precision: FP32 copy of V (first Gram-Schmidt pass)
  bool want_v32 = false;  // V32 is allocated and grown with the basis
  bool use_v32 = false;   // this solve's first Gram-Schmidt pass reads V32
  int64_t v32_cols = 0;   // leading columns of V32 that hold V rounded
  DevBuf Kred, Mred, beta;
  // called with the extra bytes before the basis grows (the server's
  // footprint accounting; may block or throw)
  std::function<void(int64_t)> grow_hook;
  DevBuf qr_work, qr_R;   // exact residual through the QR of the time factor
  int residual_qr = 0;    // sts_opts::residual_qr of the last solve

  // CG
  DevBuf cg_r, cg_p, cg_scal, cg_part, counters;
  CGRunner cg;
  // multigrid-preconditioned CG for Kx (allocated on first use)
  bool mg_ok = false;
  bool mass_cheb = false;   // Mx solves by Chebyshev iteration
  bool tri_ok = false;      // 1-D: direct tridiagonal solves for Kx and Mx
  DevBuf tri_fac;           // their elimination factors (tridiag_factor_doubles)
  bool tensor_mass = false; // 3-D trilinear mass: direct tensor-product Mx solves
  DevBuf tmass_fac;         // elimination factors of tridiag(1, 4, 1) (2 n)
  MGPlan mg_plan_{};
  std::unique_ptr<MGRunner> mg;
  // kernel timing of the last profiled solve
  Profiler prof;
  bool profiled = false;

  // small scratch
  DevBuf gram, tn_part, rinv, cinfo, norm0, smallv, Lb, T1, okflag;
  // reduced solve
  DevBuf lam, Q, eig_work, eig_meta, qb, Z, Y, RB;
  // residual
  DevBuf BT, res_part;
  double* pinned = nullptr;   // 64 doubles
  bool solved = false;
  int64_t inner_K = 0, inner_M = 0;
  int64_t inner_K32 = 0, defect_rounds = 0;   // mixed-precision Kx solves
  double alg_bytes = 0.0;
  int checks = 0;
  double last_cheap = -1.0;
  std::vector<double> shifts;   // rational Krylov shifts used so far

  unsigned* counter(int i) const { return static_cast<unsigned*>(counters.p) + i; }

  ~sts_problem() {
    if (pinned) (void)hipHostFree(pinned);
  }
};

namespace {

int64_t capacity_bytes(const sts_problem* P, int64_t kc) {
  return basis_capacity_bytes(P->ldv, P->nt, P->p, kc, P->want_v32);
}

// Make room for `need` basis columns.  V, Mx V and Kx V grow (GrowBuf)
// kGrowBlocks blocks ahead of the need, to at most `limit` columns; the
// reduced matrices, beta and the current solution Y are copied to their new
// leading dimension; the rest is scratch.  The growth hook is told the
// persistent increase plus the transient of the largest copy (the old array
// and its replacement coexist), and then that the transient is returned.
void ensure_capacity(sts_problem* P, int64_t need, int64_t limit, int64_t budget) {
  if (need <= P->kcap) return;
  const int64_t b2 = 2 * P->p;
  limit = std::max(limit, need);
  const int64_t kc = std::min(std::max(need, P->kcap + b2 * kGrowBlocks), limit);
  const int64_t ld = P->ldv;
  const int64_t nt = P->nt;
  const int64_t bytes = capacity_bytes(P, kc);
  STS_REQUIRE(budget <= 0 || bytes <= budget, STS_E_NOMEM,
              "basis of " + std::to_string(kc) + " columns needs " + std::to_string(bytes) +
                  " bytes, above the memory budget");
  const int64_t transient = ld * P->kcap * 8;
  STS_REQUIRE(P->k + P->prov <= P->kcap, STS_E_STATE, "basis columns beyond the capacity");
  if (P->grow_hook) P->grow_hook(bytes - capacity_bytes(P, P->kcap) + transient);
  hipStream_t st = P->stream;
  const int64_t old = P->kcap;
  // the kept columns include a provisional block and its images
  const int64_t keep = ld * (P->k + P->prov) * 8;
  P->V.ensure(ld * kc * 8, keep, st);
  P->MV.ensure(ld * kc * 8, keep, st);
  P->KV.ensure(ld * kc * 8, keep, st);
  if (P->want_v32) P->V32.ensure(ld * kc * 4, ld * P->v32_cols * 4, st);
  // small buffers with leading dimension kc: copy column by column
  auto regrow = [&](DevBuf& b, int64_t cols, int64_t rows_keep, int64_t cols_keep) {
    DevBuf nb;
    nb.alloc(kc * cols * 8);
    fill(nb.d(), kc * cols, 0.0, st);
    if (old && b.p && rows_keep > 0 && cols_keep > 0)
      copy_cols(rows_keep, (int)cols_keep, b.d(), old, nb.d(), kc, st);
    STS_HIP(hipStreamSynchronize(st));
    std::swap(b.p, nb.p);
    std::swap(b.bytes, nb.bytes);
    std::swap(b.dev, nb.dev);
  };
  regrow(P->Kred, kc, old, old);
  regrow(P->Mred, kc, old, old);
  regrow(P->beta, P->p, old, P->p);
  regrow(P->Y, nt, P->k_sol, P->k_sol > 0 ? nt : 0);
  P->lam.alloc(kc * 8);
  P->Q.alloc(kc * kc * 8);
  P->eig_work.alloc(eig_work_doubles((int)std::min<int64_t>(kc, kEigMaxK)) * 8);
  P->eig_meta.alloc(64);
  P->qb.alloc(kc * 4 * 8);
  P->Z.alloc(kc * nt * 8);
  P->RB.alloc(kc * nt * 8);
  P->BT.alloc(nt * (P->p + 2 * kc) * 8);
  P->tn_part.alloc(gemm_tn_partial_size_wide(std::max<int64_t>(P->nh, nt), (int)kc) * 8);
  P->kcap = kc;
  if (P->grow_hook && transient > 0) P->grow_hook(-transient);
  if (!P->smallv.p || P->smallv.bytes < (size_t)std::max<int64_t>(kc * 16, 4096) * 8)
    P->smallv.alloc(std::max<int64_t>(kc * 16, 4096) * 8);
}

TimeOps time_ops(const sts_problem* P) {
  const double* b = P->tdv.d();
  return TimeOps{b, b + P->nt, b + 2 * P->nt, b + 3 * P->nt};
}

// Copy a few device doubles to the host (synchronising the stream).
void fetch(sts_problem* P, const double* src, int n, double* dst) {
  STS_HIP(hipMemcpyAsync(P->pinned, src, n * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  STS_HIP(hipStreamSynchronize(P->stream));
  std::memcpy(dst, P->pinned, n * sizeof(double));
}

// Orthonormalise the ncols columns at V[:, k..k+ncols) against V[:, 0..k) in
// the Mx inner product (CGS2, then two Cholesky-QR passes with deflation),
// pack the kept ones at V[:, k..), fill MV, KV, the reduced matrices and beta.
// Returns the number of kept columns; keep_idx receives their source indices.
// Scratch of the block orthogonalisation, with the pending reduced-matrix
// columns of the last final block (formed in the next pass over V).
OrthScratch orth_scratch(sts_problem* P) {
  OrthScratch s;
  s.part = P->tn_part.d();
  s.G = P->gram.d();
  s.C = P->smallv.d();
  s.ldc = P->kcap;
  s.norm0 = P->norm0.d();
  s.Rinv = P->rinv.d();
  s.info = static_cast<CholInfo*>(P->cinfo.p);
  s.host = reinterpret_cast<CholInfo*>(P->pinned);
  s.V32 = P->use_v32 ? reinterpret_cast<const float*>(P->V32.base) : nullptr;
  if (P->pend_size > 0) {
    const int64_t ps = P->pend_start, ld = P->ldv, kc = P->kcap;
    s.pend_n = (int)P->pend_size;
    s.pend_K = P->KV.d() + ps * ld;
    s.pend_M = P->MV.d() + ps * ld;
    s.pend_Kout = P->Kred.d() + ps * kc;
    s.pend_Mout = P->Mred.d() + ps * kc;
    s.pend_ldc = kc;
  }
  return s;
}

// The pass over V formed the pending columns: mirror them into the rows.
void consume_pending(sts_problem* P, const OrthScratch& s) {
  if (!s.pend_done) return;
  const int64_t ps = P->pend_start, pk = P->pend_size, kc = P->kcap;
  mirror((int)ps, (int)pk, P->Kred.d() + ps * kc, kc, P->Kred.d() + ps, kc, P->stream);
  mirror((int)ps, (int)pk, P->Mred.d() + ps * kc, kc, P->Mred.d() + ps, kc, P->stream);
  P->alg_bytes += 8.0 * P->nh * 2 * pk;
  P->pend_size = 0;
}

// A final block at V[:, k0 .. k0 + kept): its reduced-matrix columns become
// pending, its rows of beta = V^T F1 are formed, V32 gets its rounding.
void register_block(sts_problem* P, int64_t k0, int kept) {
  const int64_t nh = P->nh, ld = P->ldv;
  double* W = P->V.d() + k0 * ld;
  if (P->use_v32) {
    round_cols(nh, kept, W, ld, reinterpret_cast<float*>(P->V32.base) + k0 * ld, ld, P->stream);
    P->v32_cols = k0 + kept;
  }
  P->pend_start = k0;
  P->pend_size = kept;
  gemm_tn(nh, kept, P->p, W, ld, P->F1.d(), ld, P->beta.d() + k0, P->kcap, P->tn_part.d(),
          P->stream);
  P->alg_bytes += (4.0 * 16.0 - 8.0) * nh * kept;
}

int append_block(sts_problem* P, int ncols, double defl, int* keep_idx) {
  hipStream_t st = P->stream;
  const int64_t nh = P->nh, ld = P->ldv, k = P->k;
  double* W = P->V.d() + k * ld;
  double* MW = P->MV.d() + k * ld;
  OrthScratch s = orth_scratch(P);
  double* KW = P->KV.d() + k * ld;
  const int kept = orthonormalize_block(P->grid, P->K, P->M, P->V.d(), P->MV.d(), ld, k, W, MW,
                                        ld, ncols, defl, s, keep_idx, st, KW);
  P->alg_bytes += 2.0 * s.cgs_passes * 8.0 * nh * k + s.cgs32_passes * 12.0 * nh * k +
                  8.0 * 16.0 * nh * ncols;
  consume_pending(P, s);
  if (kept == 0) return 0;
  register_block(P, k, kept);
  return kept;
}

// dst[j] = src[idx[j]] for the columns a Cholesky-QR kept (their entry norms)
__global__ void gather_kept_kernel(const double* src, const CholInfo* info, double* dst) {
  const int j = threadIdx.x;
  if (j < info->kept) dst[j] = src[info->idx[j]];
}

// Lagged re-orthogonalisation (the delayed second pass of classical
// Gram-Schmidt run twice, after Swirydowicz et al., "Low synchronization
// Gram-Schmidt and GMRES algorithms", 2020, in block form and the Mx inner
// product).  The new block W (at V[:, k + prov ..), expanded from the
// provisional block P~ = V[:, k .. k + prov)) and P~ are orthogonalised
// against the final basis V_k = V[:, 0 .. k) together: one read of V_k forms
// [c d] = V_k^T Mx [P~ W] (and the pending reduced-matrix columns), one more
// removes V_k [c d].  That is P~'s second pass and W's first, so each block
// costs two reads of V instead of four.  P~ - V_k c is then normalised
// (Cholesky-QR with deflation against its entry norms; P~ was normalised once,
// so this factor is well conditioned) and becomes final; W drops its
// components along it and is normalised provisionally, or, when final_now
// (a residual check follows), gets its second pass at once.  Spans are those
// of the classical scheme: W was expanded from P~ rather than from the final
// P, and P~ - P lies in span(V_k), whose images the nested extended Krylov
// space already holds.  Returns the kept columns of the new block, now at
// V[:, k' ..) with k' = P->k after the call (final) or provisional (the
// caller sets P->prov).
int append_lagged(sts_problem* P, int nw, double defl, bool final_now, int* idx) {
  const int bp = (int)P->prov;
  if (bp == 0 && final_now) return append_block(P, nw, defl, idx);
  hipStream_t st = P->stream;
  const Grid& g = P->grid;
  const int64_t nh = P->nh, ld = P->ldv, kc = P->kcap;
  int64_t k = P->k;
  int opsM[16];
  for (int c = 0; c < 16; ++c) opsM[c] = STS_OP_M;
  OrthScratch s = orth_scratch(P);
  auto fetch_info = [&]() {
    STS_HIP(hipMemcpyAsync(s.host, s.info, sizeof(CholInfo), hipMemcpyDeviceToHost, st));
    STS_HIP(hipStreamSynchronize(st));
    return *s.host;
  };
  double* W = P->V.d() + (k + bp) * ld;
  double* MW = P->MV.d() + (k + bp) * ld;
  // entry Mx-norms of the new block (its deflation reference) and Mx W
  stencil_apply(g, P->K, P->M, opsM, nw, W, ld, MW, ld, st);
  gemm_tn(nh, nw, nw, W, ld, MW, ld, s.G, 16, s.part, st);
  copy_cols(1, nw, s.G, 17, s.norm0, 1, st);
  P->alg_bytes += 40.0 * nh * nw;
  // [P~ W] against V_k: one read for the coefficients (with the pending
  // columns), one for the update
  if (k > 0) {
    const double* B[3] = {P->MV.d() + k * ld, s.pend_K, s.pend_M};
    const int nb[3] = {bp + nw, s.pend_n, s.pend_n};
    double* C[3] = {s.C, s.pend_Kout, s.pend_Mout};
    const int64_t ldc[3] = {s.ldc, s.pend_ldc, s.pend_ldc};
    gemm_tn_segs(nh, (int)k, P->V.d(), ld, s.pend_n > 0 ? 3 : 1, B, nb, ld, C, ldc, s.part, st);
    s.pend_done = s.pend_n > 0;
    gemm_nn_sub(nh, (int)k, bp + nw, P->V.d(), ld, s.C, s.ldc, P->V.d() + k * ld, ld, st);
    P->alg_bytes += 16.0 * nh * k + 8.0 * nh * (3 * (bp + nw) + 2 * s.pend_n);
  }
  consume_pending(P, s);
  if (bp > 0) {
    // P~ - V_k c: normalise, with its entry norms as the deflation reference
    double* Pc = P->V.d() + k * ld;
    double* MPc = P->MV.d() + k * ld;
    double* KPc = P->KV.d() + k * ld;
    stencil_apply(g, P->K, P->M, opsM, bp, Pc, ld, MPc, ld, st);
    gemm_tn(nh, bp, bp, Pc, ld, MPc, ld, s.G, 16, s.part, st);
    chol_deflate(bp, s.G, 16, P->prov_norm0.d(), defl, kBlockDefl, s.Rinv, s.info, st);
    apply_rinv(nh, bp, s.info, s.Rinv, Pc, nullptr, ld, nullptr, st);
    CholInfo h = fetch_info();
    const int kept_p = h.kept;
    if (kept_p > 0 && h.rmin < kThirdPassRatio && k > 0) {
      // a small pivot amplified the rounding left along V_k: one more pass
      stencil_apply(g, P->K, P->M, opsM, kept_p, Pc, ld, MPc, ld, st);
      gemm_tn(nh, (int)k, kept_p, P->V.d(), ld, MPc, ld, s.C, s.ldc, s.part, st);
      gemm_nn_sub(nh, (int)k, kept_p, P->V.d(), ld, s.C, s.ldc, Pc, ld, st);
      stencil_apply(g, P->K, P->M, opsM, kept_p, Pc, ld, MPc, ld, st);
      gemm_tn(nh, kept_p, kept_p, Pc, ld, MPc, ld, s.G, 16, s.part, st);
      chol_deflate(kept_p, s.G, 16, nullptr, 0.0, kBlockDefl, s.Rinv, s.info, st);
      apply_rinv(nh, kept_p, s.info, s.Rinv, Pc, nullptr, ld, nullptr, st);
      h = fetch_info();
      STS_REQUIRE(h.kept == kept_p, STS_E_NUMERIC, "block lost rank in its third pass");
      P->alg_bytes += 16.0 * nh * k;
    }
    // the provisional tags of the kept columns, in order
    std::vector<int> ptag(kept_p);
    for (int j = 0; j < kept_p; ++j) ptag[j] = P->tags[k + h.idx[j]];
    P->tags.resize(k);
    for (int j = 0; j < kept_p; ++j) P->tags.push_back(ptag[j]);
    P->prov = 0;
    if (kept_p > 0) {
      stencil_apply_km(g, P->K, P->M, kept_p, Pc, ld, KPc, ld, MPc, ld, st);   // exact images
      register_block(P, k, kept_p);
      P->blk_start = k;
      P->blk_size = kept_p;
      P->k = k + kept_p;
      P->alg_bytes += 64.0 * nh * kept_p;
    }
    // W next to the final columns (a deflated P leaves a gap), then W -= P e
    // with e = (Mx P)^T W
    if (kept_p < bp)
      for (int j = 0; j < nw; ++j)
        copy_cols(nh, 1, P->V.d() + (k + bp + j) * ld, ld, P->V.d() + (k + kept_p + j) * ld, ld,
                  st);
    if (kept_p > 0) {
      double* Wn = P->V.d() + (k + kept_p) * ld;
      gemm_tn(nh, kept_p, nw, MPc, ld, Wn, ld, s.C, s.ldc, s.part, st);
      gemm_nn_sub(nh, kept_p, nw, Pc, ld, s.C, s.ldc, Wn, ld, st);
      P->alg_bytes += 8.0 * nh * (2 * kept_p + 3 * nw);
    }
    k = P->k;
    W = P->V.d() + k * ld;
    MW = P->MV.d() + k * ld;
  }
  if (final_now) {
    // W's second pass (with the pending columns of P) and its Cholesky-QR;
    // its entry norms stay in the shared norm0 buffer
    OrthScratch s2 = orth_scratch(P);
    s2.V32 = nullptr;
    const int kept = orthonormalize_block(g, P->K, P->M, P->V.d(), P->MV.d(), ld, k, W, MW, ld,
                                          nw, defl, s2, idx, st, P->KV.d() + k * ld, true);
    P->alg_bytes += 2.0 * s2.cgs_passes * 8.0 * nh * k + 8.0 * 16.0 * nh * nw;
    consume_pending(P, s2);
    if (kept == 0) return 0;
    register_block(P, k, kept);
    return kept;
  }
  // provisional normalisation of W (one Cholesky-QR with deflation)
  stencil_apply(g, P->K, P->M, opsM, nw, W, ld, MW, ld, st);
  gemm_tn(nh, nw, nw, W, ld, MW, ld, s.G, 16, s.part, st);
  chol_deflate(nw, s.G, 16, s.norm0, defl, kBlockDefl, s.Rinv, s.info, st);
  apply_rinv(nh, nw, s.info, s.Rinv, W, nullptr, ld, nullptr, st);
  const CholInfo h = fetch_info();
  const int kept = h.kept;
  for (int j = 0; j < kept; ++j) idx[j] = h.idx[j];
  if (kept == 0) return 0;
  stencil_apply_km(g, P->K, P->M, kept, W, ld, P->KV.d() + k * ld, ld, MW, ld, st);
  // entry norms of the kept columns, the reference of the lagged pass
  gather_kept_kernel<<<1, 16, 0, st>>>(s.norm0, s.info, P->prov_norm0.d());
  STS_HIP(hipGetLastError());
  P->alg_bytes += 8.0 * nh * (6 * nw + 4 * kept);
  (void)kc;
  return kept;
}

// Form the reduced-matrix columns of the newest block now (before a reduced
// solve or Ritz values need them): [Kred Mred](:, new) = V^T [Kx W, Mx W] in
// one pass over V, then the mirrored rows.
void flush_pending(sts_problem* P) {
  if (P->pend_size <= 0) return;
  hipStream_t st = P->stream;
  const int64_t ps = P->pend_start, pk = P->pend_size, kn = ps + pk, kc = P->kcap, ld = P->ldv;
  gemm_tn2(P->nh, (int)kn, (int)pk, (int)pk, P->V.d(), ld, P->KV.d() + ps * ld,
           P->MV.d() + ps * ld, ld, P->Kred.d() + ps * kc, P->Mred.d() + ps * kc, kc,
           P->tn_part.d(), st);
  mirror((int)ps, (int)pk, P->Kred.d() + ps * kc, kc, P->Kred.d() + ps, kc, st);
  mirror((int)ps, (int)pk, P->Mred.d() + ps * kc, kc, P->Mred.d() + ps, kc, st);
  P->alg_bytes += 8.0 * P->nh * (kn + 2 * pk);
  P->pend_size = 0;
}

// Reduced solve on the first ks columns and projected residual with the block
// V[:, ks..ks+b).  Returns the relative projected residual (b = 0 -> 0).
double reduced_solve(sts_problem* P, int64_t ks, int64_t b) {
  hipStream_t st = P->stream;
  const int64_t kc = P->kcap, nt = P->nt;
  EigWork ew{};
  ew.base = P->eig_work.d();
  ew.status = static_cast<int*>(P->eig_meta.p);
  sym_eig((int)ks, P->Kred.d(), kc, P->lam.d(), P->Q.d(), kc, ew, st);
  gemm_tn(ks, (int)ks, P->p, P->Q.d(), kc, P->beta.d(), kc, P->qb.d(), kc, P->tn_part.d(), st);
  time_sweep((int)ks, (int)nt, P->p, P->lam.d(), P->qb.d(), kc, P->F2.d(), nt, time_ops(P),
             P->Z.d(), kc, st);
  gemm_nn((int)ks, (int)nt, (int)ks, P->Q.d(), kc, P->Z.d(), kc, P->Y.d(), kc, st);
  // One step of iterative refinement with the same eigendecomposition: its
  // backward error eps ||Km|| is large against the smallest eigenvalues,
  // which carry the smooth part of the solution.
  {
    const TimeOps t = time_ops(P);
    double* KY = P->RB.d();
    gemm_nn((int)ks, (int)nt, (int)ks, P->Kred.d(), kc, P->Y.d(), kc, KY, kc, st);
    reduced_residual((int)ks, (int)nt, P->p, P->beta.d(), kc, P->F2.d(), nt, KY, P->Y.d(), kc,
                     t, P->Z.d(), kc, st);
    gemm_small(true, (int)ks, (int)nt, (int)ks, 1.0, P->Q.d(), kc, P->Z.d(), kc, 0.0, KY, kc, st);
    time_sweep_full((int)ks, (int)nt, P->lam.d(), KY, kc, t, P->Z.d(), kc, st);
    gemm_small(false, (int)ks, (int)nt, (int)ks, 1.0, P->Q.d(), kc, P->Z.d(), kc, 1.0, P->Y.d(),
               kc, st);
  }
  double res2 = 0.0;
  if (b > 0) {
    // tau = Kred[ks:ks+b, 0:ks]; T1 = tau Y
    gemm_nn((int)b, (int)nt, (int)ks, P->Kred.d() + ks, kc, P->Y.d(), kc, P->T1.d(), 16, st);
    double* MWn = P->MV.d() + ks * P->ldv;
    gemm_tn(P->nh, (int)b, (int)b, MWn, P->ldv, MWn, P->ldv, P->gram.d(), 16, P->tn_part.d(), st);
    chol_lower((int)b, P->gram.d(), 16, P->Lb.d(), 16, static_cast<int*>(P->okflag.p), st);
    const TimeOps t = time_ops(P);
    cheap_residual((int)b, (int)nt, P->T1.d(), 16, P->Lb.d(), 16, t.m, t.n, P->smallv.d(),
                   P->res_part.d(), P->counter(0), st);
    P->alg_bytes += 8.0 * P->nh * b;
  }
  int status = 0;
  STS_HIP(hipMemcpyAsync(P->pinned, P->eig_meta.p, sizeof(int), hipMemcpyDeviceToHost, st));
  STS_HIP(hipStreamSynchronize(st));
  std::memcpy(&status, P->pinned, sizeof(int));
  STS_REQUIRE(status == 0, STS_E_NUMERIC, "reduced matrix is not finite");
  if (b > 0) fetch(P, P->smallv.d(), 1, &res2);
  ++P->checks;
  return std::sqrt(std::max(res2, 0.0)) / P->fnorm;
}

// ||A B^T||_F^2 for A = the column segments `segs` (mtot columns in all) and
// BT (Nt x mtot, ld Nt; overwritten when the QR path is taken), without
// forming the Nh x Nt product: directly, or through the Householder QR of BT
// (||A B^T|| = ||A R^T||) when that saves work.
double lowrank_norm2(sts_problem* P, const Seg* segs, int nseg, int mtot, double* BT) {
  hipStream_t st = P->stream;
  const int64_t nt = P->nt, ldbt = nt;
  bool use_qr = nt >= 2 * (int64_t)mtot && qr_r_supported(nt, mtot) && P->residual_qr >= 0;
  if (use_qr && P->residual_qr == 0) {
    // the direct product costs 2 Nh m Nt flops on the matrix cores, the QR
    // path 2 Nh m^2 flops plus about 60 us per 8-column panel (measured on
    // the MI355X); take it when it saves more than that at ~40 TFLOP/s
    const double saved = 2.0 * (double)P->nh * mtot * (double)(nt - mtot) / 40e12;
    use_qr = saved > (mtot / (double)kQrNb) * 60e-6;
  }
  if (use_qr) {
    // an Nh x mtot x mtot product instead of Nh x mtot x Nt
    const size_t wd = qr_r_work_doubles(nt, mtot);
    // a reallocation releases a block earlier kernels on the stream may use
    if (P->qr_work.bytes < wd * 8 || P->qr_R.bytes < (size_t)mtot * mtot * 8)
      STS_HIP(hipStreamSynchronize(st));
    if (P->qr_work.bytes < wd * 8) P->qr_work.alloc(wd * 8);
    if (P->qr_R.bytes < (size_t)mtot * mtot * 8) P->qr_R.alloc((size_t)mtot * mtot * 8);
    qr_r(nt, mtot, BT, ldbt, P->qr_R.d(), P->qr_work.d(), st);
    residual_norm2(P->nh, mtot, segs, nseg, P->qr_R.d(), mtot, P->smallv.d(), P->res_part.d(),
                   P->counter(1), st, true);
    P->alg_bytes += 8.0 * P->nh * mtot * ((mtot + 255) / 256);
  } else {
    residual_norm2(P->nh, (int)nt, segs, nseg, BT, ldbt, P->smallv.d(), P->res_part.d(),
                   P->counter(1), st);
    P->alg_bytes += 8.0 * P->nh * mtot * ((nt + 255) / 256);
  }
  double r2 = 0.0;
  fetch(P, P->smallv.d(), 1, &r2);
  return std::max(r2, 0.0);
}

// Exact relative residual ||F1 F2^T - Kx V Y Mt^T - Mx V Y Dt^T||_F / ||F||_F
// = ||[F1, Kx V, Mx V] [F2, -Mt Y^T, -Dt Y^T]^T||_F / ||F||_F.
double true_residual(sts_problem* P) {
  hipStream_t st = P->stream;
  const int64_t ks = P->k_sol, nt = P->nt, p = P->p;
  double* BT = P->BT.d();
  const int64_t ldbt = nt;
  copy_cols(nt, (int)p, P->F2.d(), nt, BT, ldbt, st);
  const TimeOps t = time_ops(P);
  bidiag_right((int)ks, (int)nt, P->Y.d(), P->kcap, t.m, t.n, -1.0, BT + p * ldbt, ldbt, st);
  bidiag_right((int)ks, (int)nt, P->Y.d(), P->kcap, t.d, t.e, -1.0, BT + (p + ks) * ldbt, ldbt,
               st);
  Seg segs[3] = {{P->F1.d(), P->ldv, (int)p}, {P->KV.d(), P->ldv, (int)ks},
                 {P->MV.d(), P->ldv, (int)ks}};
  const int nseg = ks > 0 ? 3 : 1;
  const int mtot = (int)(p + (ks > 0 ? 2 * ks : 0));
  return std::sqrt(lowrank_norm2(P, segs, nseg, mtot, BT)) / P->fnorm;
}

// ||Y||_F of the current solution: ||V Y|| in the Mx norm (V^T Mx V = I), a
// k x Nt reduction instead of a pass over V.
double y_fnorm(sts_problem* P) {
  if (P->k_sol == 0) return 0.0;
  double* part = P->res_part.d();
  sumsq(P->k_sol, (int)P->nt, P->Y.d(), P->kcap, part + 2048, part, P->counter(2), P->stream);
  double v = 0.0;
  fetch(P, part + 2048, 1, &v);
  return std::sqrt(std::max(v, 0.0));
}

// ||V Y||_F of the current solution.
double solution_fnorm(sts_problem* P) {
  const int64_t ks = P->k_sol;
  if (ks == 0) return 0.0;
  transpose((int)ks, (int)P->nt, P->Y.d(), P->kcap, P->BT.d(), P->nt, P->stream);
  Seg seg{P->V.d(), P->ldv, (int)ks};
  return std::sqrt(lowrank_norm2(P, &seg, 1, (int)ks, P->BT.d()));
}

// The exact residual is evaluated from the solution stored in FP64.  Rounding
// U's entries (relative u = 2^-53) alone moves the residual by
// Kx (delta o U) Mt^T + Mx (delta o U) Dt^T, whose expected Frobenius norm is
// u / sqrt(3) (||c_K|| rms(Mt) + ||c_M|| rms(Dt)) ||U||_F, with c_K, c_M the
// stencil coefficients and rms(A) the root mean square of the row norms of a
// time matrix.  Relative to ||F||, this grows like the condition number of
// Mx^{-1} Kx (about 1e-7 for the 1-D problem with 65535 nodes, where no FP64
// representation of the exact solution has a smaller residual).  The floor
// reported is kFloorFactor times that estimate, above what the rounded exact
// solution measures (about 3.5 times it).  The Galerkin solution adds the
// error of the reduced solve: the eigendecomposition of the order-k reduced
// matrix has a backward error near sqrt(k) u ||T|| (Householder reduction),
// which moves the small Ritz values, and so the slow modes of Y, by that
// much; the floor therefore grows like sqrt(k / kFloorCols) beyond
// kFloorCols basis columns (a 1-D solve with 29139 nodes stalls at about 46
// times the estimate with k = 600).
constexpr double kFloorFactor = 8.0;
constexpr double kFloorCols = 64.0;

double floor_growth(const sts_problem* P) {
  return std::max(1.0, std::sqrt((double)P->k_sol / kFloorCols));
}

double residual_floor(sts_problem* P) {
  return kFloorFactor * floor_growth(P) * P->floor_coef * solution_fnorm(P);
}

// Whether an exact residual res above tol is explained by the rounding floor:
// the floor must be at least tol / 2 (else the residual can still be resolved
// to tol) and res within tol + floor.  *floor receives the floor.
bool floor_accepts(sts_problem* P, double tol, double res, double* floor) {
  *floor = residual_floor(P);
  return *floor >= 0.5 * tol && res <= tol + *floor;
}

// Where the floor is at least tol / 2 the inner solves are as limited as the
// residual: a direct 1-D solve with tens of thousands of nodes returns its
// result with relative error near u kappa, so the new directions carry that
// rounding and the projected residual stalls above tol too.  A solve whose
// projected residual has not halved over kStallChecks checks is then accepted
// with an exact residual within tol + kStallFloor floor (floor_limited);
// otherwise it continues to max_outer.
constexpr int kStallChecks = 3;
constexpr double kStallFloor = 4.0;

void check_inner(const CGScal& s) {
  STS_REQUIRE(s.flag != 3, STS_E_NUMERIC,
              "inner CG broke down (non-positive curvature or non-finite value)");
  STS_REQUIRE(s.flag != 2, STS_E_NUMERIC, "inner CG reached its iteration cap");
}

// Inner solves of one block: x_j = A_j^{-1} b_j written to the next columns
// of V.  With the multigrid preconditioner the Mx columns are solved first
// (plain CG) and the Kx columns after them (preconditioned CG); perm[j] is the
// source column of result column j.  Otherwise all columns go through plain
// CG in their order.
// Inner solves of a rational Krylov step: (Kx + s Mx) x_c = b_c.  1-D: direct
// (elimination factors of the shifted matrix formed on the fly); otherwise
// CG on the shifted stencil (plain CG: the multigrid preconditioner is built
// for Kx alone).
// The multigrid's mass scale of level 0: the 2-D P1 mass is (h^2/12) times
// its pattern (centre 6), the 3-D Q1 mass (h/6)^3 times (1, 4, 1)^3 (centre 64).
double mass_scale(const Grid& g, const Stencil& M) {
  return g.dim == 3 ? M.c[13] / 64.0 : M.c[13] / 6.0;
}

void run_shifted_block(sts_problem* P, double s, int ncols, const double* const* b,
                       const sts_opts& o) {
  double* x0 = P->V.d() + (P->k + P->prov) * P->ldv;   // after a provisional block
  if (o.inner_precond != 0 && P->tri_ok) {
    // work: the CG residual vectors (2 kMaxCols columns of ldv), idle here
    tridiag_shifted_solve(P->grid, P->K, P->M, s, ncols, b, x0, P->ldv, P->cg.w.r[0], P->ldv,
                          2 * P->ldv * kMaxCols, P->stream);
    P->inner_K += ncols;
    P->alg_bytes += 40.0 * P->nh * ncols;
    return;
  }
  if (o.inner_precond != 0 && P->mg_ok) {
    // multigrid-preconditioned CG on Kx + s Mx (every level's operator gets
    // the mass term; see mg.hip and mg3.hip)
    if (!P->mg) {
      P->mg = std::make_unique<MGRunner>();
      P->mg->setup(P->mg_plan_);
    }
    MGRunner& r = *P->mg;
    const int e = r.expect;
    r.w.plan.sw0 = s * mass_scale(P->grid, P->M);
    r.w.plan.f32 = o.precond_fp32;
    r.expect = r.expect_shifted;
    CGScal out[kMaxCols];
    try {
      r.run(x0, P->ldv, ncols, b, o.inner_rtol, o.inner_maxit, out, P->stream);
    } catch (...) {
      r.w.plan.sw0 = 0.0;
      r.expect_shifted = r.expect;
      r.expect = e;
      throw;
    }
    r.w.plan.sw0 = 0.0;
    r.expect_shifted = r.expect;
    r.expect = e;
    const double bpn = r.bytes_per_node();
    for (int j = 0; j < ncols; ++j) {
      check_inner(out[j]);
      P->inner_K += out[j].iters;
      P->alg_bytes += (bpn * (out[j].iters + 1) + 40.0) * P->nh;
    }
    return;
  }
  // Kx + s Mx has the pattern of Mx (a superset of that of Kx): it runs in
  // the operator slot of Mx
  Stencil S = P->M;
  for (int i = 0; i < 27; ++i) S.c[i] = P->K.c[i] + s * P->M.c[i];
  const Stencil M0 = P->cg.M;
  const int e0 = P->cg.expect[0], e1 = P->cg.expect[1];
  P->cg.M = S;
  P->cg.expect[0] = P->cg.expect[1] = 0;
  int ops[kMaxCols];
  for (int c = 0; c < ncols; ++c) ops[c] = STS_OP_M;
  CGScal out[kMaxCols];
  P->cg.w.x = x0;
  P->cg.w.ld = P->ldv;
  auto restore = [&] {
    P->cg.M = M0;
    P->cg.expect[0] = e0;
    P->cg.expect[1] = e1;
  };
  try {
    P->cg.run(ops, ncols, b, o.inner_rtol, o.inner_maxit, out, P->stream);
  } catch (...) {
    restore();
    throw;
  }
  restore();
  for (int j = 0; j < ncols; ++j) {
    check_inner(out[j]);
    P->inner_K += out[j].iters;
    P->alg_bytes += (48.0 * out[j].iters + 32.0) * P->nh;
  }
}

// Greedy shift for real spectra (Druskin and Simoncini 2011, the adaptive
// choice Sec. 4 refers to): the maximiser over a logarithmic grid of [a, b]
// of prod_l |s - s_l| / prod_i |s + theta_i|, evaluated in logarithms.
double adaptive_shift(const double* ritz, int k, const double* shifts, int m, double a, double b,
                      int grid) {
  STS_REQUIRE(a > 0.0 && b >= a && grid >= 2 && k >= 0 && m >= 0, STS_E_INVALID,
              "adaptive shift: need 0 < a <= b, grid >= 2");
  const double la = std::log(a), step = (std::log(b) - la) / (grid - 1);
  double best = -std::numeric_limits<double>::infinity(), sbest = a;
  for (int g = 0; g < grid; ++g) {
    const double sv = g == 0 ? a : (g == grid - 1 ? b : std::exp(la + step * g));
    double f = 0.0;
    for (int l = 0; l < m; ++l) f += std::log(std::fabs(sv - shifts[l]) + 1e-300);
    for (int i = 0; i < k; ++i) f -= std::log(std::fabs(sv + ritz[i]));
    if (f > best) {
      best = f;
      sbest = sv;
    }
  }
  return sbest;
}

// Eigenvalues of the reduced pencil (Km, I) of the first k columns (host).
void ritz_values(sts_problem* P, int64_t k, std::vector<double>& out) {
  EigWork ew{};
  ew.base = P->eig_work.d();
  ew.status = static_cast<int*>(P->eig_meta.p);
  // the shift rule needs the Ritz values only
  sym_eigvals((int)k, P->Kred.d(), P->kcap, P->lam.d(), ew, P->stream);
  out.resize(k);
  STS_HIP(hipMemcpyAsync(out.data(), P->lam.d(), k * sizeof(double), hipMemcpyDeviceToHost,
                         P->stream));
  STS_HIP(hipStreamSynchronize(P->stream));
  for (double v : out) STS_REQUIRE(std::isfinite(v), STS_E_NUMERIC, "Ritz values not finite");
}

// Kx x_j = b[j] for j < nk by multigrid-preconditioned CG, x_j at x + j * ldv.
// Mixed-precision Kx solves (opts.mixed, 3-D grids with a smoothed level):
// iterative refinement with FP32 multigrid PCG as the correction solver.
// x = 0, r = b; each round solves K d = r by PCG with FP32 vectors to the
// relative tolerance max(target / ||r||, kF32ReplacedRtol), then in FP64
// x += d and r = b - K x, until ||r|| <= target = rtol ||b||.  Within a round
// d accumulates in FP64 and the FP32 residual is replaced by r - K d every
// kReplaceEvery iterations (residual replacement, as in reliable-update CG):
// the recursion cannot drift from the true residual by more than a few
// iterations' rounding, so one round usually meets the whole target and CG
// keeps its search directions.  A round that does not reduce ||r|| by
// kF32MinGain (the FP32 solve stalled or broke down in rounding) ends the
// FP32 rounds of that column and FP64 PCG solves for the rest.
constexpr double kF32MinGain = 0.1;
constexpr int kF32MaxRounds = 6;
constexpr int kReplaceEvery = 3;
constexpr double kF32ReplacedRtol = 1e-12;

bool mixed_applies(const sts_problem* P, const sts_opts& o) {
  return o.mixed != 0 && P->mg_ok && P->mg_plan_.dim == 3 && P->mg_plan_.nlev >= 1;
}
// The parts of the mixed mode: 1 = both, 2 = the Kx solves only, 3 = the
// Gram-Schmidt pass only.
bool mixed_inner(const sts_problem* P, const sts_opts& o) {
  return mixed_applies(P, o) && o.mixed != 3;
}
bool mixed_gs(const sts_problem* P, const sts_opts& o) {
  return mixed_applies(P, o) && o.mixed != 2;
}

struct RefineCount {
  int64_t its32 = 0, its64 = 0, rounds = 0;
  double bytes = 0.0;   // algorithmic bytes
};

// K x_j = b_j (j < nk, x_j at x + j * ldx, zeroed here) by the refinement
// above, on the multigrid runner r of a 3-D plan with a smoothed level.
void refined_kx_solve(MGRunner& r, int64_t nh, int nk, const double* const* b, double* x,
                      int64_t ldx, double rtol, int maxit, int precond_fp32, RefineCount& cnt,
                      hipStream_t st) {
  const int64_t ld0 = r.w.ld[0];
  if (!r.corr.p) {
    r.corr.alloc(ld0 * kMaxCols * 8);     // FP32 d (packed) or the FP64 finishing correction
    r.defect.alloc(ld0 * kMaxCols * 8);   // FP64 residuals b - K x
    r.norms.alloc(kMaxCols * 8);
  }
  double* d64 = r.corr.d();   // a round's correction, FP64 (packed columns)
  for (int j = 0; j < nk; ++j) fill(x + j * ldx, nh, 0.0, st);
  const double bpn32 = [&] {
    MGPlan q = r.w.plan;
    q.f32 = 0;
    q.f32cg = 1;
    q.x64 = 1;
    return mg3_bytes_per_node(q);
  }();
  const double nn = (double)nh;
  auto norms = [&](int n, double* out) {
    STS_HIP(hipMemcpyAsync(out, r.norms.d(), n * sizeof(double), hipMemcpyDeviceToHost, st));
    STS_HIP(hipStreamSynchronize(st));
  };
  std::vector<double> bnorm(nk, 0.0), rnorm(nk, 0.0), target(nk, 0.0);
  std::vector<int> act, fin;   // columns still in FP32 rounds / for the FP64 finish
  for (int j = 0; j < nk; ++j) act.push_back(j);
  CGScal out[kMaxCols];
  const int saved_f32 = r.w.plan.f32;
  auto restore = [&](int e) {
    r.w.plan.f32 = saved_f32;
    r.w.plan.f32cg = 0;
    r.w.plan.x64 = 0;
    r.w.col_rtol = nullptr;
    r.expect32 = r.expect;
    r.expect = e;
  };
  for (int round = 0; !act.empty(); ++round) {
    const int na = (int)act.size();
    const double* in[kMaxCols];
    double rt[kMaxCols];
    for (int s = 0; s < na; ++s) {
      const int j = act[s];
      in[s] = round == 0 ? b[j] : r.defect.d() + j * ld0;
      rt[s] = round == 0 ? std::max(rtol, kF32ReplacedRtol)
                         : std::max(target[j] / std::max(rnorm[j], 1e-300), kF32ReplacedRtol);
    }
    // FP32 PCG on the active columns, packed (slot s -> column s of d64),
    // its correction accumulated in FP64 and its residual replaced from it
    r.w.plan.f32 = 0;
    r.w.plan.f32cg = 1;
    r.w.plan.x64 = 1;
    r.w.col_rtol = rt;
    const int e = r.expect;
    r.expect = r.expect32;
    try {
      r.run(d64, ld0, na, in, kF32ReplacedRtol, maxit, out, st, kReplaceEvery);
    } catch (...) {
      restore(e);
      throw;
    }
    restore(e);
    for (int s = 0; s < na; ++s) {
      cnt.its32 += out[s].iters;
      cnt.bytes += (bpn32 * (out[s].iters + 1) + 16.0 + 20.0 * out[s].iters / kReplaceEvery) * nn;
      if (round == 0) {
        // ||b|| from the FP32 set-up's (b, b): enough for a tolerance
        bnorm[act[s]] = std::sqrt(std::max(out[s].gamma0, 0.0));
        target[act[s]] = rtol * bnorm[act[s]];
      }
    }
    // FP64: x += d, r = b - K x, (r, r)
    double* xs[kMaxCols];
    const void* ds[kMaxCols];
    const double* bs[kMaxCols];
    double* rs[kMaxCols];
    for (int s = 0; s < na; ++s) {
      const int j = act[s];
      xs[s] = x + j * ldx;
      // a column whose FP32 solve broke down contributes no correction
      ds[s] = out[s].flag == 3 ? nullptr : static_cast<const void*>(d64 + s * ld0);
      bs[s] = b[j];
      rs[s] = r.defect.d() + j * ld0;
    }
    mg3_defect(r.w, na, xs, ds, false, bs, rs, r.norms.d(), st);
    ++cnt.rounds;
    cnt.bytes += 48.0 * nn * na;
    double n2[kMaxCols];
    norms(na, n2);
    std::vector<int> next;
    for (int s = 0; s < na; ++s) {
      const int j = act[s];
      const double rn = std::sqrt(std::max(n2[s], 0.0));
      STS_REQUIRE(std::isfinite(rn), STS_E_NUMERIC,
                  "mixed-precision inner solve: non-finite residual");
      const double prev = round == 0 ? bnorm[j] : rnorm[j];
      rnorm[j] = rn;
      if (rn <= target[j]) continue;
      if (rn > kF32MinGain * prev || round + 1 >= kF32MaxRounds || out[s].flag >= 2)
        fin.push_back(j);
      else
        next.push_back(j);
    }
    act.swap(next);
  }
  if (fin.empty()) return;
  // FP64 PCG for the rest of the correction: K e = r, x += e
  const int nf = (int)fin.size();
  const double* in[kMaxCols];
  double rt[kMaxCols];
  for (int s = 0; s < nf; ++s) {
    in[s] = r.defect.d() + fin[s] * ld0;
    rt[s] = std::max(target[fin[s]] / std::max(rnorm[fin[s]], 1e-300), rtol);
  }
  r.w.plan.f32 = precond_fp32;
  r.w.col_rtol = rt;
  try {
    r.run(r.corr.d(), ld0, nf, in, rtol, maxit, out, st);
  } catch (...) {
    r.w.plan.f32 = saved_f32;
    r.w.col_rtol = nullptr;
    throw;
  }
  r.w.plan.f32 = saved_f32;
  r.w.col_rtol = nullptr;
  const double bpn = r.bytes_per_node();
  double* xs[kMaxCols];
  const void* ds[kMaxCols];
  const double* bs[kMaxCols];
  double* rs[kMaxCols];
  for (int s = 0; s < nf; ++s) {
    check_inner(out[s]);
    cnt.its64 += out[s].iters;
    cnt.bytes += (bpn * (out[s].iters + 1) + 40.0) * nn;
    xs[s] = x + fin[s] * ldx;
    ds[s] = r.corr.d() + s * ld0;
    bs[s] = b[fin[s]];
    rs[s] = r.defect.d() + fin[s] * ld0;
  }
  mg3_defect(r.w, nf, xs, ds, false, bs, rs, r.norms.d(), st);
  ++cnt.rounds;
  cnt.bytes += 48.0 * nn * nf;
}

void run_mg_k_mixed(sts_problem* P, int nk, const double* const* b, double* x, const sts_opts& o) {
  RefineCount c;
  refined_kx_solve(*P->mg, P->nh, nk, b, x, P->ldv, o.inner_rtol, o.inner_maxit, o.precond_fp32,
                   c, P->stream);
  P->inner_K += c.its32 + c.its64;
  P->inner_K32 += c.its32;
  P->defect_rounds += c.rounds;
  P->alg_bytes += c.bytes;
}

void run_mg_k(sts_problem* P, int nk, const double* const* b, double* x, const sts_opts& o) {
  if (!P->mg) {
    P->mg = std::make_unique<MGRunner>();
    P->mg->setup(P->mg_plan_);
  }
  if (mixed_inner(P, o)) return run_mg_k_mixed(P, nk, b, x, o);
  CGScal out[kMaxCols];
  P->mg->w.plan.f32 = o.precond_fp32;
  P->mg->run(x, P->ldv, nk, b, o.inner_rtol, o.inner_maxit, out, P->stream);
  const double bpn = P->mg->bytes_per_node();
  for (int j = 0; j < nk; ++j) {
    check_inner(out[j]);
    P->inner_K += out[j].iters;
    P->alg_bytes += (bpn * (out[j].iters + 1) + 40.0) * P->nh;
  }
}

void run_cg_block(sts_problem* P, const int* ops, int ncols, const double* const* b,
                  const sts_opts& o, int* perm) {
  for (int c = 0; c < ncols; ++c) perm[c] = c;
  double* x0 = P->V.d() + (P->k + P->prov) * P->ldv;   // after a provisional block
  if (o.inner_precond != 0 && P->tri_ok) {
    // 1-D: Kx and Mx are tridiagonal; solve every column directly
    tridiag_solve(P->grid, P->K, P->M, ops, ncols, b, x0, P->ldv, P->tri_fac.d(), P->stream);
    for (int c = 0; c < ncols; ++c) {
      if (ops[c] == STS_OP_K) ++P->inner_K;
      else ++P->inner_M;
    }
    P->alg_bytes += 32.0 * P->nh * ncols;
    return;
  }
  if (o.inner_precond != 0 && P->tensor_mass) {
    // 3-D trilinear mass: Mx columns directly, Kx columns by multigrid PCG
    // (plain CG on grids that do not halve)
    int nm = 0, nk = 0;
    for (int c = 0; c < ncols; ++c)
      if (ops[c] == STS_OP_M) perm[nm++] = c;
    for (int c = 0; c < ncols; ++c)
      if (ops[c] == STS_OP_K) perm[nm + nk++] = c;
    const double* b2[kMaxCols];
    for (int j = 0; j < ncols; ++j) b2[j] = b[perm[j]];
    if (nm > 0) {
      tensor_mass_solve(P->grid, P->M, nm, b2, x0, P->ldv, P->tmass_fac.d(), P->stream);
      P->inner_M += nm;
      P->alg_bytes += 48.0 * P->nh * nm;
    }
    if (nk > 0 && P->mg_ok) {
      run_mg_k(P, nk, b2 + nm, x0 + nm * P->ldv, o);
    } else if (nk > 0) {
      int ops2[kMaxCols];
      for (int j = 0; j < nk; ++j) ops2[j] = STS_OP_K;
      CGScal out[kMaxCols];
      P->cg.w.x = x0 + nm * P->ldv;
      P->cg.w.ld = P->ldv;
      P->cg.run(ops2, nk, b2 + nm, o.inner_rtol, o.inner_maxit, out, P->stream);
      for (int j = 0; j < nk; ++j) {
        check_inner(out[j]);
        P->inner_K += out[j].iters;
        P->alg_bytes += (48.0 * out[j].iters + 32.0) * P->nh;
      }
    }
    return;
  }
  const bool use_mg = o.inner_precond != 0 && P->mg_ok;
  int nm = 0, nk = 0;
  if (use_mg) {
    for (int c = 0; c < ncols; ++c)
      if (ops[c] == STS_OP_M) perm[nm++] = c;
    for (int c = 0; c < ncols; ++c)
      if (ops[c] == STS_OP_K) perm[nm + nk++] = c;
  }
  if (use_mg && nm > 0 && P->mass_cheb) {
    // Mx columns: Chebyshev iteration with the analytic spectral bounds
    const double* b2[kMaxCols];
    for (int j = 0; j < nm; ++j) b2[j] = b[perm[j]];
    const int its = mass_cheb_iters(o.inner_rtol);
    double* xb[2] = {P->cg.w.r[0], P->cg.w.r[1]};
    double* db[2] = {P->cg.w.p[0], P->cg.w.p[1]};
    mass_cheb_solve(P->grid, P->M, nm, b2, x0, P->ldv, xb, db, P->ldv, its, P->stream);
    P->inner_M += (int64_t)its * nm;
    const int launches = (its + kMassSteps - 1) / kMassSteps;
    P->alg_bytes += 40.0 * launches * P->nh * nm;
  } else if (!use_mg || nm > 0) {
    const int n = use_mg ? nm : ncols;
    int ops2[kMaxCols];
    const double* b2[kMaxCols];
    for (int j = 0; j < n; ++j) {
      ops2[j] = ops[perm[j]];
      b2[j] = b[perm[j]];
    }
    CGScal out[kMaxCols];
    P->cg.w.x = x0;
    P->cg.w.ld = P->ldv;
    P->cg.run(ops2, n, b2, o.inner_rtol, o.inner_maxit, out, P->stream);
    for (int j = 0; j < n; ++j) {
      check_inner(out[j]);
      if (ops2[j] == STS_OP_K) P->inner_K += out[j].iters;
      else P->inner_M += out[j].iters;
      P->alg_bytes += (48.0 * out[j].iters + 32.0) * P->nh;
    }
  }
  if (use_mg && nk > 0) {
    const double* b2[kMaxCols];
    for (int j = 0; j < nk; ++j) b2[j] = b[perm[nm + j]];
    run_mg_k(P, nk, b2, x0 + nm * P->ldv, o);
  }
}

int64_t numerical_rank(sts_problem* P) {
  // V is Mx-orthonormal, so the singular values of V Y in the Mx norm are those
  // of Y: eigenvalues of Y Y^T (reuses the eigen workspace; Kred untouched).
  hipStream_t st = P->stream;
  const int64_t ks = P->k_sol, nt = P->nt, kc = P->kcap;
  if (ks == 0) return 0;
  transpose((int)ks, (int)nt, P->Y.d(), kc, P->Z.d(), nt, st);   // Z <- Y^T (nt x ks)
  DevBuf gy;
  gy.alloc(ks * ks * 8);
  gemm_nn((int)ks, (int)ks, (int)nt, P->Y.d(), kc, P->Z.d(), nt, gy.d(), ks, st);
  EigWork ew{};
  ew.base = P->eig_work.d();
  ew.status = static_cast<int*>(P->eig_meta.p);
  DevBuf qtmp;
  qtmp.alloc(ks * ks * 8);
  DevBuf ltmp;
  ltmp.alloc(ks * 8);
  sym_eig((int)ks, gy.d(), ks, ltmp.d(), qtmp.d(), ks, ew, st);
  std::vector<double> ev(ks);
  STS_HIP(hipMemcpyAsync(ev.data(), ltmp.p, ks * 8, hipMemcpyDeviceToHost, st));
  STS_HIP(hipStreamSynchronize(st));
  double mx = 0.0;
  for (double v : ev) mx = std::max(mx, v);
  int64_t r = 0;
  for (double v : ev)
    if (v > 1e-16 * mx) ++r;   // sigma_i > 1e-8 sigma_1
  // Y was overwritten only in Z (scratch): the solution stays in P->Y.
  return r;
}

double orth_error(sts_problem* P) {
  const int64_t ks = P->k_sol, kc = P->kcap;
  if (ks == 0) return 0.0;
  std::vector<double> m(kc * ks);
  STS_HIP(hipMemcpyAsync(m.data(), P->Mred.p, kc * ks * 8, hipMemcpyDeviceToHost, P->stream));
  STS_HIP(hipStreamSynchronize(P->stream));
  double e = 0.0;
  for (int64_t j = 0; j < ks; ++j)
    for (int64_t i = 0; i < ks; ++i) e = std::max(e, std::fabs(m[i + j * kc] - (i == j ? 1.0 : 0.0)));
  return e;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

namespace {
sts_status run_guarded(const std::function<void()>& f) {
  try {
    g_last_error.clear();
    f();
    return STS_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return STS_E_NOMEM;
  } catch (...) {
    set_error("unexpected exception");
    return STS_E_DEVICE;
  }
}

void check_finite(const double* h, int64_t rows, int64_t cols, int64_t ld, const char* what) {
  for (int64_t j = 0; j < cols; ++j)
    for (int64_t i = 0; i < rows; ++i)
      STS_REQUIRE(std::isfinite(h[i + j * ld]), STS_E_INVALID, std::string(what) + " is not finite");
}
}  // namespace

namespace {
// Multigrid plan of a space (STS_E_INVALID if the grid does not allow one).
MGPlan require_mg(const sts_space* space, Grid* g) {
  validate_space(space);
  *g = make_grid(*space);
  MGPlan plan{};
  STS_REQUIRE(mg_plan(*g, make_stencil(*space, STS_OP_K), &plan), STS_E_INVALID,
              "multigrid needs a 2-D P1 or 3-D seven-point space whose n halves, n -> (n-1)/2, down to <= 63");
  return plan;
}

// Multigrid plan of a space for the mixed-precision V-cycle (STS_E_INVALID
// where it does not apply: 2-D spaces and 3-D grids without a smoothed level).
MGPlan require_mg_mixed(const sts_space* space, double shift, Grid* g) {
  MGPlan plan = require_mg(space, g);
  STS_REQUIRE(plan.dim == 3 && plan.nlev >= 1, STS_E_INVALID,
              "the FP32 V-cycle needs a 3-D seven-point space with n > 63 (at least one smoothed level)");
  STS_REQUIRE(shift >= 0.0 && std::isfinite(shift), STS_E_INVALID, "shift must be >= 0");
  plan.sw0 = shift * mass_scale(*g, make_stencil(*space, STS_OP_M));
  plan.f32 = 1;
  return plan;
}

sts_status cg_status(const CGScal* out, int ncols, int32_t* iters) {
  sts_status bad = STS_OK;
  for (int c = 0; c < ncols; ++c) {
    if (iters) iters[c] = out[c].iters;
    if (out[c].flag == 3) bad = STS_E_NUMERIC;
    else if (out[c].flag == 2 && bad == STS_OK) bad = STS_E_NOT_CONVERGED;
  }
  return bad;
}
}  // namespace

// Hooks for the executors in pool.hip.
namespace sts {

sts_status guarded(const std::function<void()>& f) { return run_guarded(f); }

hipStream_t problem_stream(const sts_problem* P) { return P->stream; }

void problem_bind_stream(sts_problem* P, hipStream_t s) {
  if (P->stream == s) return;
  STS_HIP(hipStreamSynchronize(P->stream));
  P->stream = s;
}

int64_t problem_footprint(const sts_space& space, int64_t nt, int p, int max_outer, bool mixed) {
  const Grid g = make_grid(space);
  const Stencil K = make_stencil(space, STS_OP_K);
  const Stencil M = make_stencil(space, STS_OP_M);
  const int64_t ld = pad_ld(g.nh);
  const int64_t kc = initial_capacity(p, max_outer);   // the capacity sts_solve allocates first
  int64_t b = 0;
  b += ld * p * 8 + nt * p * 8 + 4 * nt * 8;                       // F1, F2, time matrices
  b += 2 * 2 * ld * kMaxCols * 8 + 2 * ld * kMaxCols * 8;          // CG r, p; residual work
  MGPlan plan{};
  const bool mg = mg_plan(g, K, &plan);
  const bool mixed32 = mixed && mg && plan.dim == 3 && plan.nlev >= 1;
  b += basis_capacity_bytes(ld, nt, p, kc, mixed32);
  b += gemm_tn_partial_size(std::max<int64_t>(g.nh, nt), (int)kc) * 8;
  b += residual_norm2_partial_size(g.nh, (int)nt) * 8;
  if (mg) b += 9 * ld * kMaxCols * 8 + (int64_t)plan.exact * (plan.exact + 1) * 8;
  if (mixed32) b += 2 * ld * kMaxCols * 8;                       // refinement buffers
  if (tridiag_supported(g, K, M)) b += tridiag_factor_doubles(g.nh) * 8;
  if (tensor_mass_supported(g, M)) b += 2 * g.nx * 8;
  return b + (1 << 20);                                            // small scratch
}

int64_t problem_growth_bytes(const sts_space& space, int64_t nt, int p, int64_t cols) {
  const Grid g = make_grid(space);
  return basis_capacity_bytes(pad_ld(g.nh), nt, p, cols, false) -
         basis_capacity_bytes(pad_ld(g.nh), nt, p, 0, false);
}

void problem_set_grow_hook(sts_problem* P, std::function<void(int64_t)> hook) {
  P->grow_hook = std::move(hook);
}

double problem_cost(const sts_problem* P) {
  // inner solves dominate: grid size x columns x (log of the grid size, a
  // proxy for the outer iteration count), plus the reduced work along time
  const double nh = (double)P->nh;
  return P->p * (nh * std::log2(nh + 2.0) + 64.0 * (double)P->nt);
}

}  // namespace sts

extern "C" {

void sts_default_opts(sts_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-8;
  o->max_outer = 200;
  o->check_every = 0;
  o->inner_rtol = 1e-13;
  o->inner_maxit = 200000;
  o->verify_true = 1;
  o->defl_tol = 1e-10;
  o->mem_budget = 0;
  o->restart = 0;
  o->profile = 0;
  o->inner_precond = 1;
  o->orth_lag = 1;
}

const char* sts_last_error(void) { return g_last_error.c_str(); }

sts_status sts_time_matrices(int64_t nt, const double* t, double* dd, double* ds, double* md,
                             double* ms) {
  return run_guarded([&] {
    STS_REQUIRE(nt >= 1 && t && dd && md && (nt == 1 || (ds && ms)), STS_E_INVALID,
                "sts_time_matrices: bad arguments");
    for (int64_t l = 0; l < nt; ++l)
      STS_REQUIRE(std::isfinite(t[l]) && std::isfinite(t[l + 1]) && t[l + 1] > t[l],
                  STS_E_INVALID, "time nodes must be finite and strictly increasing");
    // On I^l the hat sigma^l rises from 0 to 1 and sigma^{l-1} falls from 1 to 0:
    // (d/dt sigma^l, tau^l) = 1, (d/dt sigma^{l-1}, tau^l) = -1, and both hats
    // integrate to |I^l| / 2 over I^l.
    for (int64_t l = 0; l < nt; ++l) {
      const double len = t[l + 1] - t[l];
      dd[l] = 1.0;
      md[l] = 0.5 * len;
      if (l > 0) {
        ds[l - 1] = -1.0;
        ms[l - 1] = 0.5 * len;
      }
    }
  });
}

sts_status sts_create(const sts_space* space, const sts_bidiag* Dt, const sts_bidiag* Mt,
                      int64_t nt, int32_t p, const double* F1, int64_t ldf1, const double* F2,
                      int64_t ldf2, int32_t mem, void* stream, sts_problem** out) {
  return run_guarded([&] {
    STS_REQUIRE(out != nullptr, STS_E_INVALID, "out is NULL");
    *out = nullptr;
    validate_space(space);
    STS_REQUIRE(Dt && Mt && Dt->diag && Mt->diag, STS_E_INVALID, "time matrices are NULL");
    STS_REQUIRE(nt >= 2, STS_E_INVALID, "nt must be >= 2");
    STS_REQUIRE(Dt->sub && Mt->sub, STS_E_INVALID, "time sub-diagonals are NULL");
    STS_REQUIRE(p >= 1 && p <= 4, STS_E_INVALID, "p must be in 1..4");
    STS_REQUIRE(F1 && F2, STS_E_INVALID, "F1 / F2 is NULL");
    STS_REQUIRE(mem == STS_MEM_HOST || mem == STS_MEM_DEVICE, STS_E_INVALID, "bad mem kind");
    const Grid g = make_grid(*space);
    STS_REQUIRE(ldf1 >= g.nh && ldf2 >= nt, STS_E_INVALID, "leading dimension too small");
    for (int64_t l = 0; l < nt; ++l) {
      STS_REQUIRE(std::isfinite(Dt->diag[l]) && Dt->diag[l] > 0.0 && std::isfinite(Mt->diag[l]) &&
                      Mt->diag[l] > 0.0,
                  STS_E_INVALID, "time matrices need positive, finite diagonals");
      if (l + 1 < nt)
        STS_REQUIRE(std::isfinite(Dt->sub[l]) && std::isfinite(Mt->sub[l]), STS_E_INVALID,
                    "time sub-diagonals must be finite");
    }
    if (mem == STS_MEM_HOST) {
      check_finite(F1, g.nh, p, ldf1, "F1");
      check_finite(F2, nt, p, ldf2, "F2");
    }
    auto P = std::make_unique<sts_problem>();
    P->space = *space;
    P->grid = g;
    P->K = make_stencil(*space, STS_OP_K);
    P->M = make_stencil(*space, STS_OP_M);
    P->nh = g.nh;
    P->nt = nt;
    P->p = p;
    P->ldv = pad_ld(g.nh);
    P->stream = static_cast<hipStream_t>(stream);
    hipStream_t st = P->stream;
    P->h_td.assign(Dt->diag, Dt->diag + nt);
    P->h_ts.assign(Dt->sub, Dt->sub + nt - 1);
    P->h_md.assign(Mt->diag, Mt->diag + nt);
    P->h_ms.assign(Mt->sub, Mt->sub + nt - 1);
    // inputs
    P->F1.alloc(P->ldv * p * 8);
    P->F2.alloc(nt * p * 8);
    if (mem == STS_MEM_HOST) {
      STS_HIP(hipMemcpy2DAsync(P->F1.p, P->ldv * 8, F1, ldf1 * 8, g.nh * 8, p,
                               hipMemcpyHostToDevice, st));
      STS_HIP(hipMemcpy2DAsync(P->F2.p, nt * 8, F2, ldf2 * 8, nt * 8, p, hipMemcpyHostToDevice, st));
    } else {
      copy_cols(g.nh, p, F1, ldf1, P->F1.d(), P->ldv, st);
      copy_cols(nt, p, F2, ldf2, P->F2.d(), nt, st);
    }
    std::vector<double> tv(4 * nt, 0.0);
    for (int64_t l = 0; l < nt; ++l) {
      tv[l] = P->h_td[l];
      tv[2 * nt + l] = P->h_md[l];
      if (l + 1 < nt) {
        tv[nt + l] = P->h_ts[l];
        tv[3 * nt + l] = P->h_ms[l];
      }
    }
    P->tdv.alloc(4 * nt * 8);
    STS_HIP(hipMemcpyAsync(P->tdv.p, tv.data(), 4 * nt * 8, hipMemcpyHostToDevice, st));
    // CG work
    const int tiles = cg_tiles(g);
    P->cg_r.alloc(2 * P->ldv * kMaxCols * 8);
    P->cg_p.alloc(2 * P->ldv * kMaxCols * 8);
    P->cg_scal.alloc(sizeof(CGScal) * 2 * kMaxCols);
    P->cg_part.alloc((size_t)2 * 2 * kMaxCols * tiles * 8);
    P->counters.alloc(64);
    STS_HIP(hipMemsetAsync(P->counters.p, 0, 64, st));
    P->cg.g = g;
    P->cg.K = P->K;
    P->cg.M = P->M;
    P->cg.w.r[0] = P->cg_r.d();
    P->cg.w.r[1] = P->cg_r.d() + P->ldv * kMaxCols;
    P->cg.w.p[0] = P->cg_p.d();
    P->cg.w.p[1] = P->cg_p.d() + P->ldv * kMaxCols;
    P->cg.w.scal = static_cast<CGScal*>(P->cg_scal.p);
    P->cg.w.partials = P->cg_part.d();
    P->cg.w.max_tiles = tiles;
    P->cg.poll.init();
    STS_HIP(hipHostMalloc(reinterpret_cast<void**>(&P->pinned), 64 * 8, hipHostMallocDefault));
    P->mg_ok = mg_plan(g, P->K, &P->mg_plan_);
    P->mass_cheb = mass_cheb_supported(g, P->M);
    P->tensor_mass = tensor_mass_supported(g, P->M);
    if (P->tensor_mass) {
      P->tmass_fac.alloc(2 * g.nx * 8);
      tensor_mass_factor(g.nx, P->tmass_fac.d(), st);
    }
    P->tri_ok = tridiag_supported(g, P->K, P->M);
    if (P->tri_ok) {
      P->tri_fac.alloc(tridiag_factor_doubles(g.nh) * 8);
      tridiag_factor(g, P->K, P->M, P->tri_fac.d(), st);
    }
    // small scratch
    P->gram.alloc(16 * 16 * 8);
    P->rinv.alloc(16 * 16 * 8);
    P->cinfo.alloc(sizeof(CholInfo));
    P->norm0.alloc(16 * 8);
    P->prov_norm0.alloc(16 * 8);
    P->Lb.alloc(16 * 16 * 8);
    P->T1.alloc(16 * nt * 8);
    P->okflag.alloc(16);
    P->res_part.alloc(std::max<int64_t>(residual_norm2_partial_size(g.nh, (int)nt), 4096) * 8);
    // ||F1 F2^T||_F^2 = trace((F1^T F1)(F2^T F2))
    P->tn_part.alloc(gemm_tn_partial_size(std::max<int64_t>(g.nh, nt), 16) * 8);
    double* G1 = P->gram.d();
    double* G2 = P->rinv.d();
    gemm_tn(g.nh, p, p, P->F1.d(), P->ldv, P->F1.d(), P->ldv, G1, 16, P->tn_part.d(), st);
    gemm_tn(nt, p, p, P->F2.d(), nt, P->F2.d(), nt, G2, 16, P->tn_part.d(), st);
    double h1[256], h2[256];
    STS_HIP(hipMemcpyAsync(h1, G1, 256 * 8, hipMemcpyDeviceToHost, st));
    STS_HIP(hipMemcpyAsync(h2, G2, 256 * 8, hipMemcpyDeviceToHost, st));
    STS_HIP(hipStreamSynchronize(st));
    double tr = 0.0;
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j) tr += h1[i + 16 * j] * h2[j + 16 * i];
    P->fnorm = std::sqrt(std::max(tr, 0.0));
    STS_REQUIRE(std::isfinite(P->fnorm), STS_E_INVALID, "F1 or F2 is not finite");
    {
      // coefficient of the FP64 rounding floor of the exact residual (see
      // residual_floor)
      double cK = 0.0, cM = 0.0;
      for (int i = 0; i < 27; ++i) {
        cK += P->K.c[i] * P->K.c[i];
        cM += P->M.c[i] * P->M.c[i];
      }
      double sm = 0.0, sd = 0.0;
      for (int64_t l = 0; l < nt; ++l) {
        const double mlo = l + 1 < nt ? P->h_ms[l] : 0.0, dlo = l + 1 < nt ? P->h_ts[l] : 0.0;
        sm += P->h_md[l] * P->h_md[l] + mlo * mlo;
        sd += P->h_td[l] * P->h_td[l] + dlo * dlo;
      }
      const double u = std::ldexp(1.0, -53);
      if (P->fnorm > 0.0)
        P->floor_coef = u / std::sqrt(3.0) *
                        (std::sqrt(cK * sm / nt) + std::sqrt(cM * sd / nt)) / P->fnorm;
    }
    *out = P.release();
  });
}

sts_status sts_solve(sts_problem* P, const sts_opts* opts_in, sts_info* info) {
  return run_guarded([&] {
    STS_REQUIRE(P != nullptr, STS_E_INVALID, "problem is NULL");
    sts_opts o;
    sts_default_opts(&o);
    if (opts_in) o = *opts_in;
    STS_REQUIRE(o.tol > 0.0 && o.max_outer >= 1 && o.inner_rtol > 0.0 && o.inner_maxit >= 1 &&
                    o.defl_tol >= 0.0 && o.defl_tol < 1.0 && o.check_every >= 0 &&
                    o.residual_qr >= -1 && o.residual_qr <= 1 && o.inner_relax >= 0 &&
                    o.inner_relax <= 6 && (o.precond_fp32 == 0 || o.precond_fp32 == 1) &&
                    o.mixed >= 0 && o.mixed <= 3 && (o.orth_lag == 0 || o.orth_lag == 1),
                STS_E_INVALID, "invalid options");
    P->residual_qr = o.residual_qr;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = P->stream;
    const int p = P->p;
    const int b2 = 2 * p;
    if (o.restart) {
      P->k = P->k_sol = P->blk_start = P->blk_size = 0;
      P->prov = 0;
      P->tags.clear();
      P->solved = false;
      P->inner_K = P->inner_M = 0;
      P->inner_K32 = P->defect_rounds = 0;
      P->v32_cols = 0;
      P->pend_size = 0;
      P->alg_bytes = 0.0;
      P->checks = 0;
      P->shifts.clear();
      P->last_cheap = -1.0;
    }
    // kernel timing for sts_kernel_profile, active until this call returns
    struct ProfGuard {
      explicit ProfGuard(Profiler* p) { set_active_profiler(p); }
      ~ProfGuard() { set_active_profiler(nullptr); }
    } prof_guard(o.profile ? &P->prof : nullptr);
    if (o.profile) P->prof.reset();
    P->profiled = o.profile != 0;
    // mixed precision keeps an FP32 copy of V for the first Gram-Schmidt pass
    const bool v32 = mixed_gs(P, o);
    if (v32 && !P->want_v32) {
      P->want_v32 = true;
      P->v32_cols = 0;
      if (P->kcap > 0) {
        if (P->grow_hook) P->grow_hook(P->ldv * P->kcap * 4);
        P->V32.ensure(P->ldv * P->kcap * 4, 0, st);
      }
    }
    // the basis grows with the space, to at most max_outer + 2 more blocks
    const int64_t cap_limit = P->k + P->prov + (int64_t)b2 * (o.max_outer + 2);
    ensure_capacity(P, P->k + P->prov + initial_capacity(p, o.max_outer), cap_limit,
                    o.mem_budget);
    if (v32 && P->v32_cols < P->k) {
      // a basis extended from an FP64 solve: round its columns once
      round_cols(P->nh, (int)(P->k - P->v32_cols), P->V.d() + P->v32_cols * P->ldv, P->ldv,
                 reinterpret_cast<float*>(P->V32.base) + P->v32_cols * P->ldv, P->ldv, st);
      P->v32_cols = P->k;
    }
    P->use_v32 = v32;
    // lagged re-orthogonalisation (sts_opts.orth_lag), except in the rational
    // space, with the FP32 first pass, and in 1-D: there V is small (its reads
    // cost microseconds) and kappa(Mx^{-1} Kx) reaches 1e10, so the next block's
    // expansion from a once-orthogonalised block amplifies its components
    // along V (a 65535-node solve no longer met its residual floor).  A
    // provisional block left by an earlier lagged solve is dropped otherwise.
    const bool lag = o.orth_lag != 0 && !o.rational && !v32 && P->grid.dim > 1;
    if (!lag && P->prov > 0) {
      P->tags.resize(P->k);
      P->prov = 0;
    }
    // STS_TRACE=1: one line per residual check on stderr
    const char* tr = std::getenv("STS_TRACE");
    const bool trace = tr && tr[0] == '1';
    sts_status result = STS_E_NOT_CONVERGED;
    std::string fail_msg;
    bool breakdown = false;
    bool floor_limited = false;
    double floor = -1.0;
    double cheap = -1.0, truer = -1.0;
    int outer = 0;
    if (P->fnorm == 0.0) {
      // zero right-hand side: U = 0
      P->k_sol = 0;
      P->solved = true;
      result = STS_OK;
      cheap = truer = 0.0;
    } else {
      if (P->k == 0) {
        // start block [Mx^{-1} F1, Kx^{-1} F1]
        int ops[kMaxCols];
        const double* b[kMaxCols];
        for (int c = 0; c < p; ++c) {
          ops[c] = STS_OP_M;
          ops[p + c] = STS_OP_K;
          b[c] = b[p + c] = P->F1.d() + c * P->ldv;
        }
        int perm[kMaxCols];
        sts_opts oi = o;
        const double relax = o.inner_relax ? std::pow(10.0, -o.inner_relax) : 0.0;
        if (o.inner_relax) oi.inner_rtol = std::max(o.inner_rtol, std::min(1e-4, relax * o.tol));
        run_cg_block(P, ops, b2, b, oi, perm);
        int idx[16];
        const int kept = append_block(P, b2, o.defl_tol, idx);
        P->blk_start = 0;
        P->blk_size = kept;
        P->tags.clear();
        for (int j = 0; j < kept; ++j) P->tags.push_back(perm[idx[j]] < p ? 0 : 1);
        P->k = kept;
        P->k_sol = 0;
        STS_REQUIRE(kept > 0, STS_E_NUMERIC, "start block vanished although F is non-zero");
      }
      int next_check = 1;
      int last_check_outer = -1;
      std::vector<double> ritz;
      double ritz_lo = std::numeric_limits<double>::infinity(), ritz_hi = 0.0;
      double last_check_res = -1.0;
      // exact / projected residual, learned from exact checks (inexact inner
      // solves make the projected value read low)
      double ratio = 1.0;
      std::vector<double> hist;   // projected residuals of the checks (stall test)
      // the rounding floor of the exact residual per unit ||Y||_F and without
      // its growth with k, from the first check (||V Y||_2 / ||Y||_F stays
      // within the square root of Mx's condition number)
      double floor_base = -1.0;
      for (outer = 1; outer <= o.max_outer; ++outer) {
        if (trace)
          std::fprintf(stderr, "sts: %.4f s outer %d k %lld\n",
                       std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(),
                       outer, (long long)P->k);
        ensure_capacity(P, P->k + P->prov + b2, cap_limit, o.mem_budget);
        // a residual check follows this block: it is made final at once
        const bool due = o.check_every > 0 ? (outer % o.check_every == 0 || outer == o.max_outer)
                                           : (outer >= next_check || outer == o.max_outer);
        // inner tolerance of this block: relaxed in inverse proportion to the
        // residual (the block's share of the solution shrinks with it)
        sts_opts oi = o;
        if (o.inner_relax) {
          const double r = P->last_cheap > 0.0 ? std::min(1.0, ratio * P->last_cheap) : 1.0;
          oi.inner_rtol = std::max(o.inner_rtol,
                                   std::min(1e-4, std::pow(10.0, -o.inner_relax) * o.tol / r));
        }
        // expand with the last block (the provisional one if there is one)
        const int64_t bs = P->prov > 0 ? P->k : P->blk_start;
        const int64_t bsz = P->prov > 0 ? P->prov : P->blk_size;
        int ops[kMaxCols];
        const double* b[kMaxCols];
        int n = 0;
        int perm[kMaxCols];
        if (o.rational) {
          // rational Krylov step: (Kx + s Mx)^{-1} Mx applied to the last
          // block, s from the Ritz values of the current basis
          flush_pending(P);
          ritz_values(P, P->k, ritz);
          for (double v : ritz) {
            ritz_lo = std::min(ritz_lo, v);
            ritz_hi = std::max(ritz_hi, v);
          }
          STS_REQUIRE(ritz_lo > 0.0, STS_E_NUMERIC, "reduced stiffness is not positive definite");
          const double sft = adaptive_shift(ritz.data(), (int)ritz.size(), P->shifts.data(),
                                            (int)P->shifts.size(), ritz_lo, ritz_hi, 1001);
          P->shifts.push_back(sft);
          for (int64_t j = 0; j < bsz; ++j) {
            b[n] = P->MV.d() + (bs + j) * P->ldv;
            perm[n] = n;
            ++n;
          }
          run_shifted_block(P, sft, n, b, oi);
        } else {
          for (int64_t j = 0; j < bsz; ++j) {
            const int tag = P->tags[bs + j];
            ops[n] = tag == 0 ? STS_OP_M : STS_OP_K;
            // positive power: Mx^{-1} (Kx v); negative power: Kx^{-1} (Mx v)
            b[n] = (tag == 0 ? P->KV.d() : P->MV.d()) + (bs + j) * P->ldv;
            ++n;
          }
          run_cg_block(P, ops, n, b, oi, perm);
        }
        std::vector<int> src_tag(n);
        for (int j = 0; j < n; ++j) src_tag[j] = P->tags[bs + perm[j]];
        int idx[16];
        // lagged: the provisional block becomes final here (P->k moves past
        // it) and the new block stays provisional unless a check follows
        const int kept = lag ? append_lagged(P, n, o.defl_tol, due, idx)
                             : append_block(P, n, o.defl_tol, idx);
        const int64_t kprev = P->k;
        for (int j = 0; j < kept; ++j) P->tags.push_back(src_tag[idx[j]]);
        if (!lag || due) {
          P->blk_start = kprev;
          P->blk_size = kept;
          P->k = kprev + kept;
        } else {
          P->prov = kept;
        }
        if (kept == 0) {
          // every new column lies in the space: it is invariant under A and
          // A^{-1}, so the Galerkin solution is exact in exact arithmetic.  A
          // deflation threshold too coarse for the problem can also empty a
          // block, so the exact residual confirms before success.
          breakdown = true;
          P->k_sol = kprev;
          flush_pending(P);
          cheap = reduced_solve(P, kprev, 0);
          if (o.verify_true) {
            truer = true_residual(P);
            if (trace) std::fprintf(stderr, "sts: outer %d breakdown, exact residual %.3e\n", outer, truer);
            if (truer > o.tol && floor_accepts(P, o.tol, truer, &floor)) floor_limited = true;
            else if (truer > o.tol) {
              result = STS_E_NUMERIC;
              fail_msg = "the space stopped growing (every new column deflated) with exact residual " +
                         std::to_string(truer) + " above tol; the factors of this iterate are kept";
              break;
            }
          }
          result = STS_OK;
          break;
        }
        if (!due) continue;
        if (o.rational) {
          // no projected-residual formula for this space: the exact residual
          // of the Galerkin solution on the whole basis decides
          P->k_sol = P->k;
          flush_pending(P);
          reduced_solve(P, P->k, 0);
          cheap = true_residual(P);
          truer = cheap;
          P->last_cheap = cheap;
          if (trace)
            std::fprintf(stderr, "sts: outer %d k %lld exact residual %.3e (rational)\n", outer,
                         (long long)P->k, cheap);
          if (cheap <= o.tol) {
            result = STS_OK;
            break;
          }
          if (o.check_every == 0) {
            int step = 1;
            if (last_check_res > 0.0 && cheap < last_check_res) {
              const double rate =
                  std::pow(cheap / last_check_res, 1.0 / std::max(1, outer - last_check_outer));
              const double need = std::log(o.tol / cheap) / std::log(rate);
              step = std::max(1, std::min(8, (int)std::ceil(need)));
            }
            last_check_outer = outer;
            last_check_res = cheap;
            next_check = outer + step;
          }
          continue;
        }
        P->k_sol = kprev;
        flush_pending(P);
        cheap = reduced_solve(P, kprev, kept);
        P->last_cheap = cheap;
        if (trace)
          std::fprintf(stderr, "sts: outer %d k %lld projected residual %.3e (x %.2f)\n", outer,
                       (long long)kprev, cheap, ratio);
        // Where the estimated floor of the exact residual exceeds tol, tol is
        // out of reach of any FP64 evaluation: the projected residual is
        // taken to tol + floor, and the exact check (floor_accepts) decides.
        // Without this the target stays at tol and such a solve iterates to
        // max_outer with its error long converged.  (The estimate is about
        // eight times the measured floor, so below tol the target stays.)
        const double ynorm = o.verify_true ? y_fnorm(P) : 0.0;
        if (o.verify_true && floor_base < 0.0 && ynorm > 0.0)
          floor_base = residual_floor(P) / (floor_growth(P) * ynorm);
        const double fl_est = std::max(0.0, floor_base) * floor_growth(P) * ynorm;
        const double goal = o.verify_true && fl_est > o.tol ? o.tol + fl_est : o.tol;
        if (ratio * cheap <= goal) {
          if (!o.verify_true) {
            result = STS_OK;
            break;
          }
          truer = true_residual(P);
          if (trace) std::fprintf(stderr, "sts: outer %d exact residual %.3e\n", outer, truer);
          if (truer <= o.tol) {
            result = STS_OK;
            break;
          }
          if (floor_accepts(P, o.tol, truer, &floor)) {
            // the projected residual met tol; the exact one is above it only
            // by the rounding floor of its own evaluation
            result = STS_OK;
            floor_limited = true;
            break;
          }
          if (cheap > 0.0) ratio = std::max(ratio, truer / cheap);
        }
        hist.push_back(ratio * cheap);
        const size_t nh = hist.size();
        if (o.verify_true && nh > kStallChecks &&
            *std::min_element(hist.end() - kStallChecks, hist.end()) >
                0.5 * hist[nh - 1 - kStallChecks]) {
          const double fl = residual_floor(P);
          if (fl >= 0.5 * o.tol) {
            truer = true_residual(P);
            if (trace)
              std::fprintf(stderr, "sts: outer %d stalled, exact residual %.3e, floor %.3e\n", outer,
                           truer, fl);
            floor = fl;
            if (truer <= o.tol + kStallFloor * fl) {
              result = STS_OK;
              floor_limited = truer > o.tol;
              break;
            }
            hist.clear();
          }
        }
        // schedule the next check from the observed convergence rate and the
        // predicted crossing of tol / ratio
        if (o.check_every == 0) {
          int step = 1;
          const double target = goal / ratio;
          if (last_check_res > 0.0 && cheap > 0.0 && cheap < last_check_res && cheap > target) {
            const double rate =
                std::pow(cheap / last_check_res, 1.0 / std::max(1, outer - last_check_outer));
            // an extra block is far cheaper than an extra check (eigensolve
            // of the reduced pencil, possibly an exact residual): aim at the
            // predicted crossing, not before it
            const double need = std::log(target / cheap) / std::log(rate);
            step = std::max(1, std::min(24, (int)std::ceil(need)));
          }
          last_check_outer = outer;
          last_check_res = cheap;
          next_check = outer + step;
        }
      }
      if (outer > o.max_outer) outer = o.max_outer;
      P->solved = true;
    }
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->outer_its = outer;
      info->checks = P->checks;
      info->k = P->k_sol;
      info->inner_its_K = P->inner_K;
      info->inner_its_fp32 = P->inner_K32;
      info->defect_rounds = P->defect_rounds;
      info->inner_its_M = P->inner_M;
      info->res_cheap = cheap;
      info->breakdown = breakdown ? 1 : 0;
      info->shifts = (int32_t)P->shifts.size();
      if (truer < 0.0 && o.verify_true && P->k_sol > 0) truer = true_residual(P);
      info->res_true = truer;
      info->orth_err = orth_error(P);
      info->rank = -1;
      info->alg_bytes = P->alg_bytes;
      info->cg_poll_restarts = P->cg.poll.poll_restarts;
      info->res_floor = floor;
      info->floor_limited = floor_limited ? 1 : 0;
    }
    STS_HIP(hipStreamSynchronize(st));
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) info->seconds = secs;
    if (result != STS_OK)
      throw Error{result, fail_msg.empty()
                              ? "max_outer reached before the residual met tol (last projected residual " +
                                    std::to_string(cheap) + ")"
                              : fail_msg};
  });
}

sts_status sts_rank(const sts_problem* P, int64_t* k) {
  return run_guarded([&] {
    STS_REQUIRE(P && k, STS_E_INVALID, "NULL argument");
    *k = P->solved ? P->k_sol : 0;
  });
}

sts_status sts_get_factors(const sts_problem* Pc, double* V, int64_t ldv, double* Y, int64_t ldy,
                           int32_t mem, void* stream) {
  return run_guarded([&] {
    STS_REQUIRE(Pc != nullptr, STS_E_INVALID, "problem is NULL");
    STS_REQUIRE(Pc->solved, STS_E_STATE, "no solution yet: call sts_solve first");
    STS_REQUIRE(mem == STS_MEM_HOST || mem == STS_MEM_DEVICE, STS_E_INVALID, "bad mem kind");
    sts_problem* P = const_cast<sts_problem*>(Pc);
    const int64_t ks = P->k_sol;
    hipStream_t st = stream ? static_cast<hipStream_t>(stream) : P->stream;
    if (st != P->stream) STS_HIP(hipStreamSynchronize(P->stream));
    const hipMemcpyKind kind = mem == STS_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (V && ks > 0) {
      STS_REQUIRE(ldv >= P->nh, STS_E_INVALID, "ldv < Nh");
      // a kernel reads V, into the caller's device buffer directly or
      // through a bounded device staging buffer for the host
      if (mem == STS_MEM_DEVICE) {
        copy_cols(P->nh, (int)ks, P->V.d(), P->ldv, V, ldv, st);
      } else {
        const int64_t per = std::max<int64_t>(1, std::min<int64_t>(ks, (32 << 20) / std::max<int64_t>(P->nh, 1)));
        DevBuf stage;
        stage.alloc((size_t)(per * P->nh) * 8);
        for (int64_t c0 = 0; c0 < ks; c0 += per) {
          const int64_t nc = std::min(per, ks - c0);
          copy_cols(P->nh, (int)nc, P->V.d() + c0 * P->ldv, P->ldv, stage.d(), P->nh, st);
          STS_HIP(hipMemcpy2DAsync(V + c0 * ldv, ldv * 8, stage.d(), P->nh * 8, P->nh * 8, nc,
                                   hipMemcpyDeviceToHost, st));
          STS_HIP(hipStreamSynchronize(st));
        }
      }
    }
    if (Y && ks > 0) {
      STS_REQUIRE(ldy >= ks, STS_E_INVALID, "ldy < k");
      STS_HIP(hipMemcpy2DAsync(Y, ldy * 8, P->Y.p, P->kcap * 8, ks * 8, P->nt, kind, st));
    }
    STS_HIP(hipStreamSynchronize(st));
  });
}

sts_status sts_solution_columns(const sts_problem* Pc, const int64_t* cols, int32_t ncols,
                                double* U, int64_t ldu, int32_t mem, void* stream) {
  return run_guarded([&] {
    STS_REQUIRE(Pc != nullptr, STS_E_INVALID, "problem is NULL");
    STS_REQUIRE(Pc->solved, STS_E_STATE, "no solution yet: call sts_solve first");
    STS_REQUIRE(mem == STS_MEM_HOST || mem == STS_MEM_DEVICE, STS_E_INVALID, "bad mem kind");
    STS_REQUIRE(cols && U && ncols >= 1 && ldu >= Pc->nh, STS_E_INVALID, "bad buffers");
    for (int32_t j = 0; j < ncols; ++j)
      STS_REQUIRE(cols[j] >= 0 && cols[j] < Pc->nt, STS_E_INVALID, "time index out of range");
    sts_problem* P = const_cast<sts_problem*>(Pc);
    const int64_t ks = P->k_sol, nh = P->nh, kc = P->kcap;
    hipStream_t st = stream ? static_cast<hipStream_t>(stream) : P->stream;
    if (st != P->stream) STS_HIP(hipStreamSynchronize(P->stream));
    // 16 columns at a time: gather Y's columns (negated), U_j = 0 - V (-Y_j)
    constexpr int kW = 16;
    DevBuf ysel, ubuf;
    ysel.alloc(std::max<int64_t>(ks, 1) * kW * 8);
    if (mem == STS_MEM_HOST) ubuf.alloc(nh * kW * 8);
    std::vector<double> h;
    for (int32_t c0 = 0; c0 < ncols; c0 += kW) {
      const int nc = std::min<int32_t>(kW, ncols - c0);
      double* dst = mem == STS_MEM_HOST ? ubuf.d() : U + (int64_t)c0 * ldu;
      const int64_t ldd = mem == STS_MEM_HOST ? nh : ldu;
      for (int j = 0; j < nc; ++j) {
        fill(dst + j * ldd, nh, 0.0, st);
        if (ks > 0) copy_cols(ks, 1, P->Y.d() + cols[c0 + j] * kc, kc, ysel.d() + j * ks, ks, st);
      }
      if (ks > 0) {
        scale(ysel.d(), ks * nc, -1.0, st);
        gemm_nn_sub(nh, (int)ks, nc, P->V.d(), P->ldv, ysel.d(), ks, dst, ldd, st);
      }
      if (mem == STS_MEM_HOST)
        STS_HIP(hipMemcpy2DAsync(U + (int64_t)c0 * ldu, ldu * 8, dst, nh * 8, nh * 8, nc,
                                 hipMemcpyDeviceToHost, st));
      STS_HIP(hipStreamSynchronize(st));
    }
  });
}

sts_status sts_true_residual(sts_problem* P, double* res) {
  return run_guarded([&] {
    STS_REQUIRE(P && res, STS_E_INVALID, "NULL argument");
    STS_REQUIRE(P->solved, STS_E_STATE, "no solution yet");
    *res = (P->fnorm == 0.0) ? 0.0 : true_residual(P);
  });
}

sts_status sts_numerical_rank(sts_problem* P, int64_t* rank) {
  return run_guarded([&] {
    STS_REQUIRE(P && rank, STS_E_INVALID, "NULL argument");
    STS_REQUIRE(P->solved, STS_E_STATE, "no solution yet");
    *rank = numerical_rank(P);
  });
}

sts_status sts_kernel_profile(sts_problem* P, int32_t kernel, double* seconds,
                              int64_t* launches, double* alg_bytes) {
  return run_guarded([&] {
    STS_REQUIRE(P != nullptr, STS_E_INVALID, "problem is NULL");
    STS_REQUIRE(kernel >= 0 && kernel < STS_K_COUNT, STS_E_INVALID, "unknown kernel");
    STS_REQUIRE(P->profiled, STS_E_STATE, "the last solve was not profiled");
    P->prof.collect();
    if (seconds) *seconds = P->prof.sec[kernel];
    if (launches) *launches = P->prof.cnt[kernel];
    if (alg_bytes) *alg_bytes = P->prof.byt[kernel];
  });
}

const char* sts_kernel_name(int32_t kernel) {
  static const char* names[STS_K_COUNT] = {
      "cg_iter",   "mg_down",  "mg_up",   "mg_coarse",     "pcg_a", "pcg_b",
      "mass_cheb", "gram",     "basis_update", "residual", "tridiag", "bisect",
      "inviter",   "backtransform", "sweep", "stencil", "tridiag_solve",
      "mg_restrict", "pcg_reduce", "residual_qr", "gram_reduce"};
  return (kernel >= 0 && kernel < STS_K_COUNT) ? names[kernel] : "";
}

void sts_release_cached_memory(void) { cache_trim(-1); }

void sts_destroy(sts_problem* P) {
  if (!P) return;
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  delete P;
}

// ---------------------------------------------------------------------------
// step-level entry points
// ---------------------------------------------------------------------------

sts_status sts_apply_op(const sts_space* space, int32_t op, const double* X, int64_t ldx,
                        double* Y, int64_t ldy, int32_t ncols, void* stream) {
  return run_guarded([&] {
    validate_space(space);
    const Grid g = make_grid(*space);
    STS_REQUIRE(op == STS_OP_K || op == STS_OP_M, STS_E_INVALID, "bad op");
    STS_REQUIRE(ncols >= 0 && ncols <= 16, STS_E_INVALID, "ncols out of range");
    STS_REQUIRE(ncols == 0 || (X && Y && ldx >= g.nh && ldy >= g.nh), STS_E_INVALID,
                "bad buffers / leading dimensions");
    const Stencil K = make_stencil(*space, STS_OP_K), M = make_stencil(*space, STS_OP_M);
    int ops[16];
    for (int c = 0; c < 16; ++c) ops[c] = op;
    hipStream_t st = static_cast<hipStream_t>(stream);
    stencil_apply(g, K, M, ops, ncols, X, ldx, Y, ldy, st);
    STS_HIP(hipStreamSynchronize(st));
  });
}

sts_status sts_cg(const sts_space* space, const int32_t* ops_in, const double* B, int64_t ldb,
                  double* X, int64_t ldx, int32_t ncols, double rtol, int32_t maxit,
                  int32_t* iters, void* stream) {
  sts_status bad = STS_OK;
  sts_status s = run_guarded([&] {
    validate_space(space);
    const Grid g = make_grid(*space);
    STS_REQUIRE(ncols >= 1 && ncols <= kMaxCols, STS_E_INVALID, "ncols must be 1..8");
    STS_REQUIRE(ops_in && B && X && ldb >= g.nh && ldx >= g.nh, STS_E_INVALID, "bad buffers");
    STS_REQUIRE(rtol > 0.0 && maxit >= 1, STS_E_INVALID, "bad rtol / maxit");
    int ops[kMaxCols];
    for (int c = 0; c < ncols; ++c) {
      STS_REQUIRE(ops_in[c] == STS_OP_K || ops_in[c] == STS_OP_M, STS_E_INVALID, "bad op");
      ops[c] = ops_in[c];
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch sc;
    const int64_t ld = pad_ld(g.nh);
    const int tiles = cg_tiles(g);
    CGRunner r;
    r.g = g;
    r.K = make_stencil(*space, STS_OP_K);
    r.M = make_stencil(*space, STS_OP_M);
    r.w.x = X;
    r.w.ld = ldx;
    r.w.r[0] = sc.get<double>(ld * ncols);
    r.w.r[1] = sc.get<double>(ld * ncols);
    r.w.p[0] = sc.get<double>(ld * ncols);
    r.w.p[1] = sc.get<double>(ld * ncols);
    // x, r, p share one leading dimension in the kernels: stage x if needed
    double* xs = X;
    if (ldx != ld) {
      xs = sc.get<double>(ld * ncols);
      r.w.x = xs;
    }
    r.w.ld = ld;
    r.w.scal = sc.get<CGScal>(2 * kMaxCols);
    r.w.partials = sc.get<double>((size_t)2 * 2 * kMaxCols * tiles);
    r.w.max_tiles = tiles;
    r.poll.init();
    const double* bcols[kMaxCols];
    for (int c = 0; c < ncols; ++c) bcols[c] = B + c * ldb;
    CGScal out[kMaxCols];
    r.run(ops, ncols, bcols, rtol, maxit, out, st);
    if (xs != X) copy_cols(g.nh, ncols, xs, ld, X, ldx, st);
    STS_HIP(hipStreamSynchronize(st));
    for (int c = 0; c < ncols; ++c) {
      if (iters) iters[c] = out[c].iters;
      if (out[c].flag == 3) bad = STS_E_NUMERIC;
      else if (out[c].flag == 2 && bad == STS_OK) bad = STS_E_NOT_CONVERGED;
    }
  });
  if (s == STS_OK && bad != STS_OK) {
    set_error(bad == STS_E_NUMERIC ? "CG breakdown" : "CG reached maxit");
    return bad;
  }
  return s;
}

sts_status sts_adaptive_shift(const double* ritz, int32_t k, const double* shifts, int32_t m,
                              double a, double b, int32_t grid, double* s) {
  return run_guarded([&] {
    STS_REQUIRE(s != nullptr && (k == 0 || ritz) && (m == 0 || shifts), STS_E_INVALID,
                "sts_adaptive_shift: null argument");
    *s = adaptive_shift(ritz, k, shifts, m, a, b, grid);
  });
}

sts_status sts_shifted_solve(const sts_space* space, double shift, const double* B, int64_t ldb,
                             double* X, int64_t ldx, int32_t ncols, double rtol, int32_t maxit,
                             int32_t* iters, void* stream) {
  sts_status bad = STS_OK;
  sts_status s = run_guarded([&] {
    validate_space(space);
    const Grid g = make_grid(*space);
    STS_REQUIRE(ncols >= 1 && ncols <= kMaxCols, STS_E_INVALID, "ncols must be 1..8");
    STS_REQUIRE(B && X && ldb >= g.nh && ldx >= g.nh, STS_E_INVALID, "bad buffers");
    STS_REQUIRE(shift >= 0.0 && std::isfinite(shift), STS_E_INVALID, "shift must be >= 0");
    STS_REQUIRE(rtol > 0.0 && maxit >= 1, STS_E_INVALID, "bad rtol / maxit");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Stencil K = make_stencil(*space, STS_OP_K);
    const Stencil M = make_stencil(*space, STS_OP_M);
    Scratch sc;
    const int64_t ld = pad_ld(g.nh);
    const double* bcols[kMaxCols];
    for (int c = 0; c < ncols; ++c) bcols[c] = B + c * ldb;
    if (tridiag_supported(g, K, M)) {
      const int64_t nw = tridiag_shifted_work_doubles(g.nh, ld, ncols);
      double* work = sc.get<double>(nw);
      tridiag_shifted_solve(g, K, M, shift, ncols, bcols, X, ldx, work, ld, nw, st);
      STS_HIP(hipStreamSynchronize(st));
      if (iters)
        for (int c = 0; c < ncols; ++c) iters[c] = 1;
      return;
    }
    MGPlan plan{};
    if (mg_plan(g, K, &plan)) {
      // multigrid-preconditioned CG on Kx + shift Mx
      plan.sw0 = shift * mass_scale(g, M);
      MGRunner r;
      r.setup(plan);
      CGScal out[kMaxCols];
      r.run(X, ldx, ncols, bcols, rtol, maxit, out, st);
      STS_HIP(hipStreamSynchronize(st));
      bad = cg_status(out, ncols, iters);
      return;
    }
    const int tiles = cg_tiles(g);
    CGRunner r;
    r.g = g;
    r.K = K;
    r.M = M;   // Kx + shift Mx, in the operator slot whose pattern contains both
    for (int i = 0; i < 27; ++i) r.M.c[i] = K.c[i] + shift * M.c[i];
    r.w.r[0] = sc.get<double>(ld * ncols);
    r.w.r[1] = sc.get<double>(ld * ncols);
    r.w.p[0] = sc.get<double>(ld * ncols);
    r.w.p[1] = sc.get<double>(ld * ncols);
    double* xs = ldx == ld ? X : sc.get<double>(ld * ncols);
    r.w.x = xs;
    r.w.ld = ld;
    r.w.scal = sc.get<CGScal>(2 * kMaxCols);
    r.w.partials = sc.get<double>((size_t)2 * 2 * kMaxCols * tiles);
    r.w.max_tiles = tiles;
    r.poll.init();
    int ops[kMaxCols];
    for (int c = 0; c < ncols; ++c) ops[c] = STS_OP_M;
    CGScal out[kMaxCols];
    r.run(ops, ncols, bcols, rtol, maxit, out, st);
    if (xs != X) copy_cols(g.nh, ncols, xs, ld, X, ldx, st);
    STS_HIP(hipStreamSynchronize(st));
    bad = cg_status(out, ncols, iters);
  });
  if (s == STS_OK && bad != STS_OK) {
    set_error(bad == STS_E_NUMERIC ? "CG breakdown" : "CG reached maxit");
    return bad;
  }
  return s;
}

sts_status sts_pcg_mg(const sts_space* space, const double* B, int64_t ldb, double* X,
                      int64_t ldx, int32_t ncols, double rtol, int32_t maxit, int32_t* iters,
                      void* stream) {
  sts_status bad = STS_OK;
  sts_status s = run_guarded([&] {
    Grid g;
    const MGPlan plan = require_mg(space, &g);
    STS_REQUIRE(ncols >= 1 && ncols <= kMaxCols, STS_E_INVALID, "ncols must be 1..8");
    STS_REQUIRE(B && X && ldb >= g.nh && ldx >= g.nh, STS_E_INVALID, "bad buffers");
    STS_REQUIRE(rtol > 0.0 && maxit >= 1, STS_E_INVALID, "bad rtol / maxit");
    hipStream_t st = static_cast<hipStream_t>(stream);
    MGRunner r;
    r.setup(plan);
    const double* bcols[kMaxCols];
    for (int c = 0; c < ncols; ++c) bcols[c] = B + c * ldb;
    CGScal out[kMaxCols];
    r.run(X, ldx, ncols, bcols, rtol, maxit, out, st);
    STS_HIP(hipStreamSynchronize(st));
    bad = cg_status(out, ncols, iters);
  });
  if (s == STS_OK && bad != STS_OK) {
    set_error(bad == STS_E_NUMERIC ? "preconditioned CG breakdown"
                                   : "preconditioned CG reached maxit");
    return bad;
  }
  return s;
}

sts_status sts_mass_solve(const sts_space* space, const double* B, int64_t ldb, double* X,
                          int64_t ldx, int32_t ncols, double rtol, int32_t* iters,
                          void* stream) {
  return run_guarded([&] {
    validate_space(space);
    const Grid g = make_grid(*space);
    const Stencil M = make_stencil(*space, STS_OP_M);
    STS_REQUIRE(ncols >= 1 && ncols <= kMaxCols, STS_E_INVALID, "ncols must be 1..8");
    STS_REQUIRE(B && X && ldb >= g.nh && ldx >= g.nh, STS_E_INVALID, "bad buffers");
    STS_REQUIRE(rtol > 0.0 && rtol < 1.0, STS_E_INVALID, "rtol must be in (0, 1)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch sc;
    if (tensor_mass_supported(g, M)) {
      double* fac = sc.get<double>(2 * g.nx);
      tensor_mass_factor(g.nx, fac, st);
      const double* bc[kMaxCols];
      for (int c = 0; c < ncols; ++c) bc[c] = B + c * ldb;
      tensor_mass_solve(g, M, ncols, bc, X, ldx, fac, st);
      STS_HIP(hipStreamSynchronize(st));
      if (iters)
        for (int c = 0; c < ncols; ++c) iters[c] = 1;
      return;
    }
    STS_REQUIRE(mass_cheb_supported(g, M), STS_E_INVALID,
                "mass solve needs a 2-D P1 or a 3-D trilinear space");
    const int64_t ld = pad_ld(g.nh);
    double* xb[2] = {sc.get<double>(ld * ncols), sc.get<double>(ld * ncols)};
    double* db[2] = {sc.get<double>(ld * ncols), sc.get<double>(ld * ncols)};
    const double* bc[kMaxCols];
    for (int c = 0; c < ncols; ++c) bc[c] = B + c * ldb;
    const int its = mass_cheb_iters(rtol);
    mass_cheb_solve(g, M, ncols, bc, X, ldx, xb, db, ld, its, st);
    STS_HIP(hipStreamSynchronize(st));
    if (iters)
      for (int c = 0; c < ncols; ++c) iters[c] = its;
  });
}

sts_status sts_tridiag_solve(const sts_space* space, const int32_t* ops, const double* B,
                             int64_t ldb, double* X, int64_t ldx, int32_t ncols, void* stream) {
  return run_guarded([&] {
    validate_space(space);
    const Grid g = make_grid(*space);
    const Stencil K = make_stencil(*space, STS_OP_K);
    const Stencil M = make_stencil(*space, STS_OP_M);
    STS_REQUIRE(tridiag_supported(g, K, M), STS_E_INVALID,
                "direct tridiagonal solve needs a 1-D P1 space");
    STS_REQUIRE(ncols >= 1 && ncols <= kMaxCols, STS_E_INVALID, "ncols must be 1..8");
    STS_REQUIRE(ops != nullptr, STS_E_INVALID, "ops is null");
    for (int c = 0; c < ncols; ++c)
      STS_REQUIRE(ops[c] == STS_OP_K || ops[c] == STS_OP_M, STS_E_INVALID, "bad operator");
    STS_REQUIRE(B && X && ldb >= g.nh && ldx >= g.nh, STS_E_INVALID, "bad buffers");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch sc;
    double* fac = sc.get<double>(tridiag_factor_doubles(g.nh));
    tridiag_factor(g, K, M, fac, st);
    const double* bc[kMaxCols];
    int op[kMaxCols];
    for (int c = 0; c < ncols; ++c) {
      bc[c] = B + c * ldb;
      op[c] = ops[c];
    }
    tridiag_solve(g, K, M, op, ncols, bc, X, ldx, fac, st);
    STS_HIP(hipStreamSynchronize(st));
  });
}

sts_status sts_mg_vcycle_shifted(const sts_space* space, double shift, const double* R,
                                 int64_t ldr, double* Z, int64_t ldz, int32_t ncols,
                                 void* stream) {
  return run_guarded([&] {
    Grid g;
    MGPlan plan = require_mg(space, &g);
    STS_REQUIRE(shift >= 0.0 && std::isfinite(shift), STS_E_INVALID, "shift must be >= 0");
    plan.sw0 = shift * mass_scale(g, make_stencil(*space, STS_OP_M));
    STS_REQUIRE(ncols >= 1 && ncols <= kMaxCols, STS_E_INVALID, "ncols must be 1..8");
    STS_REQUIRE(R && Z && ldr >= g.nh && ldz >= g.nh, STS_E_INVALID, "bad buffers");
    hipStream_t st = static_cast<hipStream_t>(stream);
    MGRunner r;
    r.setup(plan);
    copy_cols(g.nh, ncols, R, ldr, r.w.b[0], r.w.ld[0], st);
    int cols[kMaxCols];
    for (int c = 0; c < ncols; ++c) cols[c] = c;
    mg_vcycle(r.w, nullptr, cols, ncols, false, st);
    copy_cols(g.nh, ncols, r.w.e[0], r.w.ld[0], Z, ldz, st);
    STS_HIP(hipStreamSynchronize(st));
  });
}

sts_status sts_mg_vcycle_mixed(const sts_space* space, double shift, const double* R,
                               int64_t ldr, double* Z, int64_t ldz, int32_t ncols,
                               void* stream) {
  return run_guarded([&] {
    Grid g;
    const MGPlan plan = require_mg_mixed(space, shift, &g);
    STS_REQUIRE(ncols >= 1 && ncols <= kMaxCols, STS_E_INVALID, "ncols must be 1..8");
    STS_REQUIRE(R && Z && ldr >= g.nh && ldz >= g.nh, STS_E_INVALID, "bad buffers");
    hipStream_t st = static_cast<hipStream_t>(stream);
    MGRunner r;
    r.setup(plan);
    copy_cols(g.nh, ncols, R, ldr, r.w.b[0], r.w.ld[0], st);
    int cols[kMaxCols];
    for (int c = 0; c < ncols; ++c) cols[c] = c;
    mg_vcycle(r.w, nullptr, cols, ncols, false, st);
    copy_cols(g.nh, ncols, r.w.e[0], r.w.ld[0], Z, ldz, st);
    STS_HIP(hipStreamSynchronize(st));
  });
}

sts_status sts_pcg_mg_mixed(const sts_space* space, double shift, const double* B, int64_t ldb,
                            double* X, int64_t ldx, int32_t ncols, double rtol, int32_t maxit,
                            int32_t* iters, void* stream) {
  sts_status bad = STS_OK;
  sts_status s = run_guarded([&] {
    Grid g;
    const MGPlan plan = require_mg_mixed(space, shift, &g);
    STS_REQUIRE(ncols >= 1 && ncols <= kMaxCols, STS_E_INVALID, "ncols must be 1..8");
    STS_REQUIRE(B && X && ldb >= g.nh && ldx >= g.nh, STS_E_INVALID, "bad buffers");
    STS_REQUIRE(rtol > 0.0 && maxit >= 1, STS_E_INVALID, "bad rtol / maxit");
    hipStream_t st = static_cast<hipStream_t>(stream);
    MGRunner r;
    r.setup(plan);
    const double* bcols[kMaxCols];
    for (int c = 0; c < ncols; ++c) bcols[c] = B + c * ldb;
    CGScal out[kMaxCols];
    r.run(X, ldx, ncols, bcols, rtol, maxit, out, st);
    STS_HIP(hipStreamSynchronize(st));
    bad = cg_status(out, ncols, iters);
  });
  if (s == STS_OK && bad != STS_OK) {
    set_error(bad == STS_E_NUMERIC ? "preconditioned CG breakdown"
                                   : "preconditioned CG reached maxit");
    return bad;
  }
  return s;
}

sts_status sts_pcg_mg_refined(const sts_space* space, const double* B, int64_t ldb, double* X,
                              int64_t ldx, int32_t ncols, double rtol, int32_t maxit,
                              int64_t* iters_fp32, int64_t* iters_fp64, int64_t* rounds,
                              void* stream) {
  return run_guarded([&] {
    Grid g;
    const MGPlan plan = require_mg(space, &g);
    STS_REQUIRE(plan.dim == 3 && plan.nlev >= 1, STS_E_INVALID,
                "the refined FP32 solve needs a 3-D grid with a smoothed multigrid level "
                "(n > 63, halving to <= 63)");
    STS_REQUIRE(ncols >= 1 && ncols <= kMaxCols, STS_E_INVALID, "ncols must be 1..8");
    STS_REQUIRE(B && X && ldb >= g.nh && ldx >= g.nh, STS_E_INVALID, "bad buffers");
    STS_REQUIRE(rtol > 0.0 && rtol < 1.0 && maxit >= 1, STS_E_INVALID, "bad rtol / maxit");
    hipStream_t st = static_cast<hipStream_t>(stream);
    MGRunner r;
    r.setup(plan);
    const double* bcols[kMaxCols];
    for (int c = 0; c < ncols; ++c) bcols[c] = B + c * ldb;
    RefineCount cnt;
    refined_kx_solve(r, g.nh, ncols, bcols, X, ldx, rtol, maxit, 0, cnt, st);
    STS_HIP(hipStreamSynchronize(st));
    if (iters_fp32) *iters_fp32 = cnt.its32;
    if (iters_fp64) *iters_fp64 = cnt.its64;
    if (rounds) *rounds = cnt.rounds;
  });
}

sts_status sts_mg_vcycle(const sts_space* space, const double* R, int64_t ldr, double* Z,
                         int64_t ldz, int32_t ncols, void* stream) {
  return run_guarded([&] {
    Grid g;
    const MGPlan plan = require_mg(space, &g);
    STS_REQUIRE(ncols >= 1 && ncols <= kMaxCols, STS_E_INVALID, "ncols must be 1..8");
    STS_REQUIRE(R && Z && ldr >= g.nh && ldz >= g.nh, STS_E_INVALID, "bad buffers");
    hipStream_t st = static_cast<hipStream_t>(stream);
    MGRunner r;
    r.setup(plan);
    copy_cols(g.nh, ncols, R, ldr, r.w.b[0], r.w.ld[0], st);
    int cols[kMaxCols];
    for (int c = 0; c < ncols; ++c) cols[c] = c;
    mg_vcycle(r.w, nullptr, cols, ncols, false, st);
    copy_cols(g.nh, ncols, r.w.e[0], r.w.ld[0], Z, ldz, st);
    STS_HIP(hipStreamSynchronize(st));
  });
}

sts_status sts_m_orthonormalize(const sts_space* space, const double* V, const double* MV,
                                int64_t ldv, int64_t k, double* W, double* MW, int64_t ldw,
                                int32_t ncols, double defl_tol, int32_t* kept,
                                int32_t* keep_idx, void* stream) {
  return run_guarded([&] {
    validate_space(space);
    const Grid g = make_grid(*space);
    STS_REQUIRE(ncols >= 1 && ncols <= 16, STS_E_INVALID, "ncols must be 1..16");
    STS_REQUIRE(k >= 0 && (k == 0 || (V && MV && ldv >= g.nh)), STS_E_INVALID, "bad basis");
    STS_REQUIRE(W && MW && ldw >= g.nh && kept, STS_E_INVALID, "bad block buffers");
    STS_REQUIRE(defl_tol >= 0.0 && defl_tol < 1.0, STS_E_INVALID, "bad defl_tol");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Stencil K = make_stencil(*space, STS_OP_K), M = make_stencil(*space, STS_OP_M);
    Scratch sc;
    const int64_t nh = g.nh;
    OrthScratch s;
    s.part = sc.get<double>(gemm_tn_partial_size(nh, (int)std::max<int64_t>(k, 16)));
    s.G = sc.get<double>(256);
    s.ldc = std::max<int64_t>(k, 1);
    s.C = sc.get<double>(s.ldc * 16);
    s.norm0 = sc.get<double>(16);
    s.Rinv = sc.get<double>(256);
    s.info = sc.get<CholInfo>(1);
    CholInfo hbuf;
    s.host = &hbuf;
    int idx[16];
    const int nk = orthonormalize_block(g, K, M, V, MV, ldv, k, W, MW, ldw, ncols, defl_tol, s,
                                        idx, st);
    STS_HIP(hipStreamSynchronize(st));
    *kept = nk;
    if (keep_idx)
      for (int j = 0; j < ncols; ++j) keep_idx[j] = j < nk ? idx[j] : -1;
  });
}

sts_status sts_gram(int64_t rows, int32_t m, int32_t n, const double* A, int64_t lda,
                    const double* B, int64_t ldb, double* C, int64_t ldc, void* stream) {
  return run_guarded([&] {
    STS_REQUIRE(rows >= 0 && m >= 1 && n >= 1 && n <= 16, STS_E_INVALID, "bad sizes");
    STS_REQUIRE(A && B && C && lda >= rows && ldb >= rows && ldc >= m, STS_E_INVALID,
                "bad buffers");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch sc;
    double* part = sc.get<double>(gemm_tn_partial_size(std::max<int64_t>(rows, 1), m));
    gemm_tn(rows, m, n, A, lda, B, ldb, C, ldc, part, st);
    STS_HIP(hipStreamSynchronize(st));
  });
}

sts_status sts_gram_fp32(int64_t rows, int32_t m, int32_t n, const float* A, int64_t lda,
                         const double* B, int64_t ldb, double* C, int64_t ldc, void* stream) {
  return run_guarded([&] {
    STS_REQUIRE(rows >= 0 && m >= 1 && n >= 1 && n <= 16, STS_E_INVALID, "bad sizes");
    STS_REQUIRE(A && B && C && lda >= rows && ldb >= rows && ldc >= m, STS_E_INVALID,
                "bad buffers");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch sc;
    float* part = sc.get<float>(gemm_tn_partial_size(std::max<int64_t>(rows, 1), m));
    gemm_tn32(rows, m, n, A, lda, B, ldb, C, ldc, part, st);
    STS_HIP(hipStreamSynchronize(st));
  });
}

sts_status sts_basis_update(int64_t rows, int32_t m, int32_t n, const double* A, int64_t lda,
                            const double* C, int64_t ldc, double* W, int64_t ldw, void* stream) {
  return run_guarded([&] {
    STS_REQUIRE(rows >= 0 && m >= 1 && n >= 1 && n <= 16, STS_E_INVALID, "bad sizes");
    STS_REQUIRE(A && C && W && lda >= rows && ldc >= m && ldw >= rows, STS_E_INVALID,
                "bad buffers");
    hipStream_t st = static_cast<hipStream_t>(stream);
    gemm_nn_sub(rows, m, n, A, lda, C, ldc, W, ldw, st);
    STS_HIP(hipStreamSynchronize(st));
  });
}

sts_status sts_sym_eig(int64_t k, const double* A, int64_t lda, double* lam, double* Q,
                       int64_t ldq, void* stream) {
  return run_guarded([&] {
    STS_REQUIRE(k >= 1 && k <= 2048, STS_E_INVALID, "k must be 1..2048");
    STS_REQUIRE(A && lam && Q && lda >= k && ldq >= k, STS_E_INVALID, "bad buffers");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch sc;
    EigWork w{};
    w.base = sc.get<double>(eig_work_doubles((int)k));
    w.status = sc.get<int>(16);
    sym_eig((int)k, A, lda, lam, Q, ldq, w, st);
    int status = 0;
    STS_HIP(hipMemcpyAsync(&status, w.status, sizeof(int), hipMemcpyDeviceToHost, st));
    STS_HIP(hipStreamSynchronize(st));
    STS_REQUIRE(status == 0, STS_E_NUMERIC, "matrix is not finite");
  });
}

sts_status sts_time_sweep(int64_t k, int64_t nt, int32_t p, const double* lam, const double* Q,
                          int64_t ldq, const double* beta, int64_t ldb, const double* F2,
                          int64_t ldf, const sts_bidiag* Dt, const sts_bidiag* Mt, double* Y,
                          int64_t ldy, void* stream) {
  return run_guarded([&] {
    STS_REQUIRE(k >= 1 && nt >= 1 && p >= 1 && p <= 4, STS_E_INVALID, "bad sizes");
    STS_REQUIRE(lam && Q && beta && F2 && Y && ldq >= k && ldb >= k && ldf >= nt && ldy >= k,
                STS_E_INVALID, "bad buffers");
    STS_REQUIRE(Dt && Mt && Dt->diag && Mt->diag && (nt == 1 || (Dt->sub && Mt->sub)),
                STS_E_INVALID, "bad time matrices");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Scratch sc;
    std::vector<double> tv(4 * nt, 0.0);
    for (int64_t l = 0; l < nt; ++l) {
      tv[l] = Dt->diag[l];
      tv[2 * nt + l] = Mt->diag[l];
      if (l + 1 < nt) {
        tv[nt + l] = Dt->sub[l];
        tv[3 * nt + l] = Mt->sub[l];
      }
    }
    double* td = sc.get<double>(4 * nt);
    STS_HIP(hipMemcpyAsync(td, tv.data(), 4 * nt * 8, hipMemcpyHostToDevice, st));
    double* qb = sc.get<double>(k * p);
    double* Z = sc.get<double>(k * nt);
    double* part = sc.get<double>(gemm_tn_partial_size(k, (int)k));
    gemm_tn(k, (int)k, p, Q, ldq, beta, ldb, qb, k, part, st);
    time_sweep((int)k, (int)nt, p, lam, qb, k, F2, ldf, TimeOps{td, td + nt, td + 2 * nt, td + 3 * nt},
               Z, k, st);
    gemm_nn((int)k, (int)nt, (int)k, Q, ldq, Z, k, Y, ldy, st);
    STS_HIP(hipStreamSynchronize(st));
  });
}

}  // extern "C"
