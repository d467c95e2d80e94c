// Executor for many independent problems on one GPU.
//
// A solve is a host-sequenced chain of small launches with a few host waits
// per outer iteration (deflation decisions, inner-solve states, residual
// checks).  For the small grids of a batch (63^2 .. 255^2) each launch fills a
// fraction of the 256 compute units and the host waits leave the GPU idle,
// so one problem at a time uses the chip poorly.  The pool runs several
// solves at once: each worker is a host thread with its own non-blocking HIP
// stream; a worker takes the next problem from a shared list ordered by
// estimated cost, largest first (the LPT rule, which bounds the makespan of
// uneven jobs by 4/3 of the optimum), binds it to its stream for the
// duration of the solve and binds it back afterwards.
//
// The kernels take no decision from timing or from other problems, so a
// problem solved in the pool gives bitwise the same factors as solved alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "sts_internal.h"

struct sts_pool {
  int device = 0;
  std::vector<hipStream_t> streams;
  ~sts_pool() {
    for (hipStream_t s : streams)
      if (s) (void)hipStreamDestroy(s);
  }
};

namespace sts {
namespace {

constexpr int kMaxWorkers = 64;

// Solve probs[order[j]] for j = next++, ... on worker w until the list is empty.
void pool_worker(sts_pool* pool, int w, int n, sts_problem* const* probs, const int* order,
                 const sts_opts* opts, int nopts, sts_info* infos, std::atomic<int>* next,
                 sts_status* status, std::string* err) {
  if (hipSetDevice(pool->device) != hipSuccess) {
    for (int j; (j = next->fetch_add(1)) < n;) {
      status[order[j]] = STS_E_DEVICE;
      err[order[j]] = "worker could not select the pool's device";
    }
    return;
  }
  for (int j; (j = next->fetch_add(1)) < n;) {
    const int i = order[j];
    sts_problem* P = probs[i];
    const hipStream_t home = problem_stream(P);
    sts_status s = guarded([&] { problem_bind_stream(P, pool->streams[w]); });
    if (s == STS_OK) {
      const sts_opts* o = nopts == 0 ? nullptr : &opts[nopts == 1 ? 0 : i];
      s = sts_solve(P, o, infos ? &infos[i] : nullptr);
    }
    if (s != STS_OK) err[i] = sts_last_error();
    const sts_status back = guarded([&] { problem_bind_stream(P, home); });
    if (s == STS_OK && back != STS_OK) {
      s = back;
      err[i] = sts_last_error();
    }
    status[i] = s;
  }
}

}  // namespace
}  // namespace sts

using namespace sts;

extern "C" {

sts_status sts_pool_create(int32_t workers, sts_pool** out) {
  return guarded([&] {
    STS_REQUIRE(out != nullptr, STS_E_INVALID, "sts_pool_create: out is null");
    *out = nullptr;
    STS_REQUIRE(workers >= 1 && workers <= kMaxWorkers, STS_E_INVALID,
                "sts_pool_create: 1 <= workers <= 64");
    auto p = std::make_unique<sts_pool>();
    STS_HIP(hipGetDevice(&p->device));
    p->streams.assign(workers, nullptr);
    for (auto& s : p->streams) STS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    *out = p.release();
  });
}

sts_status sts_pool_workers(const sts_pool* pool, int32_t* workers) {
  return guarded([&] {
    STS_REQUIRE(pool && workers, STS_E_INVALID, "sts_pool_workers: null argument");
    *workers = (int32_t)pool->streams.size();
  });
}

sts_status sts_pool_solve(sts_pool* pool, int32_t n, sts_problem* const* probs,
                          const sts_opts* opts, int32_t nopts, sts_info* infos,
                          sts_status* status) {
  std::vector<sts_status> st;
  std::vector<std::string> err;
  const sts_status pre = guarded([&] {
    STS_REQUIRE(pool != nullptr, STS_E_INVALID, "sts_pool_solve: pool is null");
    STS_REQUIRE(n >= 0, STS_E_INVALID, "sts_pool_solve: n < 0");
    STS_REQUIRE(n == 0 || probs != nullptr, STS_E_INVALID, "sts_pool_solve: problems is null");
    STS_REQUIRE(nopts == 0 || nopts == 1 || nopts == n, STS_E_INVALID,
                "sts_pool_solve: nopts must be 0, 1 or n");
    STS_REQUIRE(nopts == 0 || opts != nullptr, STS_E_INVALID, "sts_pool_solve: opts is null");
    for (int i = 0; i < n; ++i) {
      STS_REQUIRE(probs[i] != nullptr, STS_E_INVALID, "sts_pool_solve: a problem is null");
      for (int j = 0; j < i; ++j)
        STS_REQUIRE(probs[j] != probs[i], STS_E_INVALID,
                    "sts_pool_solve: a problem appears twice");
    }
    st.assign(n, STS_E_STATE);
    err.assign(n, std::string());
  });
  if (pre != STS_OK) return pre;
  if (n == 0) return STS_OK;
  // largest estimated cost first; ties by index
  std::vector<double> cost(n);
  for (int i = 0; i < n; ++i) cost[i] = problem_cost(probs[i]);
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::atomic<int> next{0};
  const int nw = std::min<int>((int)pool->streams.size(), n);
  std::vector<std::thread> th;
  sts_status spawn = STS_OK;
  try {
    for (int w = 0; w < nw; ++w)
      th.emplace_back(pool_worker, pool, w, (int)n, probs, order.data(), opts, (int)nopts, infos,
                      &next, st.data(), err.data());
  } catch (...) {
    spawn = STS_E_DEVICE;   // fewer workers than asked; those started finish the list
  }
  if (th.empty()) {
    return guarded([&] { throw Error{STS_E_DEVICE, "sts_pool_solve: no worker thread started"}; });
  }
  for (auto& t : th) t.join();
  (void)spawn;
  if (status)
    for (int i = 0; i < n; ++i) status[i] = st[i];
  for (int i = 0; i < n; ++i) {
    if (st[i] != STS_OK) {
      const std::string msg = "problem " + std::to_string(i) + ": " + err[i];
      const sts_status code = st[i];
      return guarded([&] { throw Error{code, msg}; });
    }
  }
  return STS_OK;
}

void sts_pool_destroy(sts_pool* pool) { delete pool; }

}  // extern "C"
