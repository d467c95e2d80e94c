// Serving: a request queue in front of the solver.
//
// Requests (one space-time heat problem each: space, time matrices, low-rank
// load, options) arrive at any time.  sts_server_submit copies the request's
// host inputs and returns a ticket at once.  `workers` worker threads, each
// with its own non-blocking HIP stream, take requests in arrival order
// (first come, first served).  A request is admitted only if the device
// memory it holds at the start -- problem_footprint: inputs, inner-solve work
// and the first basis capacity sts_solve maps -- fits in the budget next to
// the requests admitted and not yet released; otherwise the queue waits until
// a release frees enough.  A request that could never fit is refused at
// submission.  While it runs, its basis grows; each growth step asks the
// server for its bytes (with the transient of its copy, returned after it)
// first and waits until they fit, except for the
// oldest running request, which always proceeds (it cannot wait on requests
// younger than itself, so some request always makes progress; the budget may
// be exceeded by that request's growth).  A finished request keeps its
// problem (basis, factors) in device memory until sts_server_release, so a
// client can fetch factors, evaluate residuals or continue the solve on the
// device.
//
// Every request is solved by the same deterministic kernels as a lone
// sts_solve, so its factors do not depend on what else is being served.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sts_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t ticket = 0;
  sts_space space{};
  int64_t nt = 0;
  int p = 0;
  std::vector<double> dtd, dts, mtd, mts;   // time matrices (host copies)
  std::vector<double> F1, F2;               // packed: ld = rows
  int64_t nh = 0;
  sts_opts opts{};
  int64_t footprint = 0;                    // bytes held: admission + growth
  int64_t admit_seq = 0;                    // admission order
  Clock::time_point submitted, admitted, finished;
  bool done = false;
  sts_status status = STS_E_STATE;
  std::string error;
  sts_info info{};
  sts_problem* prob = nullptr;
};

}  // namespace

struct sts_server {
  int device = 0;
  int64_t budget = 0;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> threads;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<int64_t, std::shared_ptr<Request>> live;   // submitted and not released
  int64_t next_ticket = 1;
  int64_t next_admit = 1;
  int64_t in_use = 0, peak = 0;
  int64_t submitted = 0, completed = 0, released = 0, running = 0;
  bool stop = false;
};

namespace sts {
namespace {

constexpr int kMaxServerWorkers = 64;

double seconds(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}

// Account for `add` more bytes of a running request before its basis grows:
// wait until they fit in the budget, unless the request is the oldest one
// running (then proceed at once).
void grow_reservation(sts_server* S, Request* r, int64_t add) {
  if (add == 0) return;
  std::unique_lock<std::mutex> lk(S->mu);
  if (add < 0) {
    // a transient of the growth step returned
    S->in_use += add;
    r->footprint += add;
    lk.unlock();
    S->cv_work.notify_all();
    return;
  }
  auto oldest = [&] {
    for (auto& kv : S->live) {
      const Request& o = *kv.second;
      if (o.admit_seq > 0 && !o.done && o.admit_seq < r->admit_seq) return false;
    }
    return true;
  };
  S->cv_work.wait(lk, [&] { return S->stop || S->in_use + add <= S->budget || oldest(); });
  S->in_use += add;
  S->peak = std::max(S->peak, S->in_use);
  r->footprint += add;
}

void server_worker(sts_server* S, int w) {
  const bool dev_ok = hipSetDevice(S->device) == hipSuccess;
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] {
        return S->stop ||
               (!S->queue.empty() && S->in_use + S->queue.front()->footprint <= S->budget);
      });
      if (S->stop) return;
      r = S->queue.front();
      S->queue.pop_front();
      S->in_use += r->footprint;
      S->peak = std::max(S->peak, S->in_use);
      ++S->running;
      r->admit_seq = S->next_admit++;
      r->admitted = Clock::now();
    }
    // the head may have changed: let another idle worker look at it
    S->cv_work.notify_all();
    sts_problem* P = nullptr;
    sts_status st = STS_E_DEVICE;
    std::string err = "worker could not select the server's device";
    sts_info info{};
    if (dev_ok) {
      const sts_bidiag Dt{r->dtd.data(), r->dts.data()};
      const sts_bidiag Mt{r->mtd.data(), r->mts.data()};
      st = sts_create(&r->space, &Dt, &Mt, r->nt, r->p, r->F1.data(), r->nh, r->F2.data(), r->nt,
                      STS_MEM_HOST, S->streams[w], &P);
      if (st == STS_OK) {
        Request* rr = r.get();
        problem_set_grow_hook(P, [S, rr](int64_t add) { grow_reservation(S, rr, add); });
        st = sts_solve(P, &r->opts, &info);
      }
      err = st == STS_OK ? std::string() : std::string(sts_last_error());
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      r->prob = P;
      r->status = st;
      r->error = err;
      r->info = info;
      r->finished = Clock::now();
      r->done = true;
      // inputs are no longer needed
      std::vector<double>().swap(r->F1);
      std::vector<double>().swap(r->F2);
      --S->running;
      ++S->completed;
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();   // growth waiters: the oldest running request may have changed
  }
}

}  // namespace
}  // namespace sts

using namespace sts;

extern "C" {

int64_t sts_footprint(const sts_space* space, int64_t nt, int32_t p, const sts_opts* opts) {
  int64_t out = -1;
  const sts_status s = guarded([&] {
    STS_REQUIRE(space && nt >= 2 && p >= 1 && p <= 4, STS_E_INVALID, "sts_footprint: bad request");
    STS_REQUIRE(space->kind >= 1 && space->kind <= 3, STS_E_INVALID, "sts_footprint: bad space");
    for (int d = 0; d < 3; ++d)
      STS_REQUIRE(space->n[d] >= 1, STS_E_INVALID, "sts_footprint: bad grid");
    sts_opts o;
    if (opts) o = *opts;
    else sts_default_opts(&o);
    STS_REQUIRE(o.max_outer >= 1, STS_E_INVALID, "sts_footprint: max_outer < 1");
    out = problem_footprint(*space, nt, p, o.max_outer, o.mixed != 0);
  });
  return s == STS_OK ? out : -1;
}

sts_status sts_server_create(int32_t workers, int64_t mem_budget, sts_server** out) {
  return guarded([&] {
    STS_REQUIRE(out != nullptr, STS_E_INVALID, "sts_server_create: out is null");
    *out = nullptr;
    STS_REQUIRE(workers >= 1 && workers <= kMaxServerWorkers, STS_E_INVALID,
                "sts_server_create: 1 <= workers <= 64");
    STS_REQUIRE(mem_budget > 0, STS_E_INVALID, "sts_server_create: mem_budget must be > 0");
    auto S = std::make_unique<sts_server>();
    STS_HIP(hipGetDevice(&S->device));
    S->budget = mem_budget;
    S->streams.assign(workers, nullptr);
    for (auto& s : S->streams) STS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    try {
      for (int w = 0; w < workers; ++w) S->threads.emplace_back(server_worker, S.get(), w);
    } catch (...) {
      {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
      }
      S->cv_work.notify_all();
      for (auto& t : S->threads) t.join();
      for (auto s : S->streams) (void)hipStreamDestroy(s);
      throw Error{STS_E_DEVICE, "sts_server_create: could not start the worker threads"};
    }
    *out = S.release();
  });
}

sts_status sts_server_submit(sts_server* S, const sts_request* req, int64_t* ticket) {
  return guarded([&] {
    STS_REQUIRE(S && req && ticket, STS_E_INVALID, "sts_server_submit: null argument");
    const int64_t nt = req->nt;
    const int p = req->p;
    STS_REQUIRE(nt >= 2 && p >= 1 && p <= 4, STS_E_INVALID, "sts_server_submit: bad nt or p");
    STS_REQUIRE(req->dt_diag && req->dt_sub && req->mt_diag && req->mt_sub && req->F1 && req->F2,
                STS_E_INVALID, "sts_server_submit: null input array");
    const int64_t fp = sts_footprint(&req->space, nt, p, &req->opts);
    STS_REQUIRE(fp > 0, STS_E_INVALID, "sts_server_submit: bad space or options");
    STS_REQUIRE(fp <= S->budget, STS_E_NOMEM,
                "sts_server_submit: the request needs " + std::to_string(fp) +
                    " bytes of device memory, above the server's budget");
    const int64_t nh = req->space.n[0] * req->space.n[1] * req->space.n[2];
    STS_REQUIRE(req->ldf1 >= nh && req->ldf2 >= nt, STS_E_INVALID,
                "sts_server_submit: leading dimension too small");
    auto r = std::make_shared<Request>();
    r->space = req->space;
    r->nt = nt;
    r->p = p;
    r->nh = nh;
    r->opts = req->opts;
    r->footprint = fp;
    r->dtd.assign(req->dt_diag, req->dt_diag + nt);
    r->dts.assign(req->dt_sub, req->dt_sub + nt - 1);
    r->mtd.assign(req->mt_diag, req->mt_diag + nt);
    r->mts.assign(req->mt_sub, req->mt_sub + nt - 1);
    r->F1.resize((size_t)nh * p);
    r->F2.resize((size_t)nt * p);
    for (int c = 0; c < p; ++c) {
      std::copy(req->F1 + c * req->ldf1, req->F1 + c * req->ldf1 + nh, r->F1.begin() + c * nh);
      std::copy(req->F2 + c * req->ldf2, req->F2 + c * req->ldf2 + nt, r->F2.begin() + c * nt);
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      STS_REQUIRE(!S->stop, STS_E_STATE, "sts_server_submit: the server is shutting down");
      r->ticket = S->next_ticket++;
      r->submitted = Clock::now();
      S->queue.push_back(r);
      S->live[r->ticket] = r;
      ++S->submitted;
      *ticket = r->ticket;
    }
    S->cv_work.notify_all();
  });
}

sts_status sts_server_wait(sts_server* S, int64_t ticket, double timeout_s, sts_result* res,
                           sts_problem** prob) {
  return guarded([&] {
    STS_REQUIRE(S != nullptr, STS_E_INVALID, "sts_server_wait: server is null");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->live.find(ticket);
    STS_REQUIRE(it != S->live.end(), STS_E_INVALID, "sts_server_wait: unknown or released ticket");
    std::shared_ptr<Request> r = it->second;
    auto ready = [&] { return r->done; };
    if (timeout_s < 0.0) S->cv_done.wait(lk, ready);
    else S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    STS_REQUIRE(r->done, STS_E_STATE, "sts_server_wait: request not finished yet");
    if (res) {
      std::memset(res, 0, sizeof(*res));
      res->status = r->status;
      res->queued_seconds = seconds(r->submitted, r->admitted);
      res->latency_seconds = seconds(r->submitted, r->finished);
      res->footprint = r->footprint;
      res->info = r->info;
    }
    if (prob) *prob = r->prob;
    if (r->status != STS_OK && !r->error.empty()) set_error(r->error);
  });
}

sts_status sts_server_release(sts_server* S, int64_t ticket) {
  sts_problem* P = nullptr;
  const sts_status s = guarded([&] {
    STS_REQUIRE(S != nullptr, STS_E_INVALID, "sts_server_release: server is null");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->live.find(ticket);
    STS_REQUIRE(it != S->live.end(), STS_E_INVALID,
                "sts_server_release: unknown or released ticket");
    STS_REQUIRE(it->second->done, STS_E_STATE, "sts_server_release: request not finished yet");
    P = it->second->prob;
    S->in_use -= it->second->footprint;
    S->live.erase(it);
    ++S->released;
  });
  if (s != STS_OK) return s;
  sts_destroy(P);
  S->cv_work.notify_all();
  return STS_OK;
}

sts_status sts_server_get_stats(sts_server* S, sts_server_stats* out) {
  return guarded([&] {
    STS_REQUIRE(S && out, STS_E_INVALID, "sts_server_get_stats: null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->released = S->released;
    out->queued = (int64_t)S->queue.size();
    out->running = S->running;
    out->mem_in_use = S->in_use;
    out->mem_peak = S->peak;
    out->mem_budget = S->budget;
  });
}

void sts_server_destroy(sts_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->queue.clear();
  }
  S->cv_work.notify_all();
  for (auto& t : S->threads) t.join();
  for (auto& kv : S->live) sts_destroy(kv.second->prob);
  S->live.clear();
  for (auto s : S->streams) (void)hipStreamDestroy(s);
  delete S;
}

}  // extern "C"
