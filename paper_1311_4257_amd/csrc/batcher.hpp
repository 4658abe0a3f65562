// Request queue and batch scheduler of a serving process: plain C++ (no HIP
// types), so that its rules run under host sanitizers.
//
// An iterative boundary-integral solver issues one matvec per iteration
// (Section 1).  A serving process keeps the plans of several geometries
// resident and receives such requests as they come.  The Batcher holds every
// submitted request and, on a worker thread of its own, starts the next pass
// of a plan when that plan's previous pass has finished:
//
// * batched mode: the pass takes the plan's queued requests in submission
//   order, up to max_rhs right-hand sides (a longer request runs alone) and
//   max_req requests, and only while the HBM footprint stays within the
//   budget.  The footprint is the resident plans plus every plan's workspace
//   at the largest pass it has run, since workspaces only grow.  Plans whose
//   oldest queued request is older go first.  Passes of different plans run
//   concurrently;
// * single mode: one request per pass and one pass in flight at a time, in
//   submission order (the plain form, for comparison).
//
// A request that cannot fit the budget even alone fails with DFMM_ENOMEM: at
// submission if it does not fit then, otherwise when it reaches the front of
// its queue (the footprint never shrinks).  The launch callback enqueues a
// pass and returns; the pass's completion is reported with complete(), from
// any thread.  No lock is held while the callback runs.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/dfmm.h"

namespace dfmm {

struct ServeReq {
  int plan = 0;
  const void* f = nullptr;
  void* u = nullptr;
  int nrhs = 0;
  double t_submit = 0.0;  // seconds on the batcher's clock
  double t_done = 0.0;
  int64_t batch = -1;     // the pass that ran it (-1: none)
  int status = DFMM_OK;
  bool done = false;
};

struct ServePass {
  int plan = 0;
  int nrhs = 0;
  std::vector<int64_t> ids;
};

class Batcher {
 public:
  // workspace bytes of plan p at n right-hand sides (0 for n = 0)
  using WsFn = std::function<size_t(int p, int n)>;
  // enqueue pass b of plan p over the requests (total nrhs n); returns DFMM_OK,
  // after which complete(b, status) must follow exactly once, or an error code
  using LaunchFn = std::function<int(int p, const std::vector<const ServeReq*>& reqs, int n, int64_t b)>;

  Batcher(int nplans, size_t resident, size_t budget, int max_rhs, int max_req, bool single, WsFn ws,
          LaunchFn launch)
      : np_(nplans), resident_(resident), budget_(budget), max_rhs_(max_rhs), max_req_(max_req),
        single_(single), ws_(std::move(ws)), launch_(std::move(launch)), q_(size_t(nplans)),
        busy_(size_t(nplans), false), cap_(size_t(nplans), 0), t0_(std::chrono::steady_clock::now()) {
    worker_ = std::thread([this]() { loop(); });
  }
  // Waits for every submitted request to finish, then stops the worker.
  ~Batcher() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    worker_.join();
  }
  Batcher(const Batcher&) = delete;
  Batcher& operator=(const Batcher&) = delete;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
  }

  int submit(int p, const void* f, void* u, int nrhs, int64_t* ticket) {
    if (p < 0 || p >= np_ || !f || !u || !ticket || nrhs < 1 || nrhs > 4096) return DFMM_EINVAL;
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stop_) return DFMM_EINVAL;
      if (footprint(p, nrhs) > budget_) return DFMM_ENOMEM;
      ServeReq r;
      r.plan = p;
      r.f = f;
      r.u = u;
      r.nrhs = nrhs;
      r.t_submit = now();
      const int64_t id = int64_t(reqs_.size());
      reqs_.push_back(r);
      (single_ ? fifo_ : q_[size_t(p)]).push_back(id);
      ++queued_;
      *ticket = id;
    }
    cv_.notify_all();
    return DFMM_OK;
  }

  // Blocks until request `id` has finished; its status, or DFMM_EINVAL for an
  // unknown ticket.
  int wait(int64_t id, double* t_submit, double* t_done) {
    std::unique_lock<std::mutex> lk(mu_);
    if (id < 0 || id >= int64_t(reqs_.size())) return DFMM_EINVAL;
    cv_.wait(lk, [&]() { return reqs_[size_t(id)].done; });
    const ServeReq& r = reqs_[size_t(id)];
    if (t_submit) *t_submit = r.t_submit;
    if (t_done) *t_done = r.t_done;
    return r.status;
  }

  // Blocks until no request is queued or in flight.
  void drain() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&]() { return queued_ == 0 && inflight_ == 0; });
  }

  // Pass b has finished on the device (status DFMM_OK or an error code).  The
  // notification is sent under the lock: once the caller has released it, the
  // batcher may be destroyed.
  void complete(int64_t b, int status) {
    std::lock_guard<std::mutex> lk(mu_);
    finish(b, status);
    cv_.notify_all();
  }

  int64_t passes() const {
    std::lock_guard<std::mutex> lk(mu_);
    return int64_t(passes_.size());
  }
  bool pass(int64_t b, ServePass* out) const {
    std::lock_guard<std::mutex> lk(mu_);
    if (b < 0 || b >= int64_t(passes_.size())) return false;
    *out = passes_[size_t(b)];
    return true;
  }
  int64_t request_pass(int64_t id) const {
    std::lock_guard<std::mutex> lk(mu_);
    return id >= 0 && id < int64_t(reqs_.size()) ? reqs_[size_t(id)].batch : -1;
  }
  size_t footprint_now() const {
    std::lock_guard<std::mutex> lk(mu_);
    return footprint(-1, 0);
  }

 private:
  size_t ws(int p, int n) const {
    if (n <= 0) return 0;
    const auto key = std::make_pair(p, n);
    auto it = wsb_.find(key);
    if (it == wsb_.end()) it = wsb_.emplace(key, ws_(p, n)).first;
    return it->second;
  }
  // HBM held with plan p's workspace grown to n (p = -1: as things stand)
  size_t footprint(int p, int n) const {
    size_t tot = resident_;
    for (int q = 0; q < np_; ++q) tot += ws(q, q == p ? std::max(cap_[size_t(q)], n) : cap_[size_t(q)]);
    return tot;
  }

  void fail_request(int64_t id, int status) {
    ServeReq& r = reqs_[size_t(id)];
    r.status = status;
    r.t_done = now();
    r.done = true;
  }

  void finish(int64_t b, int status) {
    ServePass& s = passes_[size_t(b)];
    const double t = now();
    for (int64_t id : s.ids) {
      ServeReq& r = reqs_[size_t(id)];
      r.status = status;
      r.t_done = t;
      r.done = true;
    }
    busy_[size_t(s.plan)] = false;
    --inflight_;
  }

  // Starts pass (p, ids); the lock is released while the launch callback runs.
  void launch(std::unique_lock<std::mutex>& lk, int p, std::vector<int64_t> ids, int n) {
    busy_[size_t(p)] = true;
    ++inflight_;
    cap_[size_t(p)] = std::max(cap_[size_t(p)], n);
    const int64_t b = int64_t(passes_.size());
    std::vector<const ServeReq*> rs;
    for (int64_t id : ids) {
      reqs_[size_t(id)].batch = b;
      rs.push_back(&reqs_[size_t(id)]);  // deque elements keep their addresses
    }
    passes_.push_back(ServePass{p, n, std::move(ids)});
    lk.unlock();
    const int st = launch_(p, rs, n, b);
    lk.lock();
    if (st != DFMM_OK) {
      finish(b, st);
      cv_.notify_all();
    }
  }

  // Starts every pass that can start now; false if none could.
  bool schedule(std::unique_lock<std::mutex>& lk) {
    if (single_) {
      if (inflight_ != 0 || fifo_.empty()) return false;
      const int64_t id = fifo_.front();
      fifo_.pop_front();
      --queued_;
      const ServeReq& r = reqs_[size_t(id)];
      if (footprint(r.plan, r.nrhs) > budget_) {
        fail_request(id, DFMM_ENOMEM);
        cv_.notify_all();
        return true;
      }
      launch(lk, r.plan, {id}, r.nrhs);
      return true;
    }
    std::vector<int> idle;
    for (int p = 0; p < np_; ++p)
      if (!busy_[size_t(p)] && !q_[size_t(p)].empty()) idle.push_back(p);
    if (idle.empty()) return false;
    // oldest queued request first (ids grow with submission time)
    std::sort(idle.begin(), idle.end(), [&](int a, int b) { return q_[size_t(a)].front() < q_[size_t(b)].front(); });
    bool any = false;
    for (int p : idle) {
      if (busy_[size_t(p)]) continue;
      std::deque<int64_t>& q = q_[size_t(p)];
      std::vector<int64_t> take;
      int n = 0;
      while (!q.empty() && int(take.size()) < max_req_) {
        const int64_t id = q.front();
        const int k = reqs_[size_t(id)].nrhs;
        if (!take.empty() && n + k > max_rhs_) break;
        if (footprint(p, n + k) > budget_) {
          if (!take.empty()) break;
          q.pop_front();  // cannot fit even alone, now or later
          --queued_;
          fail_request(id, DFMM_ENOMEM);
          any = true;
          continue;
        }
        take.push_back(id);
        q.pop_front();
        --queued_;
        n += k;
      }
      if (!take.empty()) {
        launch(lk, p, std::move(take), n);
        any = true;
      }
    }
    if (any) cv_.notify_all();
    return any;
  }

  void loop() {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      if (schedule(lk)) continue;
      if (stop_ && queued_ == 0 && inflight_ == 0) return;
      cv_.wait(lk);
    }
  }

  const int np_;
  const size_t resident_, budget_;
  const int max_rhs_, max_req_;
  const bool single_;
  const WsFn ws_;
  const LaunchFn launch_;
  mutable std::mutex mu_;
  std::condition_variable cv_;
  std::deque<ServeReq> reqs_;
  std::vector<std::deque<int64_t>> q_;
  std::deque<int64_t> fifo_;
  std::vector<ServePass> passes_;
  std::vector<bool> busy_;
  std::vector<int> cap_;
  mutable std::map<std::pair<int, int>, size_t> wsb_;
  int64_t queued_ = 0, inflight_ = 0;
  bool stop_ = false;
  const std::chrono::steady_clock::time_point t0_;
  std::thread worker_;
};

}  // namespace dfmm
