// The serving scheduler (batcher.hpp) on the host, with a stand-in device: the
// launch callback records each pass and the test (or a "device" thread)
// reports its completion.  Built with g++ by tests/test_host_sanitizers.py,
// once under AddressSanitizer / UndefinedBehaviorSanitizer and once under
// ThreadSanitizer; exits non-zero (or the sanitizer aborts) on the first
// failure.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <memory>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "batcher.hpp"

using namespace dfmm;

#define CHECK(c)                                                                \
  do {                                                                          \
    if (!(c)) {                                                                 \
      std::fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                             \
    }                                                                           \
  } while (0)

// Stand-in device: passes are recorded in launch order and finish only when
// the test says so (or, with `autorun`, after a short random delay on a
// device thread).  It also checks that a plan never has two passes in flight.
struct Device {
  struct Launch {
    int plan, n;
    int64_t pass;
    std::vector<int> nrhs;
  };
  std::mutex m;
  std::condition_variable cv;
  std::vector<Launch> launches;
  std::vector<int> inflight;
  int fail_plan = -1;  // launches of this plan return DFMM_EDEVICE
  std::atomic<bool> overlap{false};
  Batcher* B = nullptr;
  bool autorun = false;
  std::deque<int64_t> pending;
  bool quit = false;
  std::thread th;

  explicit Device(int nplans) : inflight(size_t(nplans), 0) {}
  ~Device() { stop(); }

  Batcher::LaunchFn fn() {
    return [this](int p, const std::vector<const ServeReq*>& rs, int n, int64_t b) -> int {
      std::lock_guard<std::mutex> lk(m);
      if (p == fail_plan) return DFMM_EDEVICE;
      int tot = 0;
      Launch L{p, n, b, {}};
      for (const ServeReq* r : rs) {
        L.nrhs.push_back(r->nrhs);
        tot += r->nrhs;
      }
      if (tot != n) std::exit(3);
      if (inflight[size_t(p)]++ != 0) overlap = true;
      launches.push_back(L);
      if (autorun) pending.push_back(b);
      cv.notify_all();
      return DFMM_OK;
    };
  }
  // blocks until `count` passes have been launched
  void wait_launches(size_t count) {
    std::unique_lock<std::mutex> lk(m);
    cv.wait(lk, [&]() { return launches.size() >= count; });
  }
  void finish(int64_t b) {
    int p = -1;
    {
      std::lock_guard<std::mutex> lk(m);
      for (const Launch& L : launches)
        if (L.pass == b) p = L.plan;
      CHECK(p >= 0);
      --inflight[size_t(p)];
    }
    B->complete(b, DFMM_OK);
  }
  void start_autorun() {
    autorun = true;
    th = std::thread([this]() {
      std::mt19937 rng(7);
      for (;;) {
        int64_t b;
        {
          std::unique_lock<std::mutex> lk(m);
          cv.wait(lk, [&]() { return quit || !pending.empty(); });
          if (pending.empty()) return;
          b = pending.front();
          pending.pop_front();
        }
        std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));
        finish(b);
      }
    });
  }
  void stop() {
    {
      std::lock_guard<std::mutex> lk(m);
      quit = true;
    }
    cv.notify_all();
    if (th.joinable()) th.join();
  }
  size_t count() {
    std::lock_guard<std::mutex> lk(m);
    return launches.size();
  }
  Launch at(size_t i) {
    std::lock_guard<std::mutex> lk(m);
    return launches[i];
  }
};

static char buf[1 << 16];
static const void* F(int i) { return buf + 2 * i; }
static void* U(int i) { return buf + 2 * i + 1; }

// workspace of 10 bytes per right-hand side
static size_t ws10(int, int n) { return size_t(10) * size_t(n > 0 ? n : 0); }

static std::unique_ptr<Batcher> make(Device& d, int np, size_t resident, size_t budget, int max_rhs, int max_req,
                                     bool single) {
  auto B = std::make_unique<Batcher>(np, resident, budget, max_rhs, max_req, single, ws10, d.fn());
  d.B = B.get();
  return B;
}

static int64_t submit(Batcher& B, int p, int nrhs, int i) {
  int64_t t = -1;
  CHECK(B.submit(p, F(i), U(i), nrhs, &t) == DFMM_OK);
  return t;
}

// requests queued while the plan is busy form the next pass in order, up to the
// rhs cap; a request longer than the rest of the cap starts the pass after
static void test_rhs_cap() {
  Device d(1);
  auto B = make(d, 1, 0, size_t(1) << 40, 16, 32, false);
  const int64_t t0 = submit(*B, 0, 1, 0);
  d.wait_launches(1);
  const int64_t t1 = submit(*B, 0, 4, 1), t2 = submit(*B, 0, 4, 2), t3 = submit(*B, 0, 16, 3),
                t4 = submit(*B, 0, 1, 4);
  d.finish(0);
  d.wait_launches(2);
  CHECK(d.at(1).nrhs == std::vector<int>({4, 4}) && d.at(1).n == 8);
  d.finish(1);
  d.wait_launches(3);
  CHECK(d.at(2).nrhs == std::vector<int>({16}));
  d.finish(2);
  d.wait_launches(4);
  CHECK(d.at(3).nrhs == std::vector<int>({1}));
  d.finish(3);
  B->drain();
  double ts = -1, td = -1;
  for (int64_t t : {t0, t1, t2, t3, t4}) {
    CHECK(B->wait(t, &ts, &td) == DFMM_OK);
    CHECK(ts >= 0 && td >= ts);
  }
  CHECK(B->request_pass(t1) == 1 && B->request_pass(t2) == 1 && B->request_pass(t3) == 2);
  CHECK(B->passes() == 4);
  ServePass P;
  CHECK(B->pass(1, &P) && P.plan == 0 && P.nrhs == 8 && P.ids.size() == 2);
  CHECK(!B->pass(4, &P));
}

// a request above the cap runs alone; a pass holds at most max_req requests
static void test_request_count_cap() {
  Device d(1);
  auto B = make(d, 1, 0, size_t(1) << 40, 4, 8, false);
  submit(*B, 0, 16, 0);
  d.wait_launches(1);
  CHECK(d.at(0).nrhs == std::vector<int>({16}));
  for (int i = 0; i < 11; ++i) submit(*B, 0, 1, 1 + i);
  d.finish(0);
  d.wait_launches(2);
  CHECK(d.at(1).nrhs.size() == 4);  // the rhs cap (4) binds before the count cap (8)
  d.finish(1);
  d.wait_launches(3);
  d.finish(2);
  d.wait_launches(4);
  CHECK(d.at(3).nrhs.size() == 3);
  d.finish(3);
  B->drain();
  Device d2(1);
  auto B2 = make(d2, 1, 0, size_t(1) << 40, 1000, 8, false);
  submit(*B2, 0, 1, 0);
  d2.wait_launches(1);
  for (int i = 0; i < 11; ++i) submit(*B2, 0, 1, 1 + i);
  d2.finish(0);
  d2.wait_launches(2);
  CHECK(d2.at(1).nrhs.size() == 8);
  d2.finish(1);
  d2.wait_launches(3);
  CHECK(d2.at(2).nrhs.size() == 3);
  d2.finish(2);
  B2->drain();
}

// admission: resident 2000, 10 B per rhs; plan 1 has run 8 rhs (80 B)
static void test_admission() {
  Device d(2);
  auto B = make(d, 2, 2000, 2000 + 80 + 100, 64, 32, false);
  submit(*B, 1, 8, 0);
  d.wait_launches(1);
  d.finish(0);
  B->drain();
  CHECK(B->footprint_now() == 2080);
  submit(*B, 0, 1, 1);  // plan 0 busy with 1 rhs
  d.wait_launches(2);
  submit(*B, 0, 4, 2);
  submit(*B, 0, 4, 3);
  submit(*B, 0, 4, 4);
  d.finish(1);
  d.wait_launches(3);
  CHECK(d.at(2).nrhs == std::vector<int>({4, 4}));  // 8 rhs -> 2160 fits, 12 -> 2200 does not
  CHECK(B->footprint_now() <= 2180);
  d.finish(2);
  d.wait_launches(4);
  CHECK(d.at(3).nrhs == std::vector<int>({4}));  // workspaces only grow: 4 rhs costs nothing new
  d.finish(3);
  B->drain();
  // a request that cannot fit even alone is refused at submission
  int64_t t = -1;
  CHECK(B->submit(0, F(5), U(5), 11, &t) == DFMM_ENOMEM);
  CHECK(B->submit(0, F(5), U(5), 10, &t) == DFMM_OK);
  d.wait_launches(5);
  d.finish(4);
  B->drain();
  CHECK(B->wait(t, nullptr, nullptr) == DFMM_OK);
}

// a queued request that stops fitting because another plan's workspace grew
// fails with DFMM_ENOMEM when it reaches the front of its queue
static void test_enomem_at_front() {
  Device d(2);
  auto B = make(d, 2, 0, 150, 64, 32, false);
  const int64_t t0 = submit(*B, 0, 1, 0);
  d.wait_launches(1);
  const int64_t tb = submit(*B, 0, 10, 1);  // fits now: 100 + 0
  const int64_t ta = submit(*B, 1, 8, 2);   // plan 1 idle: runs at once, its workspace grows to 80
  d.wait_launches(2);
  CHECK(d.at(1).plan == 1);
  d.finish(0);
  d.finish(1);
  B->drain();
  CHECK(B->wait(t0, nullptr, nullptr) == DFMM_OK);
  CHECK(B->wait(ta, nullptr, nullptr) == DFMM_OK);
  CHECK(B->wait(tb, nullptr, nullptr) == DFMM_ENOMEM);
  CHECK(d.count() == 2);
}

// single mode: one request per pass, one pass at a time, submission order
static void test_single_mode() {
  Device d(2);
  auto B = make(d, 2, 0, size_t(1) << 40, 64, 32, true);
  submit(*B, 0, 2, 0);
  d.wait_launches(1);
  submit(*B, 1, 1, 1);
  submit(*B, 0, 3, 2);
  submit(*B, 1, 4, 3);
  for (int k = 0; k < 4; ++k) {
    d.wait_launches(size_t(k + 1));
    std::this_thread::sleep_for(std::chrono::milliseconds(2));
    CHECK(d.count() == size_t(k + 1));  // nothing else starts while a pass runs
    d.finish(k);
  }
  B->drain();
  const int want_plan[4] = {0, 1, 0, 1}, want_n[4] = {2, 1, 3, 4};
  for (int k = 0; k < 4; ++k) CHECK(d.at(size_t(k)).plan == want_plan[k] && d.at(size_t(k)).n == want_n[k]);
}

// a failed launch fails its requests; the plan takes passes again afterwards
static void test_launch_failure() {
  Device d(2);
  d.fail_plan = 1;
  auto B = make(d, 2, 0, size_t(1) << 40, 64, 32, false);
  const int64_t t = submit(*B, 1, 2, 0);
  CHECK(B->wait(t, nullptr, nullptr) == DFMM_EDEVICE);
  {
    std::lock_guard<std::mutex> lk(d.m);
    d.fail_plan = -1;
  }
  const int64_t t2 = submit(*B, 1, 2, 1);
  d.wait_launches(1);
  d.finish(1);
  CHECK(B->wait(t2, nullptr, nullptr) == DFMM_OK);
}

// argument errors
static void test_arguments() {
  Device d(1);
  auto B = make(d, 1, 0, size_t(1) << 40, 16, 32, false);
  int64_t t = 0;
  CHECK(B->submit(1, F(0), U(0), 1, &t) == DFMM_EINVAL);
  CHECK(B->submit(-1, F(0), U(0), 1, &t) == DFMM_EINVAL);
  CHECK(B->submit(0, nullptr, U(0), 1, &t) == DFMM_EINVAL);
  CHECK(B->submit(0, F(0), nullptr, 1, &t) == DFMM_EINVAL);
  CHECK(B->submit(0, F(0), U(0), 0, &t) == DFMM_EINVAL);
  CHECK(B->submit(0, F(0), U(0), 4097, &t) == DFMM_EINVAL);
  CHECK(B->submit(0, F(0), U(0), 1, nullptr) == DFMM_EINVAL);
  CHECK(B->wait(0, nullptr, nullptr) == DFMM_EINVAL);  // nothing submitted yet
  CHECK(B->wait(-1, nullptr, nullptr) == DFMM_EINVAL);
}

// many submitting threads against a device thread that finishes passes after
// random delays: every request finishes once, in exactly one pass, no plan
// runs two passes at once, caps hold; destruction waits for what is queued
static void test_concurrent() {
  const int np = 3, threads = 4, per = 300;
  Device d(np);
  auto B = make(d, np, 0, size_t(1) << 40, 16, 8, false);
  d.start_autorun();
  std::vector<std::vector<int64_t>> tickets(threads);
  std::vector<std::thread> ts;
  for (int k = 0; k < threads; ++k)
    ts.emplace_back([&, k]() {
      std::mt19937 rng(unsigned(100 + k));
      for (int i = 0; i < per; ++i) {
        const int n = 1 + int(rng() % 5);
        tickets[size_t(k)].push_back(submit(*B, int(rng() % np), n, k * per + i));
        if (rng() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 100));
      }
    });
  for (auto& t : ts) t.join();
  for (auto& v : tickets)
    for (int64_t t : v) {
      double a = 0, b = 0;
      CHECK(B->wait(t, &a, &b) == DFMM_OK && b >= a);
    }
  B->drain();
  CHECK(!d.overlap);
  std::vector<int> seen(size_t(threads * per), 0);
  const int64_t np_ = B->passes();
  int64_t total = 0;
  for (int64_t b = 0; b < np_; ++b) {
    ServePass P;
    CHECK(B->pass(b, &P));
    CHECK(P.ids.size() <= 8 && (P.nrhs <= 16 || P.ids.size() == 1));
    for (int64_t id : P.ids) ++seen[size_t(id)];
    total += int64_t(P.ids.size());
  }
  CHECK(total == threads * per);
  for (int s : seen) CHECK(s == 1);
  // destruction with requests still queued: the destructor waits for them
  for (int i = 0; i < 50; ++i) submit(*B, i % np, 1, i);
  B.reset();
  d.stop();
}

int main() {
  test_arguments();
  test_rhs_cap();
  test_request_count_cap();
  test_admission();
  test_enomem_at_front();
  test_single_mode();
  test_launch_failure();
  test_concurrent();
  std::printf("batcher: ok\n");
  return 0;
}
