// Host bookkeeping of libdfmm under AddressSanitizer / UndefinedBehaviorSanitizer:
// the workspace layout (the carving of one device buffer into the vectors of an
// apply) and the stage-timer book (which recorded event closes which stage
// interval).  Built with g++ by tests/test_host_sanitizers.py; exits non-zero
// (or the sanitizer aborts) on the first failure.
#include <cstdio>
#include <cstdlib>
#include <stdexcept>
#include <utility>
#include <vector>

#include "stagebook.hpp"
#include "workspace.hpp"

using namespace dfmm;

#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                   \
    }                                                                 \
  } while (0)

// a small tree (the bytes of its layouts are touched on the host) or the
// K = 32 ellipsoid's sizes (layouts only)
static WsShape shape(int levels, bool big = false) {
  WsShape s;
  s.N = big ? 262144 : 4096;
  s.nleaf = big ? 5297 : 262;
  s.Rlf = 96;
  for (int e = 0; e < levels; ++e) {
    s.nout.push_back((big ? 10000 : 600) >> e);
    s.nin.push_back((big ? 9000 : 500) >> e);
    s.R.push_back(104 - 8 * e);
  }
  s.pair_rows = (big ? 213402LL : 11160LL) * 96;
  return s;
}

static void check_layout(const WsShape& s, int nrhs, bool pair, bool touch) {
  const WsLayout L = ws_layout(s, nrhs, pair);
  std::vector<std::pair<size_t, size_t>> r;  // (offset, bytes)
  const size_t k = size_t(nrhs);
  r.push_back({L.fs, 8 * size_t(s.N) * k});
  r.push_back({L.unear, 16 * size_t(s.N) * k});
  r.push_back({L.flf, 8 * size_t(s.nleaf) * size_t(s.Rlf) * k});
  r.push_back({L.ulf, 8 * size_t(s.nleaf) * size_t(s.Rlf) * k});
  for (size_t e = 0; e < s.R.size(); ++e) {
    r.push_back({L.F[e], 8 * size_t(s.R[e]) * k * size_t(s.nout[e])});
    r.push_back({L.U[e], 8 * size_t(s.R[e]) * k * size_t(s.nin[e])});
  }
  if (pair) r.push_back({L.Y, 8 * size_t(s.pair_rows) * k});
  for (size_t i = 0; i < r.size(); ++i) {
    CHECK(r[i].first % kWsAlign == 0);
    CHECK(r[i].first + r[i].second <= L.total);
    for (size_t j = 0; j < i; ++j)  // no two buffers overlap
      CHECK(r[i].first + r[i].second <= r[j].first || r[j].first + r[j].second <= r[i].first);
  }
  if (!touch) return;
  // write every buffer of a host allocation of the layout's size through its offset
  std::vector<unsigned char> buf(L.total);
  for (const auto& b : r)
    for (size_t q = 0; q < b.second; ++q) buf[b.first + q] = 1;
}

int main() {
  // layouts: several depths, nrhs and both forms; sizes grow with nrhs
  for (int levels = 0; levels <= 4; ++levels)
    for (int nrhs : {1, 3, 16, 32})
      for (bool pair : {false, true}) {
        check_layout(shape(levels), nrhs, pair, true);
        check_layout(shape(levels, true), nrhs, pair, false);
      }
  CHECK(ws_layout(shape(3, true), 32, false).total > ws_layout(shape(3, true), 16, false).total);
  CHECK(ws_layout(shape(3, true), 16, true).total > ws_layout(shape(3, true), 16, false).total);
  // bad shapes and sizes past size_t are refused, not wrapped
  bool threw = false;
  try {
    WsShape s = shape(2);
    s.R.pop_back();
    (void)ws_layout(s, 1, true);
  } catch (const std::invalid_argument&) {
    threw = true;
  }
  CHECK(threw);
  threw = false;
  try {
    WsShape s = shape(1);
    s.N = int64_t(1) << 60;
    (void)ws_layout(s, 4096, true);
  } catch (const std::overflow_error&) {
    threw = true;
  }
  CHECK(threw);

  // stage book: intervals of one apply on the main stream and the side stream
  StageBook b(3 * 8, 8);
  CHECK(b.begin_apply() == 0);
  CHECK(b.side_begin() == 1);
  CHECK(b.mark(0) == 2);          // stage 0: events 0 -> 2
  CHECK(b.mark(3) == 3);          // stage 3: events 2 -> 3
  CHECK(b.side_mark(10) == 4);    // stage 10: events 1 -> 4
  CHECK(b.side_mark(10) == StageBook::kNone);  // no open side interval
  CHECK(b.mark(99) == 5);         // a stage outside the table: recorded, not summed
  double ms[11];
  int64_t cnt[11];
  b.collect(ms, cnt, 11, [](size_t a, size_t c) { return float(10 * c + a); });
  CHECK(ms[0] == 20.0 && cnt[0] == 1);
  CHECK(ms[3] == 32.0 && cnt[3] == 1);
  CHECK(ms[10] == 41.0 && cnt[10] == 1);
  CHECK(cnt[1] == 0 && cnt[2] == 0);
  CHECK(b.used == 0 && b.stage.empty());
  // the pool runs out: begin_apply refuses when an apply's share does not fit,
  // marks stop at the end of the pool
  for (int a = 0; a < 3; ++a) {
    CHECK(b.begin_apply() != StageBook::kNone);
    for (int m = 0; m < 7; ++m) CHECK(b.mark(m % 11) != StageBook::kNone);
  }
  CHECK(b.begin_apply() == StageBook::kNone);
  CHECK(b.mark(1) == StageBook::kNone);
  CHECK(b.side_begin() == StageBook::kNone);
  b.collect(ms, cnt, 11, [](size_t, size_t) { return 1.0f; });
  int64_t total = 0;
  for (int i = 0; i < 11; ++i) total += cnt[i];
  CHECK(total == 21);
  std::printf("host bookkeeping: ok\n");
  return 0;
}
