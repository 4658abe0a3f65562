// Bookkeeping of the stage timer: which recorded event closes which stage
// interval.  Plain host code (no HIP types), so that it can be exercised on its
// own; StageTimer pairs it with a pool of HIP events.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace dfmm {

struct StageBook {
  static constexpr size_t kNone = ~size_t(0);
  size_t cap = 0;              // events in the pool
  size_t per_apply = 0;        // events an apply may use at most
  std::vector<int> stage;      // per used event: the stage of the interval it closes (-1: none)
  std::vector<size_t> from;    // per used event: the event that opens that interval
  size_t used = 0;
  size_t last_main = 0;        // latest event on the apply stream
  size_t side_from = kNone;    // event that opened the side-stream interval

  StageBook(size_t cap_, size_t per_apply_) : cap(cap_), per_apply(per_apply_) {}

  // Each call returns the pool index of the event to record, or kNone when
  // nothing is to be recorded (pool exhausted, or no open interval).
  size_t begin_apply() {
    if (used + per_apply > cap) return kNone;
    stage.push_back(-1);
    from.push_back(used);
    last_main = used;
    return used++;
  }
  size_t mark(int st) {  // closes the interval since the previous apply-stream event
    if (used >= cap) return kNone;
    stage.push_back(st);
    from.push_back(last_main);
    last_main = used;
    return used++;
  }
  size_t side_begin() {
    if (used >= cap) return kNone;
    stage.push_back(-1);
    from.push_back(used);
    side_from = used;
    return used++;
  }
  size_t side_mark(int st) {
    if (used >= cap || side_from == kNone) return kNone;
    stage.push_back(st);
    from.push_back(side_from);
    side_from = kNone;
    return used++;
  }
  // Sums elapsed(from, to) per stage into ms / launches (nstages entries each,
  // zeroed first); an interval whose stage is outside [0, nstages) is skipped.
  // Resets the book.
  template <class Elapsed>
  void collect(double* ms, int64_t* launches, int nstages, Elapsed&& elapsed) {
    for (int i = 0; i < nstages; ++i) {
      ms[i] = 0.0;
      launches[i] = 0;
    }
    for (size_t i = 0; i < used; ++i) {
      const int s = stage[i];
      if (s < 0 || s >= nstages) continue;
      ms[s] += double(elapsed(from[i], i));
      launches[s] += 1;
    }
    used = 0;
    last_main = 0;
    side_from = kNone;
    stage.clear();
    from.clear();
  }
};

}  // namespace dfmm
