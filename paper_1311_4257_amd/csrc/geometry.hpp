// Integer geometry of the directional octree (Section 2.2).
//
// Boxes of one level are addressed by integer coordinates i in [0, 2^l)^3;
// an offset n = i_A - i_B relates two boxes of the same level of width w.
//
// Near field: A is in N^B when it meets the closed ball about c_B of radius
// R(w) = max(sqrt(3) w / 2, 3 w^2 / 4)  (the definition gives the first radius,
// the proof of Proposition 1 the second; both are honoured).  The squared
// distance from c_B to box A is (w^2 / 4) S(n) with
// S(n) = sum_{n_k != 0} (2 |n_k| - 1)^2, so the test is 4 S(n) <= max(12, 9 w^2).
// For w < 1 this is adjacency (S <= 3).
//
// Wedges: at width w >= 1 the directions are the cells of a w x w grid on the
// six faces of the cube (6 w^2 wedges, angle O(1/w)).  Offset n goes to face
// 2a + [n_a < 0], a the axis of largest |n_k| (ties: smallest axis), and on the
// two other axes (ascending) to cell ceil((n_t + |n_a|) w / (2 |n_a|)) - 1,
// clamped to [0, w-1]; a box on a cell boundary goes to the lower cell.  A
// wedge (f, i, j) at width 2w lies in wedge (f, i/2, j/2) at width w (Figure 2).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <vector>

namespace dfmm {

// The scalar tests below are used by the host and by the list kernels.
#define DFMM_HD __host__ __device__ inline

DFMM_HD int64_t near_sum(int64_t nx, int64_t ny, int64_t nz) {
  auto t = [](int64_t v) -> int64_t {
    v = v < 0 ? -v : v;
    return v ? (2 * v - 1) * (2 * v - 1) : 0;
  };
  return t(nx) + t(ny) + t(nz);
}

// 4 * max(3, 9 w^2 / 4) for w = 2^e2 / 2 (e2 = log2(2w); e2 = 0 is w = 1/2).
DFMM_HD int64_t near_limit4_e2(int e2) {
  // 9 w^2 = 9 * 4^e2 / 4 ; for e2 = 0 that is 2.25 < 12
  if (e2 <= 1) return 12;  // w <= 1: 9 w^2 <= 9 < 12
  int64_t w = int64_t(1) << (e2 - 1);
  int64_t v = 9 * w * w;
  return v > 12 ? v : 12;
}

DFMM_HD bool is_near_e2(int64_t nx, int64_t ny, int64_t nz, int e2) {
  return 4 * near_sum(nx, ny, nz) <= near_limit4_e2(e2);
}

// Wedge index of a nonzero offset at HF width w (a power of two >= 1).
DFMM_HD int direction(int64_t nx, int64_t ny, int64_t nz, int64_t w) {
  int64_t n[3] = {nx, ny, nz};
  int64_t m = 0;
  for (int k = 0; k < 3; ++k) m = (n[k] < 0 ? -n[k] : n[k]) > m ? (n[k] < 0 ? -n[k] : n[k]) : m;
  int a = 0;
  while ((n[a] < 0 ? -n[a] : n[a]) != m) ++a;
  int face = 2 * a + (n[a] < 0 ? 1 : 0);
  int64_t c[2];
  int ci = 0;
  for (int t = 0; t < 3; ++t) {
    if (t == a) continue;
    int64_t p = (n[t] + m) * w;
    int64_t q = 2 * m;
    int64_t cc = (p + q - 1) / q - 1;  // p >= 0, q > 0: ceil(p/q) - 1
    if (cc < 0) cc = 0;
    if (cc > w - 1) cc = w - 1;
    c[ci++] = cc;
  }
  return int((face * w + c[0]) * w + c[1]);
}

// Wedge at width w2/2 containing wedge l of width w2.
DFMM_HD int direction_down(int l, int64_t w2) {
  int64_t w = w2 / 2;
  int64_t face = l / (w2 * w2);
  int64_t rem = l % (w2 * w2);
  int64_t i = rem / w2, j = rem % w2;
  return int((face * w + i / 2) * w + j / 2);
}

// All offsets n with A in N^B at the width coded by e2 (n = 0 included).
inline std::vector<int64_t> near_offsets_e2(int e2) {
  int64_t lim = near_limit4_e2(e2);
  int64_t r = 0;
  while (4 * (2 * (r + 1) - 1) * (2 * (r + 1) - 1) <= lim) ++r;
  std::vector<int64_t> out;
  for (int64_t x = -r; x <= r; ++x)
    for (int64_t y = -r; y <= r; ++y)
      for (int64_t z = -r; z <= r; ++z)
        if (4 * near_sum(x, y, z) <= lim) {
          out.push_back(x);
          out.push_back(y);
          out.push_back(z);
        }
  return out;
}

// Offsets that can appear in an interaction list at the width coded by e2:
// not near at that width, but the parent offset floor((o + n) / 2) is near at
// the parent width for some child position o.
inline std::vector<int64_t> list_offsets_e2(int e2) {
  int64_t lim2 = near_limit4_e2(e2 + 1);
  int64_t rp = 0;
  while (4 * (2 * (rp + 1) - 1) * (2 * (rp + 1) - 1) <= lim2) ++rp;
  int64_t r = 2 * rp + 2;
  auto fdiv2 = [](int64_t v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); };
  std::vector<int64_t> out;
  for (int64_t x = -r; x <= r; ++x)
    for (int64_t y = -r; y <= r; ++y)
      for (int64_t z = -r; z <= r; ++z) {
        if (is_near_e2(x, y, z, e2)) continue;
        bool ok = false;
        for (int o = 0; o < 8 && !ok; ++o) {
          int64_t mx = fdiv2(x + (o & 1)), my = fdiv2(y + ((o >> 1) & 1)),
                  mz = fdiv2(z + ((o >> 2) & 1));
          ok = 4 * near_sum(mx, my, mz) <= lim2;
        }
        if (ok) {
          out.push_back(x);
          out.push_back(y);
          out.push_back(z);
        }
      }
  return out;
}

}  // namespace dfmm
