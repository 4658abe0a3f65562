// Layout of an apply's workspace: one device buffer carved into the vectors of
// the evaluation pass at 256-byte aligned offsets.  Plain host code (no HIP
// types), shared by the plan-owned workspace of dfmm_apply and the caller's
// workspace of dfmm_apply_ws.
#pragma once

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <vector>

namespace dfmm {

// The sizes a plan's workspace depends on.
struct WsShape {
  int64_t N = 0;                 // points
  int64_t nleaf = 0;             // leaves
  int Rlf = 0;                   // padded leaf-level rank
  std::vector<int64_t> nout, nin;  // needed outgoing / incoming slots per HF level (index log2 w)
  std::vector<int> R;            // padded rank per HF level
  int64_t pair_rows = 0;         // complex rows of pair outputs per right-hand side (pair form)
};

// Byte offsets of every buffer for nrhs right-hand sides:
//   fs     complex [N][nrhs]          densities in tree order
//   unear  complex128 [nrhs][N]       near-field sums (tree order)
//   flf    complex [nleaf][nrhs][Rlf] leaf outgoing check potentials
//   ulf    complex [nleaf][nrhs][Rlf] leaf incoming check potentials
//   F[e]   complex [nout][nrhs][R]    HF outgoing check potentials of level e
//   U[e]   complex [nin][nrhs][R]     HF incoming check potentials of level e
//   Y      complex64 [pair_rows][nrhs]   pair outputs (pair form only; else empty)
struct WsLayout {
  size_t fs = 0, unear = 0, flf = 0, ulf = 0, Y = 0;
  std::vector<size_t> F, U;
  size_t total = 0;
};

constexpr size_t kWsAlign = 256;

inline size_t ws_round(size_t n) { return (n + kWsAlign - 1) / kWsAlign * kWsAlign; }

// Checked product of non-negative sizes (throws std::overflow_error past SIZE_MAX).
inline size_t ws_mul(size_t a, size_t b) {
  if (a != 0 && b > SIZE_MAX / a) throw std::overflow_error("workspace size overflows size_t");
  return a * b;
}

// csize: bytes of one complex entry of the densities and check potentials
// (8: complex64; 16: complex128 for float64 plans); the near-field sums are
// complex128 in both.
inline WsLayout ws_layout(const WsShape& s, int nrhs, bool pair_form, int csize = 8) {
  if (nrhs < 1 || s.N < 0 || s.nleaf < 0 || s.Rlf < 0 || s.nout.size() != s.R.size() ||
      s.nin.size() != s.R.size() || (csize != 8 && csize != 16))
    throw std::invalid_argument("bad workspace shape");
  const size_t cs = size_t(csize);
  WsLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = ws_round(off + bytes);
    if (off < at) throw std::overflow_error("workspace size overflows size_t");
    return at;
  };
  const size_t k = size_t(nrhs);
  L.fs = take(ws_mul(ws_mul(cs, size_t(s.N)), k));
  L.unear = take(ws_mul(ws_mul(16, size_t(s.N)), k));
  const size_t lf = ws_mul(ws_mul(ws_mul(cs, size_t(s.nleaf)), size_t(s.Rlf)), k);
  L.flf = take(lf);
  L.ulf = take(lf);
  for (size_t e = 0; e < s.R.size(); ++e) {
    const size_t r = ws_mul(ws_mul(cs, size_t(s.R[e])), k);
    L.F.push_back(take(ws_mul(r, size_t(s.nout[e] > 0 ? s.nout[e] : 1))));
    L.U.push_back(take(ws_mul(r, size_t(s.nin[e] > 0 ? s.nin[e] : 1))));
  }
  L.Y = take(pair_form ? ws_mul(ws_mul(8, size_t(s.pair_rows > 0 ? s.pair_rows : 1)), k) : 0);
  L.total = off > 0 ? off : kWsAlign;
  return L;
}

}  // namespace dfmm
