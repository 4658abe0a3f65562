// Octree construction: Morton keys and the stable key sort run on the device;
// the per-level box tables follow from the sorted keys (Section 2.2 and
// Section 3.1: level l is a 2^l x 2^l x 2^l grid of boxes of width K 2^-l in
// the cube [-K/2, K/2]^3; leaves have width 1/2, so D = log2(2K)).
//
// Point -> leaf: per axis ix = floor((x + K/2) * 2^D / K), clamped into
// [0, 2^D - 1], the sum rounded first in float64 and the scaling by a power of
// two exact.  The key interleaves the bits of (ix, iy, iz) with x lowest, so
// the root octant is the most significant digit.  Points are ordered by
// (key, original index): a stable LSD radix sort (radix.hip) over the 3D key
// bits of pairs whose values start as the identity.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "internal.hpp"

namespace dfmm {

namespace {

__global__ void k_morton(const double* __restrict__ pts, int64_t n, double half, double scale,
                         int D, unsigned long long* __restrict__ key, int* __restrict__ idx) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t top = (int64_t(1) << D) - 1;
  unsigned long long k = 0;
  for (int a = 0; a < 3; ++a) {
    double s = __dadd_rn(pts[3 * i + a], half);
    double x = __dmul_rn(s, scale);
    double f = floor(x);
    int64_t c = f < 0.0 ? 0 : (f > double(top) ? top : int64_t(f));
    for (int b = 0; b < D; ++b) k |= (unsigned long long)((c >> b) & 1) << (3 * b + a);
  }
  key[i] = k;
  idx[i] = int(i);
}

}  // namespace

// extra > 0 (adaptive trees): the points are keyed and sorted at level D + extra
// and the box tables cover every level down to it (all boxes, split or not);
// the leaf tables below are those of level D, which a uniform plan uses.
void build_tree_device(dfmm_plan_s& P, const double* points, int64_t N, double K, Tree& T, DevTree& DT,
                       int extra) {
  int D = 0;
  while (std::ldexp(1.0, D) < 2.0 * K) ++D;
  T.D = D;
  const int Dk = D + extra;  // depth of the sort keys
  if (3 * Dk > 63) throw Error{DFMM_EUNSUPPORTED, "tree too deep for 64-bit Morton keys"};
  DevBuf dpts, k0, k1, v0, v1;
  dpts.alloc(sizeof(double) * 3 * N);
  DFMM_HIP(hipMemcpy(dpts.p, points, sizeof(double) * 3 * N, hipMemcpyHostToDevice));
  k0.alloc(sizeof(unsigned long long) * N);
  k1.alloc(sizeof(unsigned long long) * N);
  v0.alloc(sizeof(int) * N);
  v1.alloc(sizeof(int) * N);
  double scale = std::ldexp(1.0, Dk) / K;  // a power of two
  int bs = 256;
  hipLaunchKernelGGL(k_morton, dim3(unsigned((N + bs - 1) / bs)), dim3(bs), 0, 0, dpts.as<double>(), N,
                     K / 2.0, scale, Dk, k0.as<unsigned long long>(), v0.as<int>());
  DFMM_HIP(hipGetLastError());
  sort_pairs_u64(k0.as<unsigned long long>(), k1.as<unsigned long long>(), v0.as<int>(), v1.as<int>(), N,
                 3 * Dk);
  std::vector<int> idx(N);
  DFMM_HIP(hipMemcpy(idx.data(), v1.p, sizeof(int) * N, hipMemcpyDeviceToHost));
  T.perm.assign(idx.begin(), idx.end());
  T.pts.resize(3 * size_t(N));
  for (int64_t s = 0; s < N; ++s)
    for (int a = 0; a < 3; ++a) T.pts[3 * s + a] = points[3 * int64_t(idx[s]) + a];

  // box tables per level, from the sorted keys (lists.hip)
  build_levels_device(k1.as<unsigned long long>(), N, Dk, T, DT);

  // sorted points on the device, split into float hi + lo parts
  std::vector<float> hi(4 * size_t(N), 0.0f), lo(4 * size_t(N), 0.0f);
  for (int64_t s = 0; s < N; ++s)
    for (int a = 0; a < 3; ++a) {
      double x = T.pts[3 * s + a];
      float h = float(x);
      hi[4 * s + a] = h;
      lo[4 * s + a] = float(x - double(h));
    }
  P.pthi.upload(hi);
  P.ptlo.upload(lo);
  std::vector<int32_t> perm32(idx.begin(), idx.end());
  P.perm_d.upload(perm32);
  std::vector<int32_t> iperm32(size_t(N), 0);
  for (int64_t s = 0; s < N; ++s) iperm32[size_t(perm32[size_t(s)])] = int32_t(s);
  P.iperm_d.upload(iperm32);
  const auto& LL = T.lv[D];
  std::vector<int32_t> ls(LL.start.begin(), LL.start.end());
  ls.push_back(int32_t(N));
  P.leaf_start.upload(ls);
  std::vector<float> lc(4 * LL.key.size(), 0.0f);
  int mx = 0;
  for (size_t b = 0; b < LL.key.size(); ++b) {
    lc[4 * b + 0] = float((double(LL.cx[b]) + 0.5) * 0.5 - K / 2.0);
    lc[4 * b + 1] = float((double(LL.cy[b]) + 0.5) * 0.5 - K / 2.0);
    lc[4 * b + 2] = float((double(LL.cz[b]) + 0.5) * 0.5 - K / 2.0);
    mx = std::max<int>(mx, int(LL.end[b] - LL.start[b]));
  }
  P.max_leaf_pts = mx;
  P.leaf_center.upload(lc);
  std::vector<int32_t> lof(static_cast<size_t>(N));
  for (size_t b = 0; b < LL.key.size(); ++b)
    for (int64_t s = LL.start[b]; s < LL.end[b]; ++s) lof[size_t(s)] = int32_t(b);
  P.leaf_of.upload(lof);

}

}  // namespace dfmm
