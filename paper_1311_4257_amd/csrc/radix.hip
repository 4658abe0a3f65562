// Device sort and scans of the tree and list construction.
//
// sort_pairs_u64 is a stable LSD radix sort of (64-bit key, int value) pairs
// over the key bits [0, end_bit), 8 bits per pass.  A pass is three launches:
// per-tile digit counts, an exclusive scan of the counts in digit-major order
// (so every digit's slots run over the tiles in order), and a scatter in which
// each tile ranks its elements in index order: iteration by iteration, wave by
// wave, lane by lane, with the lanes of a wave that share a digit found by
// eight ballots.  Equal keys therefore keep their input order.
//
// scan_incl / scan_excl are int32 prefix sums: each 1,024-element tile is scanned
// in a workgroup, the tile totals are scanned the same way (recursively) and
// added back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "internal.hpp"

namespace dfmm {

namespace {

constexpr int kSortBS = 256;                    // threads per workgroup (4 waves)
constexpr int kSortItems = 8;                   // elements per thread and pass
constexpr int kSortTile = kSortBS * kSortItems;  // elements per workgroup
constexpr int kDigits = 256;

__global__ void __launch_bounds__(kSortBS) k_digit_count(const unsigned long long* __restrict__ key, int64_t n,
                                                          int shift, int ntiles, int* __restrict__ cnt) {
  __shared__ int c[kDigits];
  const int tid = int(threadIdx.x);
  c[tid] = 0;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kSortTile;
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t e = base + int64_t(it) * kSortBS + tid;
    if (e < n) atomicAdd(&c[int((key[e] >> shift) & 0xFF)], 1);
  }
  __syncthreads();
  cnt[int64_t(tid) * ntiles + blockIdx.x] = c[tid];  // digit-major
}

template <bool VALS>
__global__ void __launch_bounds__(kSortBS) k_digit_scatter(const unsigned long long* __restrict__ kin,
                                                            const int* __restrict__ vin, int64_t n, int shift,
                                                            int ntiles, const int* __restrict__ off,
                                                            unsigned long long* __restrict__ kout,
                                                            int* __restrict__ vout) {
  __shared__ int run[kDigits];       // next output slot of each digit in this tile
  __shared__ int wcnt[4][kDigits];   // this iteration's count of each digit per wave
  const int tid = int(threadIdx.x);
  const int lane = tid & 63, wave = tid >> 6;
  run[tid] = off[int64_t(tid) * ntiles + blockIdx.x];
  const unsigned long long below = (1ull << lane) - 1ull;
  const int64_t base = int64_t(blockIdx.x) * kSortTile;
  for (int it = 0; it < kSortItems; ++it) {
    for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const int64_t e = base + int64_t(it) * kSortBS + tid;
    const bool ok = e < n;
    unsigned long long k = 0;
    int v = 0, d = 0;
    if (ok) {
      k = kin[e];
      if (VALS) v = vin[e];
      d = int((k >> shift) & 0xFF);
    }
    // lanes of this wave holding an element with the same digit
    unsigned long long same = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const unsigned long long m = __ballot(ok && ((d >> b) & 1));
      same &= ((d >> b) & 1) ? m : ~m;
    }
    const int before = __popcll(same & below);
    if (ok && before == 0) wcnt[wave][d] = __popcll(same);  // the digit's first lane
    __syncthreads();
    if (ok) {
      int r = run[d] + before;
      for (int w = 0; w < wave; ++w) r += wcnt[w][d];
      kout[r] = k;
      if (VALS) vout[r] = v;
    }
    __syncthreads();
    run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
    __syncthreads();
  }
}

constexpr int kScanBS = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBS * kScanItems;

// Tile-local prefix sums (inclusive or exclusive) and each tile's total.
__global__ void __launch_bounds__(kScanBS) k_scan_tile(const int* __restrict__ in, int* __restrict__ out,
                                                        int64_t n, bool inclusive, int* __restrict__ total) {
  __shared__ int wsum[kScanBS / 64];
  const int tid = int(threadIdx.x), lane = tid & 63, wave = tid >> 6;
  const int64_t e0 = int64_t(blockIdx.x) * kScanTile + int64_t(tid) * kScanItems;
  int x[kScanItems];
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    x[i] = e0 + i < n ? in[e0 + i] : 0;
    s += x[i];
  }
  // exclusive prefix of the thread sums over the workgroup
  int incl = s;
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int pre = incl - s;
  for (int w = 0; w < wave; ++w) pre += wsum[w];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (inclusive) pre += x[i];
    if (e0 + i < n) out[e0 + i] = pre;
    if (!inclusive) pre += x[i];
  }
  if (tid == kScanBS - 1) total[blockIdx.x] = pre;
}

__global__ void k_scan_add(int* __restrict__ out, int64_t n, const int* __restrict__ tile_off) {
  const int64_t e = int64_t(blockIdx.x) * kScanTile + threadIdx.x;
  const int add = tile_off[blockIdx.x];
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t j = e + int64_t(i) * kScanBS;
    if (j < n) out[j] += add;
  }
}

void scan(const int* in, int* out, int64_t n, bool inclusive) {
  if (n <= 0) return;
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if (ntiles > INT32_MAX) throw Error{DFMM_EUNSUPPORTED, "scan too long"};
  DevBuf total, toff;
  total.alloc(sizeof(int) * size_t(ntiles));
  hipLaunchKernelGGL(k_scan_tile, dim3(unsigned(ntiles)), dim3(kScanBS), 0, 0, in, out, n, inclusive,
                     total.as<int>());
  DFMM_HIP(hipGetLastError());
  if (ntiles > 1) {
    toff.alloc(sizeof(int) * size_t(ntiles));
    scan(total.as<int>(), toff.as<int>(), ntiles, false);
    hipLaunchKernelGGL(k_scan_add, dim3(unsigned(ntiles)), dim3(kScanBS), 0, 0, out, n, toff.as<int>());
    DFMM_HIP(hipGetLastError());
  }
}

void sort_u64(const unsigned long long* kin, unsigned long long* kout, const int* vin, int* vout, int64_t n,
              int end_bit) {
  if (n <= 0) return;
  if (n > INT32_MAX) throw Error{DFMM_EUNSUPPORTED, "sort too long"};
  const int npass = std::max(1, (std::min(end_bit, 64) + 7) / 8);
  const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  const bool vals = vin != nullptr;
  DevBuf cnt, off, ka, kb, va, vb;
  cnt.alloc(sizeof(int) * size_t(kDigits * ntiles));
  off.alloc(sizeof(int) * size_t(kDigits * ntiles));
  if (npass > 1) {
    ka.alloc(sizeof(unsigned long long) * size_t(n));
    if (vals) va.alloc(sizeof(int) * size_t(n));
  }
  if (npass > 2) {
    kb.alloc(sizeof(unsigned long long) * size_t(n));
    if (vals) vb.alloc(sizeof(int) * size_t(n));
  }
  const unsigned long long* ks = kin;
  const int* vs = vin;
  for (int p = 0; p < npass; ++p) {
    const bool last = p == npass - 1;
    unsigned long long* kd = last ? kout : ((p & 1) ? kb.as<unsigned long long>() : ka.as<unsigned long long>());
    int* vd = !vals ? nullptr : last ? vout : ((p & 1) ? vb.as<int>() : va.as<int>());
    hipLaunchKernelGGL(k_digit_count, dim3(unsigned(ntiles)), dim3(kSortBS), 0, 0, ks, n, 8 * p, int(ntiles),
                       cnt.as<int>());
    DFMM_HIP(hipGetLastError());
    scan(cnt.as<int>(), off.as<int>(), kDigits * ntiles, false);
    if (vals)
      hipLaunchKernelGGL(k_digit_scatter<true>, dim3(unsigned(ntiles)), dim3(kSortBS), 0, 0, ks, vs, n, 8 * p,
                         int(ntiles), off.as<int>(), kd, vd);
    else
      hipLaunchKernelGGL(k_digit_scatter<false>, dim3(unsigned(ntiles)), dim3(kSortBS), 0, 0, ks, vs, n, 8 * p,
                         int(ntiles), off.as<int>(), kd, vd);
    DFMM_HIP(hipGetLastError());
    ks = kd;
    vs = vd;
  }
}

}  // namespace

void scan_incl(const int* in, int* out, int64_t n) { scan(in, out, n, true); }
void scan_excl(const int* in, int* out, int64_t n) { scan(in, out, n, false); }

void sort_pairs_u64(const unsigned long long* kin, unsigned long long* kout, const int* vin, int* vout, int64_t n,
                    int end_bit) {
  sort_u64(kin, kout, vin, vout, n, end_bit);
}

void sort_keys_u64(const unsigned long long* kin, unsigned long long* kout, int64_t n, int end_bit) {
  sort_u64(kin, kout, nullptr, nullptr, n, end_bit);
}

}  // namespace dfmm
