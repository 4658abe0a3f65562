// The evaluation pass (Algorithm 1, Section 2.3) as HIP kernels for gfx950,
// plus the near-field sum between adjacent leaves that Eq. 1 needs.
//
// Device layout (per plan): points sorted in Morton order, each coordinate as
// a float hi part and a float lo part (x = hi + lo to ~2^-48 relative), so that
// differences of nearby points keep full float precision.  Vectors are
// complex64 laid out [slot][row][rhs]: F (outgoing equivalent charges) per
// needed (box, wedge) slot of an HF level or per leaf, U (incoming check
// potentials) likewise.  Every kernel works in float32 except the leaf
// evaluation, which accumulates each target's sum in float64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <type_traits>
#include <utility>

#include "internal.hpp"

namespace dfmm {

namespace {


__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ void cfma(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x));
  acc.y = fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y));
}

// G for a separation given in float64: the distance and the phase reduction
// r - rint(r) are done in float64 (the phase error stays ~2e-7 rad however far
// apart the points are), sin/cos of the reduced phase and 1/r in float32.
__device__ __forceinline__ double2 green_d(double dx, double dy, double dz) {
  const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
  if (r2 == 0.0) return make_double2(0.0, 0.0);
  const double r = sqrt(r2);
  float s, c;
  sincospif(2.0f * float(r - rint(r)), &s, &c);  // the phase reduced in float64 first
  const double ri = 1.0 / r;
  return make_double2(double(c) * ri, double(s) * ri);
}

// G for a float32 separation: r from float32 squares and the hardware
// reciprocal square root, phase t = r - rint(r) in turns, and the hardware
// sine and cosine, which take turns (over |t| <= 1/2 they are within 1.3e-7
// of sin and cos of 2 pi t, rms 3.5e-8).  Phase error ~2e-7 r rad: for the
// eps >= 1e-5 plans.  A coincident pair (r = 0) gives 0 without a branch (1/r
// taken as 0, so r and the phase are 0 too).
__device__ __forceinline__ float2 green_f(float dx, float dy, float dz) {
  const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  const float ri = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
  const float r = r2 * ri;
  const float t = r - rintf(r);
  return make_float2(__builtin_amdgcn_cosf(t) * ri, __builtin_amdgcn_sinf(t) * ri);
}

inline unsigned nblocks(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

// ---- permutation into Morton order ------------------------------------------
// The densities of a batch of requests: batch column k belongs to the last
// request r with k0[r] <= k (a select chain over uniform kernel arguments).
__device__ __forceinline__ int req_of(const ReqTable& R, int k) {
  int r = 0;
  for (int q = 1; q < R.n; ++q) r = k >= R.k0[q] ? q : r;
  return r;
}

__global__ void k_permute_in(const ReqTable R, float2* __restrict__ fs, const int* __restrict__ perm, int64_t N,
                             int nrhs) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N * nrhs) return;
  int64_t s = i / nrhs;
  int k = int(i % nrhs);
  const int r = req_of(R, k);
  fs[i] = R.f[r][int64_t(k - R.k0[r]) * N + perm[s]];
}

// Many right-hand sides: the permutation through a tile in LDS of PT_P points,
// taken in the caller's order, by PT_C columns.  The caller's side is read (or
// written) as runs of PT_P consecutive points per column, the tree-order side
// ([point][rhs]) as runs of the tile's columns per point; iperm maps a caller
// index to its tree position.
constexpr int PT_P = 64, PT_C = 32, PT_BS = 256;
__global__ void __launch_bounds__(PT_BS) k_permute_in_tile(const ReqTable R, float2* __restrict__ fs,
                                                           const int* __restrict__ iperm, int64_t N, int nrhs) {
  __shared__ float2 t[PT_C][PT_P + 1];
  const int64_t i0 = int64_t(blockIdx.x) * PT_P;
  const int c0 = int(blockIdx.y) * PT_C;
  const int nc = min(PT_C, nrhs - c0);
  const int np = int(min(int64_t(PT_P), N - i0));
  const int p = int(threadIdx.x) % PT_P;
  if (p < np)
    for (int c = int(threadIdx.x) / PT_P; c < nc; c += PT_BS / PT_P) {
      const int k = c0 + c;
      const int r = req_of(R, k);
      t[c][p] = R.f[r][int64_t(k - R.k0[r]) * N + i0 + p];
    }
  __syncthreads();
  for (int e = threadIdx.x; e < np * PT_C; e += PT_BS) {
    const int q = e / PT_C, c = e % PT_C;
    if (c < nc) fs[int64_t(iperm[i0 + q]) * nrhs + c0 + c] = t[c][q];
  }
}

// The inverse: potentials in tree order ut ([point][rhs]) to the caller's
// outputs (each request's [rhs][N] in the caller's point order).
__global__ void __launch_bounds__(PT_BS) k_permute_out_tile(const ReqTable R, const float2* __restrict__ ut,
                                                            const int* __restrict__ iperm, int64_t N, int nrhs) {
  __shared__ float2 t[PT_C][PT_P + 1];
  const int64_t i0 = int64_t(blockIdx.x) * PT_P;
  const int c0 = int(blockIdx.y) * PT_C;
  const int nc = min(PT_C, nrhs - c0);
  const int np = int(min(int64_t(PT_P), N - i0));
  for (int e = threadIdx.x; e < np * PT_C; e += PT_BS) {
    const int q = e / PT_C, c = e % PT_C;
    if (c < nc) t[c][q] = ut[int64_t(iperm[i0 + q]) * nrhs + c0 + c];
  }
  __syncthreads();
  const int p = int(threadIdx.x) % PT_P;
  if (p < np)
    for (int c = int(threadIdx.x) / PT_P; c < nc; c += PT_BS / PT_P) {
      const int k = c0 + c;
      const int r = req_of(R, k);
      R.u[r][int64_t(k - R.k0[r]) * N + i0 + p] = t[c][p];
    }
}

// ---- per-point leaf weights (plan time, float64) -----------------------------------
// For sorted point j in leaf B (centre c):
//   V[j][p] = G(c + a_p, x_j)                       (S2M: check potential weights)
//   W[j][q] = sum_p G(x_j, c + a_p) D_LF[q][p]      (L2T: incoming check potentials
//                                                    at b_q -> potential at x_j)
// W is formed in float64 because the incoming equivalent charges D^T U are
// large and cancel; the product is a well-scaled interpolation weight that
// float32 holds without loss.  One block per leaf, points in sequence.
constexpr int LW_BS = 64;
__device__ __forceinline__ void put_w(float2* p, double re, double im) { *p = make_float2(float(re), float(im)); }
__device__ __forceinline__ void put_w(double2* p, double re, double im) { *p = make_double2(re, im); }
template <class WT>  // float2 (float32 plans) or double2 (float64 plans)
__global__ void __launch_bounds__(LW_BS) k_leaf_weights(const double* __restrict__ pts, const int* __restrict__ lstart,
                                                         const float4* __restrict__ lcen,
                                                         const double4* __restrict__ a_all,
                                                         const double2* __restrict__ DT_all,
                                                         const int* __restrict__ ra, const int* __restrict__ sk_of,
                                                         int R, WT* __restrict__ V, WT* __restrict__ W) {
  extern __shared__ double2 gs[];  // Ra
  const int b = blockIdx.x;
  const float4 c = lcen[b];
  // this leaf's skeleton (one per LF width): check points at R offsets, D^T at R R
  const int sk = sk_of[b];
  const int Ra = ra[sk];
  const double4* __restrict__ a_lf = a_all + int64_t(sk) * R;
  const double2* __restrict__ DT = DT_all + int64_t(sk) * R * R;
  for (int j = lstart[b]; j < lstart[b + 1]; ++j) {
    const double x = pts[3 * int64_t(j)] - double(c.x);
    const double y = pts[3 * int64_t(j) + 1] - double(c.y);
    const double z = pts[3 * int64_t(j) + 2] - double(c.z);
    __syncthreads();
    for (int p = threadIdx.x; p < R; p += LW_BS) {
      double2 gv = make_double2(0.0, 0.0);
      if (p < Ra) {
        const double4 ap = a_lf[p];
        const double dx = x - ap.x, dy = y - ap.y, dz = z - ap.z;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        double sn, cs;
        sincospi(2.0 * r, &sn, &cs);
        gv = make_double2(cs / r, sn / r);
        gs[p] = gv;
      }
      put_w(&V[int64_t(j) * R + p], gv.x, gv.y);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < R; q += LW_BS) {
      double wr = 0.0, wi = 0.0;
      for (int p = 0; p < Ra; ++p) {
        const double2 gv = gs[p], d = DT[int64_t(p) * R + q];
        wr += gv.x * d.x - gv.y * d.y;
        wi += gv.x * d.y + gv.y * d.x;
      }
      put_w(&W[int64_t(j) * R + q], wr, wi);
    }
  }
}

// ---- leaf S2M: outgoing check potentials chk[p] = sum_j V[j][p] f_j ----------------
// One block per leaf, threads over check points (the weights of consecutive
// check points are contiguous).  D_LF is folded into the operators that read
// these potentials.  With few right-hand sides the loop over the leaf's
// sources is bound by load latency, so the weights of SU sources are loaded
// before any of them is used (the products are still added in source order).
constexpr int S2M_BS = 128;
template <int RC>  // right-hand sides per pass
__global__ void __launch_bounds__(S2M_BS) k_s2m(const int* __restrict__ lstart, const float2* __restrict__ V,
                                                 const float2* __restrict__ fs, int R, int nrhs,
                                                 const int* __restrict__ gid, float2* __restrict__ clf) {
  constexpr int SU = RC <= 8 ? 4 : 1;  // sources per loaded batch
  const int b = blockIdx.x;
  const int bo = gid ? gid[b] : b;  // the leaf's LF vector (adaptive trees)
  const int s0 = lstart[b], s1 = lstart[b + 1];
  for (int k0 = 0; k0 < nrhs; k0 += RC) {
    const int nk = min(RC, nrhs - k0);
    for (int p = threadIdx.x; p < R; p += S2M_BS) {
      float2 acc[RC];
#pragma unroll
      for (int k = 0; k < RC; ++k) acc[k] = make_float2(0.f, 0.f);
      int j = s0;
      for (; j + SU <= s1; j += SU) {
        float2 v[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) v[u] = V[int64_t(j + u) * R + p];
#pragma unroll
        for (int u = 0; u < SU; ++u)
#pragma unroll
          for (int k = 0; k < RC; ++k)
            if (k < nk) cfma(acc[k], v[u], fs[int64_t(j + u) * nrhs + k0 + k]);
      }
      for (; j < s1; ++j) {
        const float2 v = V[int64_t(j) * R + p];
#pragma unroll
        for (int k = 0; k < RC; ++k)
          if (k < nk) cfma(acc[k], v, fs[int64_t(j) * nrhs + k0 + k]);
      }
#pragma unroll
      for (int k = 0; k < RC; ++k)
        if (k < nk) clf[(int64_t(bo) * nrhs + k0 + k) * R + p] = acc[k];
    }
  }
}

typedef float v4f __attribute__((ext_vector_type(4)));  // an MFMA accumulator tile

// S2M for many right-hand sides as a complex GEMM on MFMA: per leaf, the
// outgoing check potentials are V^T (R x points) times the leaf's densities
// (points x rhs).  A workgroup takes (leaf, 16 NCT right-hand sides); the
// leaf's densities of those columns are staged in LDS (zeros past the last
// point, an even count), and the waves take the 8-row tiles of R in turn.
// The fragments are those of the near field and of L2T: the lane's A entry is
// component (row parity) xor (k part) of V (negated on even rows' Im
// entries), its B entry component (k part) of a density; float32 sums over
// the leaf's points, as in the VALU form.
constexpr int S2M_MT_NW = 4;  // waves per workgroup
template <int NCT>
__global__ void __launch_bounds__(64 * S2M_MT_NW) k_s2m_mfma(const int* __restrict__ lstart,
                                                             const float2* __restrict__ V,
                                                             const float2* __restrict__ fs, int R, int nrhs,
                                                             const int* __restrict__ gid, float2* __restrict__ clf) {
  constexpr int NCOL = 16 * NCT;
  extern __shared__ float2 fsh[];  // [point (even count)][NCOL]
  const int b = blockIdx.x;
  const int bo = gid ? gid[b] : b;  // the leaf's LF vector (adaptive trees)
  const int c0 = int(blockIdx.y) * NCOL;
  const int s0 = lstart[b], s1 = lstart[b + 1];
  const int np = s1 - s0, np2 = (np + 1) & ~1;
  const int nc = min(NCOL, nrhs - c0);
  for (int e = threadIdx.x; e < np2 * NCOL; e += 64 * S2M_MT_NW) {
    const int j = e / NCOL, c = e - j * NCOL;
    fsh[e] = (j < np && c < nc) ? fs[int64_t(s0 + j) * nrhs + c0 + c] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  if (np == 0) return;  // uniform
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int jr = lane & 15, kr = lane >> 4;  // A row / B column, k index of this lane
  const int kp = kr & 1;                      // Re / Im part of k
  const bool rodd = (jr & 1) != 0;
  const int comp = (rodd ? 1 : 0) ^ kp;
  const unsigned neg = (!rodd && kp) ? 0x80000000u : 0u;
  const float* fb = reinterpret_cast<const float*>(fsh + (kr >> 1) * NCOL + jr) + kp;
  for (int m = w; m < R / 8; m += S2M_MT_NW) {
    const int p = m * 8 + (jr >> 1);  // this lane's row (complex)
    v4f acc[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
    // MFMA step q covers points 2q, 2q + 1 of the leaf (past the last point the
    // weights of the last one, against zero densities)
#pragma unroll 4
    for (int q = 0; q < np2 / 2; ++q) {
      const int j = min(2 * q + (kr >> 1), np - 1);
      const float av = __uint_as_float(
          __float_as_uint(reinterpret_cast<const float*>(V + int64_t(s0 + j) * R + p)[comp]) ^ neg);
#pragma unroll
      for (int c = 0; c < NCT; ++c)
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, fb[2 * (2 * q * NCOL + c * 16)], acc[c], 0, 0, 0);
    }
    // lane holds rows 4 kr .. 4 kr + 3 = (Re, Im) of rows 2 kr, 2 kr + 1 of the tile, column jr
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int col = c * 16 + jr;
      if (col >= nc) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h)
        clf[(int64_t(bo) * nrhs + c0 + col) * R + m * 8 + 2 * kr + h] = make_float2(acc[c][2 * h], acc[c][2 * h + 1]);
    }
  }
}

// ---- grouped gather GEMM on MFMA: Y[vdst] = A[op] X[vsrc] ------------------------
// The complex product y = A x is done as a real product on interleaved data:
// real row 2q (re) of A is (Re A[q][p], -Im A[q][p]) per column pair (2p, 2p+1)
// and row 2q+1 (im) is (Im, Re); x and y stay in their natural interleaved
// layout.  One workgroup (NW = 2 or 4 waves) handles NT*16 vector columns of
// one group (one operator).  The 16-row M-tiles m of the group go to the waves
// as m = wave + NW (slice + slices t), t = 0, 1, ... (slice = blockIdx.y), and each
// wave walks its tiles one after the other, so a group's own M_g sets the work
// and no MFMA runs on an empty tile.  The K dimension of a tile is split into
// four quarters, one per group of 16 lanes (MFMA k index): a lane reads four
// consecutive k values of its quarter with one 16-byte load from LDS (B) and
// from the fragment-ordered operator (A).  The column block sits in LDS,
// [column][k] with a row stride S = 4 (mod 32) floats.  The (tile, k-step)
// sequence of a wave is one flat loop; the operator loads of the next few step
// pairs are in flight in a register ring, and a load is issued for every step
// pair (past the end it repeats the last address) so that each wait is for the
// oldest load only.

__host__ __device__ inline int gg_stride(int K) {
  int s = 2 * K;
  return s + ((4 - (s % 32)) + 32) % 32;
}

// operator loads in flight per lane (each covers two k-steps)
template <int NT>
struct GgDepth {
  static constexpr int value = NT == 1 ? 4 : (NT == 2 ? 4 : 3);
};

// the float4 of the neighbouring lane (lane ^ 1), by DPP quad permutation [1, 0, 3, 2]
__device__ __forceinline__ float4 swap_pair(const float4 v) {
  auto sw = [](float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));
  };
  return make_float4(sw(v.x), sw(v.y), sw(v.z), sw(v.w));
}

// ---- split 16-bit products (FP16X3 / BF16X3 plans) -----------------------------------
// A 32-bit word holds two 16-bit values, the first in the low half.  x = hi + lo
// with hi the 16-bit rounding of x and lo that of the (exact) remainder.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
constexpr int PREC_F16 = 1, PREC_BF16 = 2;

template <int PREC>
__device__ __forceinline__ void split_pair(float a, float b, unsigned& hi, unsigned& lo) {
  if constexpr (PREC == PREC_F16) {
    const _Float16 ha = _Float16(a), hb = _Float16(b);
    const _Float16 la = _Float16(a - float(ha)), lb = _Float16(b - float(hb));
    hi = unsigned(__builtin_bit_cast(unsigned short, ha)) | (unsigned(__builtin_bit_cast(unsigned short, hb)) << 16);
    lo = unsigned(__builtin_bit_cast(unsigned short, la)) | (unsigned(__builtin_bit_cast(unsigned short, lb)) << 16);
  } else {
    auto rne = [](float x) {  // bfloat16 bits, round to nearest even
      const unsigned u = __float_as_uint(x);
      return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
    };
    const unsigned ha = rne(a), hb = rne(b);
    hi = ha | (hb << 16);
    lo = rne(a - __uint_as_float(ha << 16)) | (rne(b - __uint_as_float(hb << 16)) << 16);
  }
}

// (x, y) -> (y, x) of a word's two halves
__device__ __forceinline__ unsigned rot16(unsigned x) { return __builtin_amdgcn_alignbit(x, x, 16); }

template <int PREC>
__device__ __forceinline__ v4f mfma16(v4u a, v4u b, v4f c) {
  if constexpr (PREC == PREC_F16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a), __builtin_bit_cast(v8h, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0,
                                                   0);
}

// ALDS: stage the workgroup's operator tiles in LDS first.  ACC64: every two
// k-steps (32 real products per output) the float32 MFMA sums are added into
// float64 partial sums, so the rounding of long float32 dot products (which
// grows with their length) stays at that of 32 terms.
template <int NT, bool ALDS, bool ACC64, int NW, int PREC>
__device__ __forceinline__ void ggemm_tile(const float4* __restrict__ A, const int64_t* __restrict__ aoff,
                                           const int* __restrict__ aexp,
                                           const int* __restrict__ gmk, int M, int K, int split,
                                           const int* __restrict__ gops, const int* __restrict__ gv0,
                                           const int* __restrict__ vsrc, const int* __restrict__ vdst,
                                           const int* __restrict__ chunk_grp, const int* __restrict__ chunk_c0,
                                           int nrhs, const float2* __restrict__ X, float2* __restrict__ Y,
                                           int chunk, int slice, int nslices) {
  static_assert(!(ACC64 && PREC), "split 16-bit products are for fast plans");
  extern __shared__ float4 xs[];
  constexpr int NC = NT * 16;
  constexpr int PD = GgDepth<NT>::value;
  constexpr int BS = 64 * NW;
  // 16-bit plans: operators packed with K_g padded to 16 (two k-steps per MFMA)
  auto kp = [](int k) { return PREC ? (k + 15) / 16 * 16 : k; };
  const int S4 = gg_stride(split * kp(K)) / 4;  // float4 per LDS column (split K >= every K_g)
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = lane & 15, kr = lane >> 4;
  const bool odd = (j & 1) != 0;
  const int g = chunk_grp[chunk];
  const int Mg = gmk[2 * g], Kr = gmk[2 * g + 1];  // this group's operator size
  const int Kg = kp(Kr);                 // packed K (Kr + zero columns in 16-bit plans)
  const int Q4 = Kg / 8;                 // k-steps per tile (K_g / 2 real k per quarter, 4 per step)
  const int nM = Mg / 8, nMall = M / 8;  // 16-row real M-tiles with data / in the vector stride
  const int m0 = wave + NW * slice, mstep = NW * nslices;
  const int mcnt = m0 < nM ? (nM - m0 + mstep - 1) / mstep : 0;
  const int64_t c0 = chunk_c0[chunk];
  const int vbeg = gv0[g];
  const int64_t ncol = int64_t(gv0[g + 1] - vbeg) * nrhs;
  const int nc = int(min<int64_t>(NC, ncol - c0));

  // stage the source vectors: column c -> X[(src * nrhs + k) * K], its first K_g
  // complex entries.  The column sources go through a small LDS table (one
  // division per column); each thread then walks its elements (q4 fastest, so
  // a wave reads long contiguous runs) with incremental indices, issuing a
  // batch of loads before storing them.
  const int per_col = Kg / 2;  // float4 per column
  const int pcs = per_col / split;  // float4 per source vector (split = 2: each read twice)
  const int preal = Kr / 2;         // float4 of the column that the vector holds (rest: zero padding)
  const float4* Aop = A + aoff[gops[g]];
  const int tile4 = Q4 * 32;  // float4 per M-tile in the fragment order
  float4* as = xs + NC * S4;  // ALDS: the tiles of this slice, [t][wave][tile4]

  // operator fragment stream of this wave: flat step i = (t, s) reads tile base
  // + s * 32 + this lane's offset.  The two lanes of a row pair (j, j ^ 1) need
  // the same 16 bytes, so one load serves two steps: the even lane fetches step
  // i and the odd lane step i + 1, and a lane swap gives each both.  From global
  // memory the first loads are issued before the column staging, so their
  // latency overlaps it.
  const int total = mcnt * Q4;  // flat (tile, k-step) sequence of this wave
  const int lofs = (j >> 1) * 4 + kr;
  // Offsets are 32-bit (one operator holds far fewer than 2^31 float4) and
  // strictly increase along the sequence (every advance adds at least 32), so
  // clamping to the last step's offset repeats it past the end.  The loop
  // bookkeeping is scalar work that competes with the MFMAs for issue slots,
  // hence no branches and no 64-bit arithmetic here.
  const int tbase0 = ALDS ? wave * tile4 : m0 * tile4;
  const int tjump = ALDS ? NW * tile4 : mstep * tile4;
  const float4* abase = (ALDS ? static_cast<const float4*>(as) : Aop) + lofs;
  const int last = tbase0 + (mcnt - 1) * tjump + (Q4 - 1) * 32;
  const int pwrap = tjump - (Q4 - 1) * 32;  // from a tile's last k-step to the next tile's first
  int ps = 0;                 // k-step of the next prefetch within its tile
  int pofs = tbase0;          // its offset
  auto advance = [&]() {
    const bool wrap = ++ps == Q4;
    ps = wrap ? 0 : ps;
    pofs += wrap ? pwrap : 32;
  };
  auto fetch = [&]() -> float4 {  // the next two steps: the even lane's, then the odd lane's
    const int o0 = min(pofs, last);
    advance();
    const int o1 = min(pofs, last);
    advance();
    return abase[odd ? o1 : o0];
  };
  float4 ring[PD];
  if (!ALDS && total > 0) {
#pragma unroll
    for (int p = 0; p < PD; ++p) ring[p] = fetch();
  }
  __shared__ const float4* colsrc[NC];
  if (threadIdx.x < NC) {
    const int col = threadIdx.x;
    const float4* p = nullptr;
    if (col < nc) {
      const int64_t cc = c0 + col;
      const int src = vsrc[vbeg + int(cc / nrhs)];
      if (src >= 0) p = reinterpret_cast<const float4*>(X + (int64_t(src) * nrhs + int(cc % nrhs)) * K);
    }
    colsrc[col] = p;
  }
  __syncthreads();
  {
    constexpr int UB = 4;  // loads in flight per thread
    const int nel = NC * per_col;
    const int dcol = BS / per_col, dq = BS % per_col;
    int col = int(threadIdx.x) / per_col, q4 = int(threadIdx.x) % per_col;
    for (int base = int(threadIdx.x); base < nel; base += UB * BS) {
      float4 v[UB];
      int dst[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        dst[u] = -1;
        if (base + u * BS < nel) {
          const float4* p = colsrc[col];
          if (p && (!PREC || q4 < preal)) v[u] = p[q4 < pcs ? q4 : q4 - pcs];
          dst[u] = col * S4 + q4;
        }
        col += dcol;
        q4 += dq;
        if (q4 >= per_col) {
          q4 -= per_col;
          ++col;
        }
      }
#pragma unroll
      for (int u = 0; u < UB; ++u)
        if (dst[u] >= 0) xs[dst[u]] = v[u];
    }
  }
  __shared__ int cexp[NC];  // 16-bit plans: power-of-two scale exponent of each column
  if constexpr (PREC != 0) {
    __syncthreads();  // the float32 columns are staged
    if (threadIdx.x < NC) {
      int e = 0;
      if constexpr (PREC == PREC_F16) {  // largest column entry below 2^14 after scaling
        float mx = 0.f;
        const float4* c = xs + threadIdx.x * S4;
        for (int q = 0; q < per_col; ++q) {
          const float4 v = c[q];
          mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
        if (mx > 0.f) {
          int E;
          (void)frexpf(mx, &E);
          e = 14 - E;
        }
      }
      cexp[threadIdx.x] = e;
    }
    __syncthreads();
    for (int idx = int(threadIdx.x); idx < NC * per_col; idx += BS) {
      const int col = idx / per_col, q = idx - col * per_col;
      float4 v = xs[col * S4 + q];
      if constexpr (PREC == PREC_F16) {
        const int e = cexp[col];
        v = make_float4(ldexpf(v.x, e), ldexpf(v.y, e), ldexpf(v.z, e), ldexpf(v.w, e));
      }
      unsigned h0, l0, h1, l1;
      split_pair<PREC>(v.x, v.y, h0, l0);
      split_pair<PREC>(v.z, v.w, h1, l1);
      xs[col * S4 + q] = make_float4(__uint_as_float(h0), __uint_as_float(h1), __uint_as_float(l0), __uint_as_float(l1));
    }
  }
  if (ALDS) {
    const int tmax = nM > NW * slice ? (nM - NW * slice + mstep - 1) / mstep : 0;
    const int nel = 4 * tmax * tile4;
    const int dblk = BS / tile4, doff = BS % tile4;
    int blk = int(threadIdx.x) / tile4, off = int(threadIdx.x) % tile4;
    for (int idx = int(threadIdx.x); idx < nel; idx += BS) {
      const int m = (blk % NW) + NW * slice + mstep * (blk / NW);
      as[idx] = m < nM ? Aop[int64_t(m) * tile4 + off] : make_float4(0.f, 0.f, 0.f, 0.f);
      blk += dblk;
      off += doff;
      if (off >= tile4) {
        off -= tile4;
        ++blk;
      }
    }
  }
  __syncthreads();
  if (ALDS && total > 0) {
#pragma unroll
    for (int p = 0; p < PD; ++p) ring[p] = fetch();
  }

  // this lane's output columns
  float2* yp[NT];
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int col = n * 16 + j;
    yp[n] = nullptr;
    if (col < nc) {
      const int64_t cc = c0 + col;
      const int vv = vbeg + int(cc / nrhs);
      yp[n] = Y + (int64_t(vdst[vv]) * nrhs + int(cc % nrhs)) * M;
    }
  }

  if constexpr (PREC != 0) {
    if (total > 0) {
      // operator scale of the group and column scales: the sums are unscaled at the write
      const int ea = PREC == PREC_F16 ? aexp[gops[g]] : 0;
      float osc[NT];
#pragma unroll
      for (int n = 0; n < NT; ++n) osc[n] = ldexpf(1.0f, -(ea + cexp[n * 16 + j]));
      v4f acc[NT];
#pragma unroll
      for (int n = 0; n < NT; ++n) acc[n] = v4f{0.f, 0.f, 0.f, 0.f};
      const float4* bcol = xs + j * S4 + kr * Q4;
      float4 b0[NT], b1[NT];  // steps s, s + 1 of every column tile (hi, hi, lo, lo words)
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        b0[n] = bcol[n * 16 * S4];
        b1[n] = bcol[n * 16 * S4 + 1];
      }
      int s = 0, t = 0;
      constexpr unsigned SG = 0x80000000u;  // sign of a word's high half
      // one ring slot = two k-steps = one 16x16x32 MFMA per product term; the
      // even row of a complex row pair is (Re, -Im), the odd row (Im, Re)
      auto dstep = [&](const float4 vf, const float4 wf) {
        const unsigned vx = __float_as_uint(vf.x), vy = __float_as_uint(vf.y), vz = __float_as_uint(vf.z),
                       vw = __float_as_uint(vf.w), wx = __float_as_uint(wf.x), wy = __float_as_uint(wf.y),
                       wz = __float_as_uint(wf.z), ww = __float_as_uint(wf.w);
        const v4u ah = odd ? v4u{rot16(wx), rot16(wy), rot16(vx), rot16(vy)} : v4u{vx ^ SG, vy ^ SG, wx ^ SG, wy ^ SG};
        const v4u al = odd ? v4u{rot16(wz), rot16(ww), rot16(vz), rot16(vw)} : v4u{vz ^ SG, vw ^ SG, wz ^ SG, ww ^ SG};
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          const v4u bh = {__float_as_uint(b0[n].x), __float_as_uint(b0[n].y), __float_as_uint(b1[n].x),
                          __float_as_uint(b1[n].y)};
          const v4u bl = {__float_as_uint(b0[n].z), __float_as_uint(b0[n].w), __float_as_uint(b1[n].z),
                          __float_as_uint(b1[n].w)};
          acc[n] = mfma16<PREC>(ah, bh, acc[n]);
          acc[n] = mfma16<PREC>(ah, bl, acc[n]);
          acc[n] = mfma16<PREC>(al, bh, acc[n]);
        }
        s += 2;
        const int s2 = s == Q4 ? 0 : s;  // the next step pair (the column is the same for every M-tile)
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          b0[n] = bcol[n * 16 * S4 + s2];
          b1[n] = bcol[n * 16 * S4 + s2 + 1];
        }
        if (s == Q4) {  // tile done: lane holds real rows 4kr .. 4kr+3 = complex rows 2kr, 2kr+1
          const int m = m0 + mstep * t;
#pragma unroll
          for (int n = 0; n < NT; ++n) {
            const v4f a = acc[n];
            const float4 o = make_float4(a[0] * osc[n], a[1] * osc[n], a[2] * osc[n], a[3] * osc[n]);
            if (yp[n]) reinterpret_cast<float4*>(yp[n] + 8 * m + 2 * kr)[0] = o;
            acc[n] = v4f{0.f, 0.f, 0.f, 0.f};
          }
          s = 0;
          ++t;
        }
      };
      int i0 = 0;  // total is even: Q4 is even in 16-bit plans
      for (; i0 + 2 * PD <= total; i0 += 2 * PD) {
#pragma unroll
        for (int p = 0; p < PD; ++p) {
          const float4 v = ring[p], w = swap_pair(v);
          dstep(v, w);
          ring[p] = fetch();
        }
      }
#pragma unroll
      for (int p = 0; p < PD; ++p) {
        if (i0 + 2 * p >= total) break;
        const float4 v = ring[p], w = swap_pair(v);
        dstep(v, w);
      }
    }
  } else if (total > 0) {
    v4f acc[NT];  // consecutive MFMAs on one accumulator chain through its C operand
    double a64[ACC64 ? NT : 1][4];
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[n] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int n = 0; n < (ACC64 ? NT : 1); ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) a64[n][r] = 0.0;
    int s = 0, t = 0;
    // B fragments: a ring of two steps (slot p & 1 of the unrolled loop)
    const float4* bcol = xs + j * S4 + kr * Q4;
    const int s1 = Q4 > 1 ? 1 : 0;
    float4 bq[2][NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      bq[0][n] = bcol[n * 16 * S4];
      bq[1][n] = bcol[n * 16 * S4 + s1];
    }
    // the complex A fragments of a step pair as real rows (even row: Re, -Im;
    // odd row: Im, Re): v is this lane's load, w its neighbour's
    auto frag0 = [&](const float4 v, const float4 w, float (&av)[4]) {  // step i
      av[0] = odd ? w.y : v.x;
      av[1] = odd ? w.x : -v.y;
      av[2] = odd ? w.w : v.z;
      av[3] = odd ? w.z : -v.w;
    };
    auto frag1 = [&](const float4 v, const float4 w, float (&av)[4]) {  // step i + 1
      av[0] = odd ? v.y : w.x;
      av[1] = odd ? v.x : -w.y;
      av[2] = odd ? v.w : w.z;
      av[3] = odd ? v.z : -w.w;
    };
    int s2 = 2 % Q4;  // the k-step two ahead of s, within its tile
    auto step = [&](const float (&av)[4], float4 (&b)[NT]) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          const float bv = u == 0 ? b[n].x : (u == 1 ? b[n].y : (u == 2 ? b[n].z : b[n].w));
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], bv, acc[n], 0, 0, 0);
        }
#pragma unroll
      for (int n = 0; n < NT; ++n) b[n] = bcol[n * 16 * S4 + s2];
      s2 = s2 + 1 == Q4 ? 0 : s2 + 1;  // s advances by one step, cyclically within the tile
      if constexpr (ACC64) {
        if ((s & 1) || s + 1 == Q4) {
#pragma unroll
          for (int n = 0; n < NT; ++n) {
#pragma unroll
            for (int r = 0; r < 4; ++r) a64[n][r] += double(acc[n][r]);
            acc[n] = v4f{0.f, 0.f, 0.f, 0.f};
          }
        }
      }
      if (++s == Q4) {  // tile done: lane holds real rows 4kr .. 4kr+3 = complex rows 2kr, 2kr+1
        const int m = m0 + mstep * t;
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          float4 o;
          if constexpr (ACC64) {
            o = make_float4(float(a64[n][0]), float(a64[n][1]), float(a64[n][2]), float(a64[n][3]));
#pragma unroll
            for (int r = 0; r < 4; ++r) a64[n][r] = 0.0;
          } else {
            const v4f a = acc[n];
            o = make_float4(a[0], a[1], a[2], a[3]);
          }
          if (yp[n]) reinterpret_cast<float4*>(yp[n] + 8 * m + 2 * kr)[0] = o;
          acc[n] = v4f{0.f, 0.f, 0.f, 0.f};
        }
        s = 0;
        ++t;
      }
    };
    // each load's register is refilled after its two steps have consumed it
    int i0 = 0;
    float av0[4], av1[4];
    for (; i0 + 2 * PD <= total; i0 += 2 * PD) {
#pragma unroll
      for (int p = 0; p < PD; ++p) {
        const float4 v = ring[p], w = swap_pair(v);
        frag0(v, w, av0);
        frag1(v, w, av1);
        step(av0, bq[0]);
        step(av1, bq[1]);
        ring[p] = fetch();
      }
    }
#pragma unroll
    for (int p = 0; p < PD; ++p) {
      if (i0 + 2 * p >= total) break;
      const float4 v = ring[p], w = swap_pair(v);
      frag0(v, w, av0);
      frag1(v, w, av1);
      step(av0, bq[0]);
      if (i0 + 2 * p + 1 < total) step(av1, bq[1]);
    }
  }
  // tiles between the group's M_g and the vector stride M hold zeros
  for (int m = m0 + mstep * mcnt; m < nMall; m += mstep)
#pragma unroll
    for (int n = 0; n < NT; ++n)
      if (yp[n]) reinterpret_cast<float4*>(yp[n] + 8 * m + 2 * kr)[0] = make_float4(0.f, 0.f, 0.f, 0.f);
}

#define DFMM_GG_PARAMS                                                                                       \
  const float4 *__restrict__ A, const int64_t *__restrict__ aoff, const int *__restrict__ aexp,               \
      const int *__restrict__ gmk, int M, int K,                                                               \
      int split, const int *__restrict__ gops, const int *__restrict__ gv0, const int *__restrict__ vsrc,      \
      const int *__restrict__ vdst, const int *__restrict__ chunk_grp, const int *__restrict__ chunk_c0,       \
      int nrhs, const float2 *__restrict__ X, float2 *__restrict__ Y
#define DFMM_GG_ARGS A, aoff, aexp, gmk, M, K, split, gops, gv0, vsrc, vdst, chunk_grp, chunk_c0, nrhs, X, Y

// The same tile engine under two names, so that kernel traces separate the
// translations (M2L of Algorithm 1) from the pair-form tree transfers (M2M and L2L).
template <int NT, bool ALDS, bool ACC64, int NW, int PREC>
__global__ void __launch_bounds__(64 * NW) k_m2l(DFMM_GG_PARAMS) {
  ggemm_tile<NT, ALDS, ACC64, NW, PREC>(DFMM_GG_ARGS, int(blockIdx.x), int(blockIdx.y), int(gridDim.y));
}
template <int NT, bool ALDS, bool ACC64, int NW, int PREC>
__global__ void __launch_bounds__(64 * NW) k_transfer(DFMM_GG_PARAMS) {
  ggemm_tile<NT, ALDS, ACC64, NW, PREC>(DFMM_GG_ARGS, int(blockIdx.x), int(blockIdx.y), int(gridDim.y));
}

// All M2L launches of an apply (every HF level and the leaf level) in one
// launch: they read only the upward pass's outputs, so their chunks can share
// the GPU (the HBM-bound HF chunks beside the compute-bound leaf-level ones).
// A chunk names its problem and M-slice; each problem writes its own pair
// scratch, reduced afterwards in the order of the separate launches.
constexpr int kMaxProbs = 8;
struct GgProb {
  const float4* A;
  const int64_t* aoff;
  const int* aexp;
  const int* gmk;
  const int* gops;
  const int* gv0;
  const int* vsrc;
  const int* vdst;
  const float2* X;
  float2* Y;
  int M, K, split, slices;
};
struct GgProbs {
  GgProb p[kMaxProbs];
};
template <int NT, int NW, int PREC>
__global__ void __launch_bounds__(64 * NW) k_m2l_fused(const GgProbs P, const int* __restrict__ chunk_ps,
                                                        const int* __restrict__ chunk_grp,
                                                        const int* __restrict__ chunk_c0, int nrhs) {
  const int c = int(blockIdx.x);
  const int ps = chunk_ps[c];  // problem | slice << 4
  const GgProb& q = P.p[ps & 15];
  ggemm_tile<NT, false, false, NW, PREC>(q.A, q.aoff, q.aexp, q.gmk, q.M, q.K, q.split, q.gops, q.gv0, q.vsrc,
                                         q.vdst, chunk_grp, chunk_c0, nrhs, q.X, q.Y, c, ps >> 4, q.slices);
}
#undef DFMM_GG_PARAMS
#undef DFMM_GG_ARGS

// ---- slot-form GEMM: every output slot sums its terms in registers ---------------
// A workgroup owns one output vector (a slot, 16 NT of its right-hand sides)
// and one wave per 16-row M-tile of it.  It walks the slot's terms in their
// fixed order: each term's source columns are staged in LDS (double-buffered:
// the next term's columns are loaded into registers while this term's
// products run, and stored after them), and each wave holds the whole tile of
// the term's operator in registers, loaded one term ahead.  A term's products
// accumulate in float32 MFMA chains (one operator row against the column, as
// in the pair form) and are added into float64 sums across terms, so the slot's
// sum has the rounding of the pair form's fixed-order reduction without its
// stored pair outputs.  The terms of a launch are of two kinds with their own
// operator and source arrays (a level's M2L pairs and its L2L terms).
struct SlotArgs {
  const int* order;   // launch order of the groups
  const int* t0;      // term range of each group
  const int* gm;      // padded rows of each group's operators
  const int4* terms;  // (operator float4 offset, source vector, K | split << 12 | kind << 14, 0)
  const float4* A0;
  const float4* A1;
  const float2* X0;
  const float2* X1;
  int KX0, KX1;       // row strides of the two kinds' source vectors
  int M;              // row stride of the output vectors
  int cpg;            // column chunks per group
  int S4;             // LDS column stride in float4
  int waves;          // waves per workgroup (M-tiles per slice)
  const int* gdst;    // output vector of each group (null: the group's own index)
};
constexpr int SLOT_UB = 2;  // staged float4 per thread and term
// s_waitcnt immediate for vmcnt(0) alone (gfx9 encoding: vmcnt bits 3:0 and
// 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their maxima)
constexpr int kWaitVm0 = 0x0F70;

// f(std::integral_constant<int, q>) for the runtime q in 1 .. QMAX (nothing
// for any other q): one branch-free body per term length
template <int QMAX, typename F, int... I>
__device__ __forceinline__ void slot_dispatch_seq(int q, F&& f, std::integer_sequence<int, I...>) {
  (void)((q == I + 1 && (f(std::integral_constant<int, I + 1>{}), true)) || ...);
}
template <int QMAX, typename F>
__device__ __forceinline__ void slot_dispatch(int q, F&& f) {
  slot_dispatch_seq<QMAX>(q, static_cast<F&&>(f), std::make_integer_sequence<int, QMAX>{});
}

template <int NT, int PMAX>
__device__ __forceinline__ void slot_gemm(const SlotArgs& a, int nrhs, float2* __restrict__ Y) {
  constexpr int NC = NT * 16;
  extern __shared__ float4 xs[];  // two buffers of NC columns, S4 float4 each, then the group's terms
  const int BS = 64 * a.waves;
  const int tid = int(threadIdx.x);
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int j = lane & 15, kr = lane >> 4;
  const bool odd = (j & 1) != 0;
  const int chunk = int(blockIdx.x);
  const int g = a.order[chunk / a.cpg];
  const int c0 = (chunk % a.cpg) * NC;
  const int nc = min(NC, nrhs - c0);
  const int tb = a.t0[g], te = a.t0[g + 1];
  const int nM = a.gm[g] / 8;
  const int m = int(blockIdx.y) * a.waves + wave;
  const bool act = m < nM;  // wave-uniform: this wave's tile has operator rows
  const int S4 = a.S4;
  const int lofs = (j >> 1) * 4 + kr;

  struct Tm {
    const float4* A;
    const float2* X;  // column c0 of the source slot
    int KX, Kg, split, mg;
  };
  auto decode = [&](int4 e) {  // e: the term's table entry (wave-uniform)
    e.x = __builtin_amdgcn_readfirstlane(e.x);
    e.y = __builtin_amdgcn_readfirstlane(e.y);
    e.z = __builtin_amdgcn_readfirstlane(e.z);
    e.w = __builtin_amdgcn_readfirstlane(e.w);
    const int kind = (e.z >> 14) & 1;
    Tm r;
    r.KX = kind ? a.KX1 : a.KX0;
    r.A = (kind ? a.A1 : a.A0) + e.x;
    r.X = (kind ? a.X1 : a.X0) + (int64_t(e.y) * nrhs + c0) * r.KX;
    r.Kg = e.z & 0xFFF;
    r.split = (e.z >> 12) & 3;
    r.mg = e.w;
    return r;
  };
  float4 xv[SLOT_UB];
  // thread index idx < 2^11 as (column, float4 of the column): idx / (Kg / 2) by
  // the term's multiplier
  auto x_load = [&](const Tm& T) {  // this thread's share of the term's columns
    const int per_col = T.Kg / 2, pcs = per_col / T.split, nel = NC * per_col;
#pragma unroll
    for (int u = 0; u < SLOT_UB; ++u) {
      const int idx = tid + u * BS;
      xv[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (idx < nel) {
        const int col = int(__umul24(unsigned(idx), unsigned(T.mg)) >> 23), q4 = idx - col * per_col;
        if (col < nc)
          xv[u] = reinterpret_cast<const float4*>(T.X + int64_t(col) * T.KX)[q4 < pcs ? q4 : q4 - pcs];
      }
    }
  };
  auto x_store = [&](int buf, const Tm& T) {
    const int per_col = T.Kg / 2, nel = NC * per_col;
    float4* xb = xs + buf * NC * S4;
#pragma unroll
    for (int u = 0; u < SLOT_UB; ++u) {
      const int idx = tid + u * BS;
      if (idx < nel) {
        const int col = int(__umul24(unsigned(idx), unsigned(T.mg)) >> 23), q4 = idx - col * per_col;
        xb[col * S4 + q4] = xv[u];
      }
    }
  };
  // this wave's tile of a term's operator (Q4 k-steps from base): pair p holds
  // k-steps 2p (even lane) and 2p + 1 (odd lane); pairs past the end repeat the
  // last step, so every load stays inside the tile
  auto op_pair = [&](const float4* base, int Q4, int p) { return base[min(2 * p + (odd ? 1 : 0), Q4 - 1) * 32]; };
  double a64[NT][4];
#pragma unroll
  for (int n = 0; n < NT; ++n)
#pragma unroll
    for (int q = 0; q < 4; ++q) a64[n][q] = 0.0;
  // The products of one term of Q4 k-steps (a compile-time count, so the body
  // has no branches).  The operator tile lives in one set of registers: as soon
  // as pair p has been turned into MFMA fragments, the next term's pair p is
  // loaded into it (a term of Q4n steps from base rn), so that load has a whole
  // term of products to land.
  auto compute = [&](auto q4c, float4 (&r)[PMAX], int buf, const float4* rn, int Q4n) {
    constexpr int Q4 = decltype(q4c)::value;
    // kr made opaque for each term: otherwise the compiler hoists kr * Q4 for
    // every length out of the term loop and spills the fourteen offsets
    int kro = kr;
    asm volatile("" : "+v"(kro));
    const float4* bcol = xs + buf * NC * S4 + j * S4 + kro * Q4;
    v4f acc[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[n] = v4f{0.f, 0.f, 0.f, 0.f};
    // The workgroup barrier keeps a SIMD's waves in step, so they reach their
    // staging work (term decode, column loads and stores) together and the
    // matrix core idles meanwhile; a wave in its products takes issue
    // priority over one that is staging.
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int p = 0; p < (Q4 + 1) / 2; ++p) {
      const float4 v = r[p], w = swap_pair(v);
      // the complex A fragments as real rows (even row: Re, -Im; odd row: Im, Re)
      const float a0[4] = {odd ? w.y : v.x, odd ? w.x : -v.y, odd ? w.w : v.z, odd ? w.z : -v.w};
      const float a1[4] = {odd ? v.y : w.x, odd ? v.x : -w.y, odd ? v.w : w.z, odd ? v.z : -w.w};
      r[p] = op_pair(rn, Q4n, p);
      // the scheduler would otherwise move the reload down to the end of the
      // term, where it can no longer land during the products
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const float4 b = bcol[n * 16 * S4 + 2 * p];
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[0], b.x, acc[n], 0, 0, 0);
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[1], b.y, acc[n], 0, 0, 0);
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[2], b.z, acc[n], 0, 0, 0);
        acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[3], b.w, acc[n], 0, 0, 0);
      }
      if (2 * p + 1 < Q4) {
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          const float4 b = bcol[n * 16 * S4 + 2 * p + 1];
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[0], b.x, acc[n], 0, 0, 0);
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[1], b.y, acc[n], 0, 0, 0);
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[2], b.z, acc[n], 0, 0, 0);
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[3], b.w, acc[n], 0, 0, 0);
        }
      }
    }
    __builtin_amdgcn_s_setprio(0);
    // the next term is longer than this one
#pragma unroll
    for (int p = (Q4 + 1) / 2; p < PMAX; ++p) r[p] = op_pair(rn, Q4n, p);
#pragma unroll
    for (int n = 0; n < NT; ++n)
#pragma unroll
      for (int q = 0; q < 4; ++q) a64[n][q] += double(acc[n][q]);
  };

  if (tb < te) {
    // the group's term table in LDS (decoding a term is then one broadcast read)
    int4* tl = reinterpret_cast<int4*>(xs + 2 * NC * S4);
    for (int i = tid; i < te - tb; i += BS) tl[i] = a.terms[tb + i];
    __syncthreads();
    float4 r[PMAX];
    Tm T = decode(tl[0]);
    if (act) {
      const float4* base = T.A + m * (T.Kg / 8 * 32) + lofs;
#pragma unroll
      for (int p = 0; p < PMAX; ++p) r[p] = op_pair(base, T.Kg / 8, p);
    }
    x_load(T);
    x_store(0, T);
    __syncthreads();
    // Each term first retires every load in flight (its operator tile, loaded
    // during the previous term) and only then issues the next term's column
    // loads: without this wait the compiler waits for the prefetch itself
    // before the first product.  The last term reloads its own tile (a
    // harmless repeat) so that the body is the same for every term.
    for (int t = tb, buf = 0;; ++t, buf ^= 1) {
      const bool more = t + 1 < te;
      Tm Tn = T;
      __builtin_amdgcn_s_waitcnt(kWaitVm0);
      if (more) {
        Tn = decode(tl[t + 1 - tb]);
        x_load(Tn);
      }
      if (act) {
        const int Q4n = Tn.Kg / 8;
        const float4* rn = Tn.A + m * (Q4n * 32) + lofs;
        slot_dispatch<2 * PMAX>(T.Kg / 8, [&](auto q4c) { compute(q4c, r, buf, rn, Q4n); });
      }
      if (more) x_store(buf ^ 1, Tn);
      __syncthreads();
      if (!more) break;
      T = Tn;
    }
  }
  // lane (j, kr) holds real rows 4 kr .. 4 kr + 3 (complex rows 2 kr, 2 kr + 1) of
  // tile m for column j of each column tile; tiles past M_g are written as zeros
  const int gy = a.gdst ? a.gdst[g] : g;
  if (m < a.M / 8) {
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const int col = n * 16 + j;
      if (col < nc) {
        float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
        if (act) o = make_float4(float(a64[n][0]), float(a64[n][1]), float(a64[n][2]), float(a64[n][3]));
        reinterpret_cast<float4*>(Y + (int64_t(gy) * nrhs + c0 + col) * a.M + 8 * m + 2 * kr)[0] = o;
      }
    }
  }
}

// The slot form under two names, so that kernel traces separate the upward
// transfers (M2M) from the downward pass (M2L pairs and L2L terms of a level).
template <int NT, int PMAX>
__global__ void __launch_bounds__(1024) k_m2m_slot(const SlotArgs a, int nrhs, float2* __restrict__ Y) {
  slot_gemm<NT, PMAX>(a, nrhs, Y);
}
template <int NT, int PMAX>
__global__ void __launch_bounds__(1024) k_m2l_slot(const SlotArgs a, int nrhs, float2* __restrict__ Y) {
  slot_gemm<NT, PMAX>(a, nrhs, Y);
}

// ---- U[slot] (+)= sum of Y over the pairs of the slot -------------------------------
__global__ void k_reduce(const int* __restrict__ rs, const int* __restrict__ ri, const float2* __restrict__ Y,
                         int64_t nslot, int RN, int accumulate, float2* __restrict__ U) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nslot * RN) return;
  int64_t s = t / RN;
  int e = int(t % RN);
  // the pair contributions of one slot cancel to a large extent: sum in float64
  double ax = 0.0, ay = 0.0;
  if (accumulate) {
    const float2 u0 = U[t];
    ax = u0.x;
    ay = u0.y;
  }
  int j = rs[s];
  const int j1 = rs[s + 1];
  for (; j + 4 <= j1; j += 4) {  // four loads in flight, added in order
    const float2 y0 = Y[int64_t(ri[j]) * RN + e], y1 = Y[int64_t(ri[j + 1]) * RN + e];
    const float2 y2 = Y[int64_t(ri[j + 2]) * RN + e], y3 = Y[int64_t(ri[j + 3]) * RN + e];
    ax += y0.x; ay += y0.y;
    ax += y1.x; ay += y1.y;
    ax += y2.x; ay += y2.y;
    ax += y3.x; ay += y3.y;
  }
  for (; j < j1; ++j) {
    const float2 y = Y[int64_t(ri[j]) * RN + e];
    ax += y.x;
    ay += y.y;
  }
  U[t] = make_float2(float(ax), float(ay));
}

// ---- leaf evaluation: L2T plus the near-field sum, written in user order ----------
// One wave per leaf.  Lane = (target t = lane % 16, slice s = lane / 16): the
// wave takes the leaf's targets 16 at a time and every lane sums over a quarter
// of the sources (rows q of the L2T weights W, points of the adjacent leaves
// for the near field); the four partial sums of a target are combined with
// lane shuffles.  The adjacent leaves' points are staged in LDS in chunks.
// Near-field terms accumulate in float64.  PRECISE (plans with eps < 1e-5)
// forms the point differences from the hi/lo parts in float64 (green_d);
// otherwise they are float32 hi/lo differences and green_f.
constexpr int EV_BS = 64;

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
  return __shfl_xor(v, m, 64);
}

constexpr int EV_CHUNK = 256;  // source points staged in LDS at a time
// near leaves whose point ranges are tabled at a time (the lookup of the leaf
// holding a staged point searches 32 entries)
constexpr int NB_CHUNK = 32;
constexpr int EV_SUM = 16;     // fast plans: products summed in float32 this many at a time
// Separations come from the hi/lo float parts of the points: the hi parts of a
// close pair subtract exactly, so even a pair at distance 0.01 keeps its
// separation to ~1e-14 (leaf-local float32 coordinates would leave ~1e-8
// absolute, i.e. 1e-6 relative in 1/r for such pairs).  Fast plans (eps >= 1e-5)
// then work in float32 and sum EV_SUM products at a time before adding them in
// float64; precise plans form the separations, 1/r and the products in float64.
// The near field of every target goes to unear (float64, sorted order); it
// needs only the permuted densities, so it runs on a second stream beside the
// far-field passes, and k_l2t adds it to the far field.
template <bool PRECISE, int RC>  // RC: right-hand sides per pass
__global__ void __launch_bounds__(EV_BS) k_leaf_eval(const float4* __restrict__ phi, const float4* __restrict__ plo,
                                                      const int* __restrict__ lstart,
                                                      const int* __restrict__ nstart, const int* __restrict__ nsrc,
                                                      const float2* __restrict__ fs, int nrhs, int64_t N,
                                                      double2* __restrict__ unear) {
  __shared__ float4 sh[EV_CHUNK], sq[EV_CHUNK];
  __shared__ float2 sf[EV_CHUNK * RC];
  __shared__ int nb_beg[EV_BS], nb_off[EV_BS + 1];
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  const int tl = lane & 15, sl = lane >> 4;
  const int s0 = lstart[b], s1 = lstart[b + 1];
  const int n0 = nstart[b];
  // near leaves: 27 at most in a uniform tree, more for a coarse leaf of an
  // adaptive one; their point ranges are tabled NB_CHUNK leaves at a time
  const int ntot = nstart[b + 1] - n0;
  for (int k0 = 0; k0 < nrhs; k0 += RC) {
    const int nk = min(RC, nrhs - k0);
    for (int t0 = s0; t0 < s1; t0 += 16) {
      const int t = t0 + tl;
      const bool act = t < s1;
      const int tt = act ? t : s0;
      const float4 th = phi[tt], tq = plo[tt];
      double ar[RC], ai[RC];
#pragma unroll
      for (int k = 0; k < RC; ++k) ar[k] = ai[k] = 0.0;
      for (int c0 = 0; c0 < ntot; c0 += NB_CHUNK) {
        const int nn = min(NB_CHUNK, ntot - c0);
        __syncthreads();  // the previous tables and points are consumed
        {  // this chunk's neighbour ranges; offsets by a wave prefix sum
          int beg = 0, cnt = 0;
          if (lane < nn) {
            const int A = nsrc[n0 + c0 + lane];
            beg = lstart[A];
            cnt = lstart[A + 1] - beg;
          }
          int incl = cnt;
          for (int d = 1; d < EV_BS; d <<= 1) {
            const int v = __shfl_up(incl, d, EV_BS);
            if (lane >= d) incl += v;
          }
          nb_beg[lane] = beg;
          nb_off[lane] = incl - cnt;
          if (lane == EV_BS - 1) nb_off[EV_BS] = incl;
        }
        __syncthreads();
        const int total = nb_off[nn];
        // the chunk's points are staged in LDS EV_CHUNK at a time
        for (int base = 0; base < total; base += EV_CHUNK) {
          const int fill = min(EV_CHUNK, total - base);
          __syncthreads();
          for (int i = lane; i < fill; i += EV_BS) {
            const int gidx = base + i;
            int kk = 0;  // the neighbour holding element gidx: largest kk with nb_off[kk] <= gidx
#pragma unroll
            for (int step = 16; step > 0; step >>= 1)
              if (kk + step < nn && nb_off[kk + step] <= gidx) kk += step;
            const int j = nb_beg[kk] + (gidx - nb_off[kk]);
            sh[i] = phi[j];
            sq[i] = plo[j];
            for (int k = 0; k < nk; ++k) sf[i * RC + k] = fs[int64_t(j) * nrhs + k0 + k];
          }
          __syncthreads();
          if constexpr (PRECISE) {  // 1/r and the products in float64
            for (int i = sl; i < fill; i += 4) {
              const float4 h = sh[i], l = sq[i];
              const double dx = (double(th.x) - double(h.x)) + (double(tq.x) - double(l.x));
              const double dy = (double(th.y) - double(h.y)) + (double(tq.y) - double(l.y));
              const double dz = (double(th.z) - double(h.z)) + (double(tq.z) - double(l.z));
              const double2 gg = green_d(dx, dy, dz);
#pragma unroll
              for (int k = 0; k < RC; ++k) {
                if (k < nk) {
                  const float2 fk = sf[i * RC + k];
                  ar[k] += gg.x * double(fk.x) - gg.y * double(fk.y);
                  ai[k] += gg.x * double(fk.y) + gg.y * double(fk.x);
                }
              }
            }
          } else {
            for (int i0 = sl; i0 < fill; i0 += 4 * EV_SUM) {
              const int i1 = min(fill, i0 + 4 * EV_SUM);
              float cr[RC], ci[RC];
#pragma unroll
              for (int k = 0; k < RC; ++k) cr[k] = ci[k] = 0.f;
              for (int i = i0; i < i1; i += 4) {
                const float4 h = sh[i], l = sq[i];
                const float2 gg = green_f((th.x - h.x) + (tq.x - l.x), (th.y - h.y) + (tq.y - l.y),
                                          (th.z - h.z) + (tq.z - l.z));
#pragma unroll
                for (int k = 0; k < RC; ++k) {
                  if (k < nk) {
                    const float2 fk = sf[i * RC + k];
                    cr[k] = fmaf(gg.x, fk.x, fmaf(-gg.y, fk.y, cr[k]));
                    ci[k] = fmaf(gg.x, fk.y, fmaf(gg.y, fk.x, ci[k]));
                  }
                }
              }
#pragma unroll
              for (int k = 0; k < RC; ++k) {
                ar[k] += cr[k];
                ai[k] += ci[k];
              }
            }
          }
        }
      }  // neighbour chunks
#pragma unroll
      for (int k = 0; k < RC; ++k) {
        ar[k] += shfl_xor_d(ar[k], 16);
        ai[k] += shfl_xor_d(ai[k], 16);
        ar[k] += shfl_xor_d(ar[k], 32);
        ai[k] += shfl_xor_d(ai[k], 32);
      }
      if (act && sl == 0)
        for (int k = 0; k < nk; ++k) unear[int64_t(k0 + k) * N + t] = make_double2(ar[k], ai[k]);
    }
  }
}

// Near field for many right-hand sides (fast plans): per leaf, U[t][k] +=
// sum_s G(x_t, x_s) F[s][k] as a complex GEMM on MFMA.  A workgroup takes a
// leaf, a block of up to NM_TB of its targets and 16 NCT right-hand sides;
// the adjacent leaves' points are taken NM_SC at a time, one per lane of every
// wave (in registers), and their densities staged in LDS.
// Each wave owns 8-target row tiles (w, w + 4, ...): it evaluates G for its 8
// targets x NM_SC sources once (one source per lane, the hi/lo separations of
// the VALU path) into LDS, then runs the products on v_mfma_f32_16x16x4f32 with
// complex as interleaved real (A row 2t = (Re G, -Im G), row 2t + 1 =
// (Im G, Re G) over k = (Re F, Im F) of a source).  Partial sums go to
// float64 every 16 sources, as in the VALU path.
constexpr int NM_SC = 64;   // sources per staged chunk
constexpr int kNearMfmaMinRhs = 4;  // fast plans with at least this many rhs take the MFMA path
constexpr int NM_NW = 4;    // waves per workgroup
constexpr int NM_MAXT = 2;  // row tiles per wave
constexpr int NM_TB = 8 * NM_NW * NM_MAXT;  // targets per workgroup (64)
template <int NCT, int PREC>
__global__ void __launch_bounds__(64 * NM_NW) k_near_mfma(const float4* __restrict__ phi, const float4* __restrict__ plo,
                                                          const int* __restrict__ lstart,
                                                          const int* __restrict__ nstart, const int* __restrict__ nsrc,
                                                          const float2* __restrict__ fs, int nrhs, int64_t N,
                                                          double2* __restrict__ unear) {
  constexpr int NCOL = 16 * NCT;
  constexpr int GS = NM_SC + 1;  // G row stride (float2): rows of different targets on different banks
  static_assert(NM_SC == 64 && NB_CHUNK <= 32, "one source per lane; the neighbour search covers 32 ranges");
  static_assert(NM_SC * NCOL % (64 * NM_NW) == 0, "whole staged densities per thread");
  __shared__ float4 th[NM_TB], tq[NM_TB];
  __shared__ float2 sf[NM_SC * NCOL];
  __shared__ float2 sg[NM_NW * 8 * GS];
  __shared__ int nb_beg[64], nb_off[65];
  __shared__ int fexp[NCOL];  // 16-bit plans: scale exponent of each staged density column
  const int b = blockIdx.x;
  const int c0 = int(blockIdx.y) * NCOL;
  const int s0 = lstart[b] + int(blockIdx.z) * NM_TB;
  const int s1 = min(lstart[b + 1], s0 + NM_TB);
  if (s0 >= s1) return;  // uniform: this target block is past the leaf's end
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int n0 = nstart[b];
  // near leaves: 27 at most in a uniform tree, more for a coarse leaf of an
  // adaptive one; their point ranges are tabled NB_CHUNK leaves at a time
  const int ntot = nstart[b + 1] - n0;
  for (int i = threadIdx.x; i < NM_TB; i += 64 * NM_NW) {
    const int t = min(s0 + i, s1 - 1);
    th[i] = phi[t];
    tq[i] = plo[t];
  }
  const int ntiles = (s1 - s0 + 7) / 8;
  const int rr = lane & 15, kk = lane >> 4;  // A row / B column, k index of this lane
  const int tr = rr >> 1, kp = kk & 1;       // target of the row, Re/Im part of k
  const bool rodd = (rr & 1) != 0;
  v4f acc[NM_MAXT][NCT];
  double a64[NM_MAXT][NCT][4];
#pragma unroll
  for (int i = 0; i < NM_MAXT; ++i)
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      acc[i][c] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) a64[i][c][r] = 0.0;
    }
  float2* gw = sg + w * 8 * GS;
  for (int c0n = 0; c0n < ntot; c0n += NB_CHUNK) {
    const int nn = min(NB_CHUNK, ntot - c0n);
    __syncthreads();  // the previous tables and points are consumed
    if (w == 0) {  // this chunk's neighbour ranges and their offsets (wave prefix sum)
      int beg = 0, cnt = 0;
      if (lane < nn) {
        const int A = nsrc[n0 + c0n + lane];
        beg = lstart[A];
        cnt = lstart[A + 1] - beg;
      }
      int incl = cnt;
      for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d, 64);
        if (lane >= d) incl += v;
      }
      nb_beg[lane] = beg;
      nb_off[lane] = incl - cnt;
      if (lane == 63) nb_off[64] = incl;
    }
    __syncthreads();
    const int total = nb_off[nn];
    for (int base = 0; base < total; base += NM_SC) {
      const int fill = min(NM_SC, total - base);
      // every wave finds the chunk's sources itself, lane i -> source base + i,
      // and keeps that point (hi/lo parts) in registers; the densities are
      // loaded through the index of their source's lane, all before the
      // barrier, so the loads overlap the other waves' products
      const bool sval = lane < fill;
      int j = -1;
      float4 h = make_float4(0.f, 0.f, 0.f, 0.f), l = h;  // an unused lane's source: a finite point (zero densities)
      if (sval) {
        const int g = base + lane;
        int q = 0;  // the neighbour holding element g: largest q with nb_off[q] <= g
#pragma unroll
        for (int step = 16; step > 0; step >>= 1)
          if (q + step < nn && nb_off[q + step] <= g) q += step;
        j = nb_beg[q] + (g - nb_off[q]);
        h = phi[j];
        l = plo[j];
      }
      constexpr int FPT = NM_SC * NCOL / (64 * NM_NW);  // staged densities per thread
      float2 fv[FPT];
#pragma unroll
      for (int k = 0; k < FPT; ++k) {
        const int e = int(threadIdx.x) + k * 64 * NM_NW;
        const int i = e / NCOL, c = e % NCOL;
        const int ji = __shfl(j, i, 64);
        fv[k] = (ji >= 0 && c0 + c < nrhs) ? fs[int64_t(ji) * nrhs + c0 + c] : make_float2(0.f, 0.f);
      }
      __syncthreads();  // the previous chunk is consumed
#pragma unroll
      for (int k = 0; k < FPT; ++k) sf[int(threadIdx.x) + k * 64 * NM_NW] = fv[k];
      __syncthreads();
      if constexpr (PREC != 0) {  // densities as (hi re | hi im, lo re | lo im) words, scaled per column
        if (threadIdx.x < NCOL) {
          int e = 0;
          if constexpr (PREC == PREC_F16) {
            float mx = 0.f;
            for (int i = 0; i < NM_SC; ++i) {
              const float2 v = sf[i * NCOL + threadIdx.x];
              mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
            }
            if (mx > 0.f) {
              int E;
              (void)frexpf(mx, &E);
              e = 14 - E;
            }
          }
          fexp[threadIdx.x] = e;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < NM_SC * NCOL; e += 64 * NM_NW) {
          const int x = fexp[e % NCOL];
          const float2 v = sf[e];
          unsigned hi, lo;
          split_pair<PREC>(ldexpf(v.x, x), ldexpf(v.y, x), hi, lo);
          sf[e] = make_float2(__uint_as_float(hi), __uint_as_float(lo));
        }
        __syncthreads();
      }
#pragma unroll
      for (int i = 0; i < NM_MAXT; ++i) {
        const int rt = w + NM_NW * i;
        if (rt >= ntiles) break;
        // G for this tile's 8 targets and this lane's source
        float2 gv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const float4 a = th[rt * 8 + t], c = tq[rt * 8 + t];
          gv[t] = green_f((a.x - h.x) + (c.x - l.x), (a.y - h.y) + (c.y - l.y), (a.z - h.z) + (c.z - l.z));
          // float32 products need no mask: unused sources have zero densities
          // and rows past the leaf's targets are not stored; the 16-bit split
          // scales by the tile's largest |G|, which must see only real pairs
          if (PREC != 0 && (!sval || s0 + rt * 8 + t >= s1)) gv[t] = make_float2(0.f, 0.f);
        }
        int eg = 0;  // 16-bit plans: the tile's scale exponent (largest |G| below 2^14)
        if constexpr (PREC == PREC_F16) {
          float mx = 0.f;
#pragma unroll
          for (int t = 0; t < 8; ++t) mx = fmaxf(mx, fmaxf(fabsf(gv[t].x), fabsf(gv[t].y)));
#pragma unroll
          for (int m = 32; m > 0; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m, 64));
          if (mx > 0.f) {
            int E;
            (void)frexpf(mx, &E);
            eg = 14 - E;
          }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          float2 g = gv[t];
          if constexpr (PREC != 0) {  // (hi re | hi im, lo re | lo im) words
            unsigned hi, lo;
            split_pair<PREC>(ldexpf(g.x, eg), ldexpf(g.y, eg), hi, lo);
            g = make_float2(__uint_as_float(hi), __uint_as_float(lo));
          }
          gw[t * GS + lane] = g;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if constexpr (PREC != 0) {
          // products: one 16x16x32 MFMA per term covers 16 sources; lane k-group kk
          // holds sources 4 kk .. 4 kk + 3 of the block, (Re, Im) each
          float osc[NCT];
#pragma unroll
          for (int c = 0; c < NCT; ++c) osc[c] = ldexpf(1.0f, -(eg + fexp[c * 16 + rr]));
          constexpr unsigned SG = 0x80000000u;
#pragma unroll 1
          for (int q = 0; q < NM_SC / 16; ++q) {
            const int sb = 16 * q + 4 * kk;
            unsigned ah[4], al[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float2 g = gw[tr * GS + sb + e];
              const unsigned h = __float_as_uint(g.x), o = __float_as_uint(g.y);
              ah[e] = rodd ? rot16(h) : (h ^ SG);  // even row (Re G, -Im G), odd row (Im G, Re G)
              al[e] = rodd ? rot16(o) : (o ^ SG);
            }
            const v4u av = {ah[0], ah[1], ah[2], ah[3]}, aw = {al[0], al[1], al[2], al[3]};
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
              unsigned bh[4], bl[4];
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const float2 f = sf[(sb + e) * NCOL + c * 16 + rr];
                bh[e] = __float_as_uint(f.x);
                bl[e] = __float_as_uint(f.y);
              }
              const v4u bv = {bh[0], bh[1], bh[2], bh[3]}, bw = {bl[0], bl[1], bl[2], bl[3]};
              v4f a = mfma16<PREC>(av, bv, v4f{0.f, 0.f, 0.f, 0.f});
              a = mfma16<PREC>(av, bw, a);
              a = mfma16<PREC>(aw, bv, a);
#pragma unroll
              for (int r = 0; r < 4; ++r) a64[i][c][r] += double(a[r] * osc[c]);
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          continue;
        }
        // products: MFMA step q covers sources 2q, 2q + 1.  The lane's A entry
        // is component rodd ^ kp of G (Re G, -Im G on even rows, Im G, Re G on
        // odd ones: negated where the row is even and k is Im), its B entry
        // component kp of the density: single-float reads, no selects.
        const float* gf = reinterpret_cast<const float*>(gw + tr * GS + (kk >> 1)) + ((rodd ? 1 : 0) ^ kp);
        const float* ff = reinterpret_cast<const float*>(sf + (kk >> 1) * NCOL + rr) + kp;
        const unsigned gneg = (!rodd && kp) ? 0x80000000u : 0u;
#pragma unroll 4
        for (int q = 0; q < NM_SC / 2; ++q) {
          const float av = __uint_as_float(__float_as_uint(gf[2 * 2 * q]) ^ gneg);
#pragma unroll
          for (int c = 0; c < NCT; ++c)
            acc[i][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, ff[2 * (2 * q * NCOL + c * 16)], acc[i][c], 0, 0, 0);
          if ((q & 7) == 7) {
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
#pragma unroll
              for (int r = 0; r < 4; ++r) a64[i][c][r] += double(acc[i][c][r]);
              acc[i][c] = v4f{0.f, 0.f, 0.f, 0.f};
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  }  // neighbour chunks
  // lane holds rows 4 kk .. 4 kk + 3 = (Re, Im) of targets 2 kk, 2 kk + 1, column rr
#pragma unroll
  for (int i = 0; i < NM_MAXT; ++i) {
    const int rt = w + NM_NW * i;
    if (rt >= ntiles) break;
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int col = c0 + c * 16 + rr;
      if (col >= nrhs) continue;
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        const int t = s0 + rt * 8 + 2 * kk + h2;
        if (t < s1) unear[int64_t(col) * N + t] = make_double2(a64[i][c][2 * h2], a64[i][c][2 * h2 + 1]);
      }
    }
  }
}

// L2T and the output: u[k][perm[t]] = sum_q W[t][q] U_LF[leaf(t)][k][q] + unear[k][t],
// u of batch column k being the output of its request.
// 16 lanes per target read 16 consecutive q at a time (128-byte runs); a
// lane keeps its W values over the right-hand sides.
constexpr int L2T_BS = 256;
constexpr int L2T_QMAX = 16;  // W values per lane: R <= 16 * L2T_QMAX
__global__ void __launch_bounds__(L2T_BS) k_l2t(const float2* __restrict__ W, const float2* __restrict__ ulf,
                                                 const int* __restrict__ leaf_of, const double2* __restrict__ unear,
                                                 const int* __restrict__ perm, int R, int nrhs, int64_t N,
                                                 const ReqTable Q) {
  const int64_t t = (int64_t(blockIdx.x) * L2T_BS + threadIdx.x) >> 4;
  const int l = threadIdx.x & 15;
  const bool act = t < N;
  const int64_t tt = act ? t : 0;
  const int leaf = leaf_of[tt];
  float2 w[L2T_QMAX];
  const int nq = (R - l + 15) / 16;  // this lane's q = l, l + 16, ...
#pragma unroll
  for (int i = 0; i < L2T_QMAX; ++i)
    if (i < nq) w[i] = W[tt * R + l + 16 * i];
  const int64_t o = act ? perm[tt] : 0;
  for (int k = 0; k < nrhs; ++k) {
    const float2* ur = ulf + (int64_t(leaf) * nrhs + k) * R;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int i = 0; i < L2T_QMAX; ++i)
      if (i < nq) cfma(acc, w[i], ur[l + 16 * i]);
#pragma unroll
    for (int m = 8; m > 0; m >>= 1) {
      acc.x += __shfl_xor(acc.x, m, 16);
      acc.y += __shfl_xor(acc.y, m, 16);
    }
    if (act && l == 0) {
      const double2 nf = unear[int64_t(k) * N + tt];
      const int r = req_of(Q, k);
      Q.u[r][int64_t(k - Q.k0[r]) * N + o] = make_float2(float(double(acc.x) + nf.x), float(double(acc.y) + nf.y));
    }
  }
}

// L2T for many right-hand sides: one block per leaf stages the leaf's incoming
// potentials of kc right-hand sides in LDS once, instead of every target
// re-reading them for every right-hand side; 16 lanes per target and the same
// summation order as k_l2t.
__global__ void __launch_bounds__(L2T_BS) k_l2t_leaf(const float2* __restrict__ W, const float2* __restrict__ ulf,
                                                      const int* __restrict__ lstart, const int* __restrict__ gid,
                                                      const double2* __restrict__ unear,
                                                      const int* __restrict__ perm, int R, int nrhs, int kc,
                                                      int64_t N, const ReqTable Q) {
  extern __shared__ float2 us[];  // [kc][R]
  const int b = blockIdx.x;
  const int bo = gid ? gid[b] : b;  // the leaf's LF vector (adaptive trees)
  const int s0 = lstart[b], s1 = lstart[b + 1];
  const int g = threadIdx.x >> 4, l = threadIdx.x & 15;
  const int nq = (R - l + 15) / 16;
  for (int k0 = 0; k0 < nrhs; k0 += kc) {
    const int nk = min(kc, nrhs - k0);
    __syncthreads();  // the previous rows are consumed
    const float2* src = ulf + (int64_t(bo) * nrhs + k0) * R;
    for (int i = threadIdx.x; i < nk * R; i += L2T_BS) us[i] = src[i];
    __syncthreads();
    for (int t = s0 + g; t < s1; t += L2T_BS / 16) {
      float2 w[L2T_QMAX];
#pragma unroll
      for (int i = 0; i < L2T_QMAX; ++i)
        if (i < nq) w[i] = W[int64_t(t) * R + l + 16 * i];
      const int64_t o = perm[t];
      for (int k = 0; k < nk; ++k) {
        const float2* ur = us + k * R;
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int i = 0; i < L2T_QMAX; ++i)
          if (i < nq) cfma(acc, w[i], ur[l + 16 * i]);
#pragma unroll
        for (int m = 8; m > 0; m >>= 1) {
          acc.x += __shfl_xor(acc.x, m, 16);
          acc.y += __shfl_xor(acc.y, m, 16);
        }
        if (l == 0) {
          const int kk = k0 + k;
          const double2 nf = unear[int64_t(kk) * N + t];
          const int r = req_of(Q, kk);
          Q.u[r][int64_t(kk - Q.k0[r]) * N + o] = make_float2(float(double(acc.x) + nf.x), float(double(acc.y) + nf.y));
        }
      }
    }
  }
}

// L2T for many right-hand sides as a complex GEMM on MFMA: per leaf, the
// potentials of its targets are W (targets x R) times the leaf's incoming
// potentials (R x rhs).  A workgroup takes (leaf, 16 NCT right-hand sides,
// block of L2T_MT_TB targets); the incoming potentials of those columns are
// staged in LDS, and each wave owns 8-target row tiles.  Complex is
// interleaved real as in the near field: the lane's A entry is component
// (row parity) xor (k part) of W (negated on even rows' Im entries), its B
// entry component (k part) of the potential; products sum in float32 over
// the R ranks, as in the VALU form, and the near-field sum is added in
// float64 before the float32 store.  The potentials go to ut in tree order,
// [point][rhs] (k_permute_out_tile then writes the caller's order), so that a
// wave's stores of one target are its 16 consecutive columns.
constexpr int L2T_MT_NW = 4;                      // waves per workgroup
constexpr int L2T_MT_MAXT = 2;                    // row tiles per wave
constexpr int L2T_MT_TB = 8 * L2T_MT_NW * L2T_MT_MAXT;  // targets per workgroup (64)
template <int NCT>
__global__ void __launch_bounds__(64 * L2T_MT_NW) k_l2t_mfma(const float2* __restrict__ W,
                                                             const float2* __restrict__ ulf,
                                                             const int* __restrict__ lstart,
                                                             const int* __restrict__ gid,
                                                             const double2* __restrict__ unear, int R, int RS,
                                                             int nrhs, int64_t N, float2* __restrict__ ut) {
  constexpr int NCOL = 16 * NCT;
  extern __shared__ float2 us[];  // [NCOL][RS]: the leaf's incoming potentials of this block's columns
  const int b = blockIdx.x;
  const int bo = gid ? gid[b] : b;  // the leaf's LF vector (adaptive trees)
  const int c0 = int(blockIdx.y) * NCOL;
  const int s0 = lstart[b] + int(blockIdx.z) * L2T_MT_TB;
  const int s1 = min(lstart[b + 1], s0 + L2T_MT_TB);
  if (s0 >= s1) return;  // uniform: this target block is past the leaf's end
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int nc = min(NCOL, nrhs - c0);
  for (int e = threadIdx.x; e < NCOL * R; e += 64 * L2T_MT_NW) {
    const int c = e / R, q = e - c * R;
    us[c * RS + q] = c < nc ? ulf[(int64_t(bo) * nrhs + c0 + c) * R + q] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int ntiles = (s1 - s0 + 7) / 8;
  const int j = lane & 15, kr = lane >> 4;  // A row / B column, k index of this lane
  const int kp = kr & 1;                     // Re / Im part of k
  const bool rodd = (j & 1) != 0;
  const int comp = (rodd ? 1 : 0) ^ kp;
  const unsigned neg = (!rodd && kp) ? 0x80000000u : 0u;
#pragma unroll
  for (int i = 0; i < L2T_MT_MAXT; ++i) {
    const int rt = w + L2T_MT_NW * i;
    if (rt >= ntiles) break;
    // this lane's target row (rows past the leaf's end repeat its last target)
    const int t = min(s0 + rt * 8 + (j >> 1), s1 - 1);
    const float* wa = reinterpret_cast<const float*>(W + int64_t(t) * R + (kr >> 1)) + comp;
    const float* ub = reinterpret_cast<const float*>(us + j * RS + (kr >> 1)) + kp;
    v4f acc[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
    // MFMA step q covers ranks 2q, 2q + 1 (R is a multiple of 8)
#pragma unroll 4
    for (int q = 0; q < R / 2; ++q) {
      const float av = __uint_as_float(__float_as_uint(wa[2 * 2 * q]) ^ neg);
#pragma unroll
      for (int c = 0; c < NCT; ++c)
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, ub[2 * (2 * q + c * 16 * RS)], acc[c], 0, 0, 0);
    }
    // lane holds rows 4 kr .. 4 kr + 3 = (Re, Im) of targets 2 kr, 2 kr + 1, column j
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int col = c0 + c * 16 + j;
      if (col >= nrhs) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int tt = s0 + rt * 8 + 2 * kr + h;
        if (tt < s1) {
          const double2 nf = unear[int64_t(col) * N + tt];
          ut[int64_t(tt) * nrhs + col] =
              make_float2(float(double(acc[c][2 * h]) + nf.x), float(double(acc[c][2 * h + 1]) + nf.y));
        }
      }
    }
  }
}

__global__ void k_zero(float2* __restrict__ p, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_float2(0.f, 0.f);
}


}  // namespace

// Work chunks of a grouped GEMM for a given nrhs: (group, first column) per workgroup.
static void make_chunks(const GGemm& G, int nrhs, int NC, std::vector<int32_t>& grp, std::vector<int32_t>& col0) {
  grp.clear();
  col0.clear();
  for (int64_t g = 0; g < G.ngroups; ++g) {
    int64_t ncol = int64_t(G.v0_h[g + 1] - G.v0_h[g]) * nrhs;
    for (int64_t c = 0; c < ncol; c += NC) {
      grp.push_back(int32_t(g));
      col0.push_back(int32_t(c));
    }
  }
}

struct Launch {        // one grouped-GEMM launch prepared for the current nrhs
  const GGemm* G = nullptr;
  int nt = 4;          // 16-column tiles per workgroup
  int slices = 1;      // M-slices (grid y)
  int nw = 4;          // waves per workgroup (2 or 4)
  bool alds = false;   // operator slice staged in LDS (4-wave workgroups)
  bool m2l = false;    // translation launch (kernel name k_m2l) or tree transfer (k_transfer)
  int64_t nchunks = 0;
  DevBuf grp, col0;
};

// All M2L launches of an apply fused into one k_m2l_fused launch, when the
// tuner finds that faster than the separate launches.
struct Fused {
  int nt = 0;                 // 16-column tiles per workgroup; 0: separate launches
  int64_t nchunks = 0;
  DevBuf ps, grp, col0;       // per chunk: problem | slice << 4, group, first column
  std::vector<int64_t> yoff;  // per problem: offset (float2) of its pair outputs in the pair scratch
};

// One slot-form launch prepared for the current nrhs.
struct SlotLaunch {
  const SlotGemm* S = nullptr;
  int nt = 1;          // 16-column tiles per workgroup
  int slices = 1;      // M-slices (grid y)
  int waves = 1;       // waves per workgroup
  int pmax = 8;        // operator pairs per lane held in registers (>= K / 16)
  int cpg = 1;         // column chunks per group
  int64_t nchunks = 0;
};

// The GEMM launches of one nrhs (chunk tables and tuned shapes).
struct LaunchSet {
  std::vector<Launch> m2m, l2l, m2l;  // per HF level (pair form)
  Launch lf_m2l;
  Fused fused;
  bool slot = false;                  // slot form: M2M, and M2L + L2L per level, without pair outputs
  std::vector<SlotLaunch> up, down;   // per HF level
  SlotLaunch lf_down;
  std::vector<SlotLaunch> lfd_up, lfd_down;  // per LF level below width 1/2 (adaptive trees)
};

// The M2L problems of a plan in apply order: HF levels from the top down, then
// the leaf level (level -1).
static std::vector<const GGemm*> m2l_problems(const dfmm_plan_s& P, std::vector<int>* level = nullptr) {
  std::vector<const GGemm*> v;
  for (int e = int(P.hf.size()) - 1; e >= 0; --e)
    if (P.hf[size_t(e)].m2l.ngroups > 0) {
      v.push_back(&P.hf[size_t(e)].m2l);
      if (level) level->push_back(e);
    }
  if (P.lf.m2l.ngroups > 0) {
    v.push_back(&P.lf.m2l);
    if (level) level->push_back(-1);
  }
  return v;
}

// Pair-scratch rows (complex entries per right-hand side): the largest M2M /
// L2L launch, the largest of every launch, and the transfers' plus every M2L
// level's (fast plans: the fused M2L form).
static int64_t pair_rows_transfer(const dfmm_plan_s& P) {
  int64_t y = 0;
  for (const auto& H : P.hf) y = std::max({y, H.m2m_npairs * H.R, H.l2l_npairs * H.Rc});
  return y;
}
static int64_t pair_rows_separate(const dfmm_plan_s& P) {
  int64_t y = std::max(pair_rows_transfer(P), P.lf.npairs * P.lf.R);
  for (const auto& H : P.hf) y = std::max(y, H.npairs * H.R);
  return y;
}
static int64_t pair_rows_fused(const dfmm_plan_s& P) {
  if (P.precise) return 0;
  int64_t y = pair_rows_transfer(P);
  for (const GGemm* G : m2l_problems(P)) y += G->nvec * G->M;
  return y;
}


// A device pointer with the accessor of DevBuf.
struct WsPtr {
  void* p = nullptr;
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};
// The buffers of one apply, carved out of a workspace by ws_layout.
struct Ws {
  WsPtr fs, unear, flf, ulf, Y;
  std::vector<WsPtr> F, U;  // per HF level
};

// Plan state of the applies: the plan-owned workspace of dfmm_apply (grow-only,
// sized for the largest nrhs seen), the launch sets per nrhs and the second
// stream of the near field.  `mu` guards all of it: dfmm_apply_ws may be
// called from several threads on one plan.
struct ApplyState {
  std::mutex mu;
  DevBuf buf;                 // plan-owned workspace
  std::vector<DevBuf> retired;  // workspaces replaced after a graph capture (captured graphs hold them)
  bool captured = false;      // an apply of this plan has been captured into a graph
  std::map<int, std::unique_ptr<LaunchSet>> sets;
  // second stream for the near field (default priority) and its fork/join events
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  void ensure_side() {
    if (side) return;
    DFMM_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    DFMM_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    DFMM_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
  }
  ~ApplyState() {
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (side) (void)hipStreamDestroy(side);
  }
};

void destroy_apply_state(ApplyState* s) { delete s; }

// The hardware hands workgroups to the 8 XCDs round-robin by linear workgroup
// id, and each XCD has its own L2.  Chunks of one group read the same operator,
// so the chunk table is laid out such that the workgroups that land on one XCD
// take a contiguous range of chunks (a group's chunks share that XCD's L2).
constexpr int kXcds = 8;
static void xcd_order(std::initializer_list<std::vector<int32_t>*> cols) {
  const int64_t n = int64_t((*cols.begin())->size());
  if (n <= kXcds) return;
  int64_t start[kXcds + 1];
  start[0] = 0;
  for (int x = 0; x < kXcds; ++x) start[x + 1] = start[x] + (n - x + kXcds - 1) / kXcds;  // ids b = x mod 8
  for (std::vector<int32_t>* v : cols) {
    std::vector<int32_t> w(static_cast<size_t>(n));
    for (int64_t b = 0; b < n; ++b) w[size_t(b)] = (*v)[size_t(start[b % kXcds] + b / kXcds)];
    v->swap(w);
  }
}

// Chunks and grid for one (tile width, M-slices, waves, operator-in-LDS) choice.
static void prepare_cfg(Launch& L, const GGemm& G, int nrhs, int nt, int slices, int nw = 4, bool alds = false) {
  L.G = &G;
  L.nt = nt;
  L.nw = nw;
  L.alds = alds;
  std::vector<int32_t> grp, col0;
  make_chunks(G, nrhs, L.nt * 16, grp, col0);
  xcd_order({&grp, &col0});
  L.nchunks = int64_t(grp.size());
  L.slices = slices;
  L.grp.upload(grp);
  L.col0.upload(col0);
}

// Default choice: narrow tiles when the average group holds few columns; few
// chunks: split the M-tiles over more workgroups (at least ~4 per CU).
static void prepare(Launch& L, const GGemm& G, int nrhs) {
  double avg = G.ngroups ? double(G.nvec) * nrhs / double(G.ngroups) : 0.0;
  int nt = avg < 40.0 ? 2 : 4;
  int64_t nchunks = 0;
  for (int64_t g = 0; g < G.ngroups; ++g)
    nchunks += (int64_t(G.v0_h[g + 1] - G.v0_h[g]) * nrhs + nt * 16 - 1) / (nt * 16);
  int nM = G.M / 8;
  int max_slices = std::max(1, (nM + 3) / 4);
  int slices = 1;
  while (slices < max_slices && nchunks * slices < 1024) ++slices;
  prepare_cfg(L, G, nrhs, nt, slices);
}

static size_t gg_lds_bytes(int K, int nt) { return sizeof(float) * size_t(gg_stride(K)) * size_t(nt * 16); }
static size_t gg_lds_total(int K, int nt, int mt, bool alds) {
  return gg_lds_bytes(K, nt) + (alds ? size_t(2048) * mt * (K / 8) : 0);  // 4 waves x mt tiles
}

// dynamic LDS limit of the GEMM kernels: 160 KB less 1 KB for their static LDS
// (the column source table)
constexpr int kGgDynLds = 159 * 1024;

// M-tiles per wave of the largest group for a given number of M-slices
static int gg_mt(const GGemm& G, int slices) { return (G.M / 8 + 4 * slices - 1) / (4 * slices); }

// Raise a GEMM kernel's dynamic LDS limit, once per (kernel, device): the
// attribute belongs to the device that is current when it is set.
static void ensure_lds_limit(const void* fn) {
  static std::mutex mu;
  static std::set<std::pair<const void*, int>> done;
  int dev = 0;
  DFMM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if (done.count({fn, dev})) return;
  DFMM_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kGgDynLds));
  done.insert({fn, dev});
}

template <int NT, bool ALDS, bool ACC64, int NW, int PREC>
static void launch_nt_a(const Launch& L, int nrhs, const float2* X, float2* Y, hipStream_t st) {
  const GGemm& G = *L.G;
  const size_t lds = gg_lds_total(kpad(G.K, G.prec) * G.split, NT, gg_mt(G, L.slices), ALDS);
  auto kern = L.m2l ? &k_m2l<NT, ALDS, ACC64, NW, PREC> : &k_transfer<NT, ALDS, ACC64, NW, PREC>;
  ensure_lds_limit(reinterpret_cast<const void*>(kern));
  hipLaunchKernelGGL(kern, dim3(unsigned(L.nchunks), unsigned(L.slices)), dim3(64 * NW), lds, st,
                     G.A.as<float4>(), G.aoff.as<int64_t>(), G.aexp.as<int>(), G.gmk.as<int>(), G.M, G.K, G.split,
                     G.ops.as<int>(),
                     G.v0.as<int>(), G.vsrc.as<int>(), G.vdst.as<int>(), L.grp.as<int>(), L.col0.as<int>(), nrhs,
                     X, Y);
}

template <int NT, int PREC>
static void launch_nt_p(const Launch& L, int nrhs, const float2* X, float2* Y, hipStream_t st) {
  if (L.nw == 2) launch_nt_a<NT, false, false, 2, PREC>(L, nrhs, X, Y, st);
  else if (L.alds) launch_nt_a<NT, true, false, 4, PREC>(L, nrhs, X, Y, st);
  else launch_nt_a<NT, false, false, 4, PREC>(L, nrhs, X, Y, st);
}

template <int NT>
static void launch_nt(const Launch& L, int nrhs, const float2* X, float2* Y, hipStream_t st) {
  if (L.G->prec == DFMM_PREC_FP16X3) return launch_nt_p<NT, PREC_F16>(L, nrhs, X, Y, st);
  if (L.G->prec == DFMM_PREC_BF16X3) return launch_nt_p<NT, PREC_BF16>(L, nrhs, X, Y, st);
  if (L.nw == 2) {
    if (L.G->acc64) launch_nt_a<NT, false, true, 2, 0>(L, nrhs, X, Y, st);  // precise plans
    else launch_nt_a<NT, false, false, 2, 0>(L, nrhs, X, Y, st);
  } else {
    if (L.G->acc64) launch_nt_a<NT, false, true, 4, 0>(L, nrhs, X, Y, st);
    else if (L.alds) launch_nt_a<NT, true, false, 4, 0>(L, nrhs, X, Y, st);
    else launch_nt_a<NT, false, false, 4, 0>(L, nrhs, X, Y, st);
  }
}

static bool gg_fits(const GGemm& G, int nt, int slices, bool alds, int nw) {
  if (alds && (G.acc64 || nw != 4)) return false;
  return gg_lds_total(kpad(G.K, G.prec) * G.split, nt, gg_mt(G, slices), alds) <= size_t(kGgDynLds);
}

static void launch_gemm(const Launch& L, int nrhs, const float2* X, float2* Y, hipStream_t st) {
  if (L.nchunks == 0) return;
  const GGemm& G = *L.G;
  if (G.T != 1) throw Error{DFMM_EUNSUPPORTED, "grouped GEMM with more than one term per group"};
  if (!gg_fits(G, L.nt, L.slices, L.alds, L.nw))
    throw Error{DFMM_EUNSUPPORTED, "skeleton rank too large for the GEMM kernel"};
  if (L.nt == 4) launch_nt<4>(L, nrhs, X, Y, st);
  else if (L.nt == 3) launch_nt<3>(L, nrhs, X, Y, st);
  else if (L.nt == 2) launch_nt<2>(L, nrhs, X, Y, st);
  else launch_nt<1>(L, nrhs, X, Y, st);
}

// ---- slot-form launches ----------------------------------------------------------------
// Columns per slot-form workgroup: 32 from 17 right-hand sides on (padding one
// chunk is cheaper than a second chunk that reads every operator again).
static int slot_nt(int nrhs) { return nrhs > 16 ? 2 : 1; }

// The slot form pads its work to whole 32-column chunks and costs about 0.92 of
// the pair form per column at 32 columns (0.90-1.02 over the six serving plans
// and the K = 32 ellipsoid), so a fast float32 plan takes it where the padded
// columns still cost less: 30-32, 59-64, ... right-hand sides.
static bool slot_pays(int nrhs) {
  if (nrhs <= 16) return false;
  const int padded = (nrhs + 31) / 32 * 32;
  return 0.92 * padded <= double(nrhs);
}

static size_t slot_lds_bytes(const SlotGemm& S, int nt) {
  return size_t(2) * size_t(nt * 16) * size_t(gg_stride(S.Kmax)) * sizeof(float) +
         size_t(S.max_terms) * sizeof(int4);
}

// nt column tiles; one wave per M-tile (at most 16 per workgroup: larger ranks
// take more M-slices), and enough waves to stage a term's columns
static bool prepare_slot(SlotLaunch& L, const SlotGemm& S, int nrhs, int nt) {
  L.S = &S;
  L.nt = nt;
  const int NC = 16 * nt;
  L.cpg = (nrhs + NC - 1) / NC;
  L.nchunks = S.ngroups * L.cpg;
  const int nMall = std::max(1, S.M / 8);
  L.slices = (nMall + 15) / 16;
  L.waves = (nMall + L.slices - 1) / L.slices;
  const int need = (NC * (S.Kmax / 2) + 64 * SLOT_UB - 1) / (64 * SLOT_UB);
  L.waves = std::max(L.waves, need);
  L.pmax = S.Kmax <= 64 ? 4 : (S.Kmax <= 112 ? 7 : 8);
  return L.waves <= 16 && S.Kmax <= 128 && S.KXmax <= 128 && !S.split2 &&
         slot_lds_bytes(S, nt) <= size_t(kGgDynLds);
}

// The slot form serves fast float32 plans where it pays (DFMM_SLOT=0 forces the
// pair form, =1 the slot form wherever its launches fit).
static bool use_slot(const dfmm_plan_s& P, int nrhs) {
  if (P.leaf_max > 0) {  // adaptive trees run the LF levels in the slot form only
    const int nt = slot_nt(nrhs);
    SlotLaunch tmp;
    bool ok = prepare_slot(tmp, P.lf.down, nrhs, nt);
    for (const auto& H : P.hf) ok = ok && prepare_slot(tmp, H.up, nrhs, nt) && prepare_slot(tmp, H.down, nrhs, nt);
    for (const auto& Q : P.lfd) ok = ok && prepare_slot(tmp, Q.up, nrhs, nt) && prepare_slot(tmp, Q.down, nrhs, nt);
    if (!ok) throw Error{DFMM_EUNSUPPORTED, "an adaptive plan's slot-form launches exceed the kernel's limits"};
    return true;
  }
  if (P.precise || P.prec != DFMM_PREC_FP32) return false;
  bool want = slot_pays(nrhs);
  if (const char* e = std::getenv("DFMM_SLOT")) {
    if (e[0] == '0') return false;
    if (e[0] == '1') want = true;
  }
  if (!want) return false;
  const int nt = slot_nt(nrhs);
  SlotLaunch tmp;
  for (const auto& H : P.hf)
    if (!prepare_slot(tmp, H.up, nrhs, nt) || !prepare_slot(tmp, H.down, nrhs, nt)) return false;
  return prepare_slot(tmp, P.lf.down, nrhs, nt);
}

template <int NT, int PMAX>
static void launch_slot_t(const SlotLaunch& L, const SlotArgs& a, int nrhs, float2* Y, bool m2l, hipStream_t st) {
  const size_t lds = slot_lds_bytes(*L.S, NT);
  auto kern = m2l ? &k_m2l_slot<NT, PMAX> : &k_m2m_slot<NT, PMAX>;
  ensure_lds_limit(reinterpret_cast<const void*>(kern));
  hipLaunchKernelGGL(kern, dim3(unsigned(L.nchunks), unsigned(L.slices)), dim3(64 * L.waves), lds, st, a, nrhs, Y);
}

// kind 0: operators A0 on source vectors X0 (row stride KX0); kind 1 likewise
static void launch_slot(const SlotLaunch& L, const float4* A0, const float2* X0, int KX0, const float4* A1,
                        const float2* X1, int KX1, int nrhs, float2* Y, bool m2l, hipStream_t st,
                        const int* gdst = nullptr) {
  if (L.nchunks == 0) return;
  const SlotGemm& S = *L.S;
  SlotArgs a{S.order.as<int>(), S.t0.as<int>(), S.gm.as<int>(), S.terms.as<int4>(), A0, A1 ? A1 : A0, X0,
             X1 ? X1 : X0, KX0, X1 ? KX1 : KX0, S.M, L.cpg, gg_stride(S.Kmax) / 4, L.waves, gdst};
  if (L.nt == 2) {
    if (L.pmax == 4) launch_slot_t<2, 4>(L, a, nrhs, Y, m2l, st);
    else if (L.pmax == 7) launch_slot_t<2, 7>(L, a, nrhs, Y, m2l, st);
    else launch_slot_t<2, 8>(L, a, nrhs, Y, m2l, st);
  } else {
    if (L.pmax == 4) launch_slot_t<1, 4>(L, a, nrhs, Y, m2l, st);
    else if (L.pmax == 7) launch_slot_t<1, 7>(L, a, nrhs, Y, m2l, st);
    else launch_slot_t<1, 8>(L, a, nrhs, Y, m2l, st);
  }
}

static void prepare_slot_set(const dfmm_plan_s& P, int nrhs, LaunchSet& LS) {
  const int nt = slot_nt(nrhs);
  LS.slot = true;
  LS.up.resize(P.hf.size());
  LS.down.resize(P.hf.size());
  for (size_t e = 0; e < P.hf.size(); ++e) {
    prepare_slot(LS.up[e], P.hf[e].up, nrhs, nt);
    prepare_slot(LS.down[e], P.hf[e].down, nrhs, nt);
  }
  prepare_slot(LS.lf_down, P.lf.down, nrhs, nt);
  LS.lfd_up.resize(P.lfd.size());
  LS.lfd_down.resize(P.lfd.size());
  for (size_t k = 0; k < P.lfd.size(); ++k) {
    prepare_slot(LS.lfd_up[k], P.lfd[k].up, nrhs, nt);
    prepare_slot(LS.lfd_down[k], P.lfd[k].down, nrhs, nt);
  }
}

// ---- fused M2L launch ----------------------------------------------------------------
static bool fused_fits(const dfmm_plan_s& P, int nt) {
  const auto probs = m2l_problems(P);
  if (P.precise || probs.size() < 2 || probs.size() > size_t(kMaxProbs)) return false;
  for (const GGemm* G : probs)
    if (G->T != 1 || !gg_fits(*G, nt, 1, false, 4)) return false;
  return true;
}

static void prepare_fused(const dfmm_plan_s& P, int nrhs, int nt, Fused& F) {
  const auto probs = m2l_problems(P);
  std::vector<int32_t> ps, grp, col0;
  F.yoff.clear();
  int64_t off = pair_rows_transfer(P) * nrhs;  // past the transfers' scratch
  for (size_t i = 0; i < probs.size(); ++i) {
    std::vector<int32_t> g1, c1;
    make_chunks(*probs[i], nrhs, nt * 16, g1, c1);
    for (size_t k = 0; k < g1.size(); ++k) {
      ps.push_back(int32_t(i));
      grp.push_back(g1[k]);
      col0.push_back(c1[k]);
    }
    F.yoff.push_back(off);
    off += probs[i]->nvec * probs[i]->M * nrhs;
  }
  xcd_order({&ps, &grp, &col0});
  F.nt = nt;
  F.nchunks = int64_t(ps.size());
  F.ps.upload(ps);
  F.grp.upload(grp);
  F.col0.upload(col0);
}

template <int NT, int PREC>
static void launch_fused_t(const GgProbs& pr, size_t lds, const Fused& F, int nrhs, hipStream_t st) {
  ensure_lds_limit(reinterpret_cast<const void*>(&k_m2l_fused<NT, 4, PREC>));
  hipLaunchKernelGGL((k_m2l_fused<NT, 4, PREC>), dim3(unsigned(F.nchunks)), dim3(256), lds, st, pr, F.ps.as<int>(),
                     F.grp.as<int>(), F.col0.as<int>(), nrhs);
}

template <int PREC>
static void launch_fused_p(const GgProbs& pr, size_t lds, const Fused& F, int nrhs, hipStream_t st) {
  if (F.nt == 4) launch_fused_t<4, PREC>(pr, lds, F, nrhs, st);
  else if (F.nt == 2) launch_fused_t<2, PREC>(pr, lds, F, nrhs, st);
  else launch_fused_t<1, PREC>(pr, lds, F, nrhs, st);
}

// X of problem i: the level's outgoing potentials (the leaves' for the leaf level)
static void launch_fused(const dfmm_plan_s& P, const Ws& S, const Fused& F, int nrhs, hipStream_t st) {
  if (F.nchunks == 0) return;
  std::vector<int> level;
  const auto probs = m2l_problems(P, &level);
  GgProbs pr{};
  size_t lds = 0;
  for (size_t i = 0; i < probs.size(); ++i) {
    const GGemm& G = *probs[i];
    const float2* X = level[i] >= 0 ? S.F[size_t(level[i])].as<float2>() : S.flf.as<float2>();
    pr.p[i] = GgProb{G.A.as<float4>(), G.aoff.as<int64_t>(), G.aexp.as<int>(), G.gmk.as<int>(), G.ops.as<int>(),
                     G.v0.as<int>(), G.vsrc.as<int>(), G.vdst.as<int>(), X, S.Y.as<float2>() + F.yoff[i], G.M,
                     G.K, G.split, 1};
    lds = std::max(lds, gg_lds_total(kpad(G.K, G.prec) * G.split, F.nt, gg_mt(G, 1), false));
  }
  if (P.prec == DFMM_PREC_FP16X3) launch_fused_p<PREC_F16>(pr, lds, F, nrhs, st);
  else if (P.prec == DFMM_PREC_BF16X3) launch_fused_p<PREC_BF16>(pr, lds, F, nrhs, st);
  else launch_fused_p<0>(pr, lds, F, nrhs, st);
}

// Tile autotuner: time every (tile width, M-slices, waves per workgroup,
// operator-in-LDS) candidate of one launch on the apply stream (its output goes
// to the pair scratch Y only) and keep the fastest.  Runs once per plan and nrhs.
static void autotune(Launch& L, const GGemm& G, int nrhs, const float2* X, float2* Y, hipStream_t st) {
  prepare(L, G, nrhs);
  if (G.ngroups == 0) return;
  const char* env = std::getenv("DFMM_AUTOTUNE");
  if (env && env[0] == '0') return;
  const int nM = G.M / 8;
  hipEvent_t e0, e1;
  DFMM_HIP(hipEventCreate(&e0));
  DFMM_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int best_nt = L.nt, best_sl = L.slices, best_nw = L.nw;
  bool best_alds = false;
  for (int nw : {4, 2})
  for (int alds = 0; alds < 2; ++alds)
  for (int nt : {1, 2, 3, 4})
    for (int sl = 1; sl <= std::min(std::max(1, (nM + nw - 1) / nw), 4); ++sl) {
      if (!gg_fits(G, nt, sl, alds != 0, nw)) continue;
      prepare_cfg(L, G, nrhs, nt, sl, nw, alds != 0);
      launch_gemm(L, nrhs, X, Y, st);  // warm-up
      DFMM_HIP(hipEventRecord(e0, st));
      for (int i = 0; i < 3; ++i) launch_gemm(L, nrhs, X, Y, st);
      DFMM_HIP(hipEventRecord(e1, st));
      DFMM_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      DFMM_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_nt = nt;
        best_sl = sl;
        best_nw = nw;
        best_alds = alds != 0;
      }
    }
  DFMM_HIP(hipEventDestroy(e0));
  DFMM_HIP(hipEventDestroy(e1));
  prepare_cfg(L, G, nrhs, best_nt, best_sl, best_nw, best_alds);
}

// The sizes the workspace of a plan depends on.
static WsShape ws_shape(const dfmm_plan_s& P) {
  WsShape z;
  z.N = P.N;
  z.nleaf = P.nlfbox;
  z.Rlf = P.lf.R;
  for (const auto& H : P.hf) {
    z.nout.push_back(H.nout);
    z.nin.push_back(H.nin);
    z.R.push_back(H.R);
  }
  // separate launches reuse one scratch; the fused form keeps the transfers'
  // scratch and every M2L level's pair outputs side by side
  z.pair_rows = std::max(pair_rows_separate(P), pair_rows_fused(P));
  return z;
}

// Layout for nrhs: with pair scratch unless the launch set of nrhs (the one
// that exists, else the one that would be made) takes the slot form.  The
// caller holds the plan's apply lock if the plan has an apply state.
static WsLayout plan_layout(const dfmm_plan_s& P, int nrhs) {
  bool slot = use_slot(P, nrhs);
  if (P.ws) {
    auto it = P.ws->sets.find(nrhs);
    if (it != P.ws->sets.end()) slot = it->second->slot;
  }
  return ws_layout(ws_shape(P), nrhs, !slot);
}

size_t workspace_bytes(const dfmm_plan_s& P, int nrhs) {
  if (P.prec == DFMM_PREC_FP64) return ws_layout(ws_shape64(P), nrhs, false, 16).total;
  if (!P.ws) return plan_layout(P, nrhs).total;
  std::lock_guard<std::mutex> lock(P.ws->mu);
  return plan_layout(P, nrhs).total;
}

static Ws carve(const WsLayout& L, void* base) {
  char* b = static_cast<char*>(base);
  Ws W;
  W.fs.p = b + L.fs;
  W.unear.p = b + L.unear;
  W.flf.p = b + L.flf;
  W.ulf.p = b + L.ulf;
  W.Y.p = b + L.Y;
  for (size_t o : L.F) W.F.push_back(WsPtr{b + o});
  for (size_t o : L.U) W.U.push_back(WsPtr{b + o});
  return W;
}

// Grow the plan-owned workspace to `bytes` (the launch sets hold no buffer
// addresses, so they stay valid).  The old buffer is freed once earlier applies
// are done with it, or kept until the plan is destroyed if an apply has been
// captured into a graph (the graph still addresses it).
static void ensure_workspace(ApplyState& S, size_t bytes) {
  if (S.buf.p && S.buf.bytes >= bytes) return;
  DFMM_HIP(hipDeviceSynchronize());  // earlier applies may still use the old buffer
  if (S.captured && S.buf.p) S.retired.push_back(std::move(S.buf));
  S.buf.alloc(bytes);
}

// ---- tuning record: the chosen (tile width, M-slices, LDS operator) per launch,
// kept in the plan's cache directory under a key of the launch shapes, nrhs and
// the device, so that later plans of the same shape skip the trial launches.
static void fnv(uint64_t& h, const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
}

static std::string tune_path(const dfmm_plan_s& P, const std::vector<const GGemm*>& gs, int nrhs) {
  if (P.tune_dir.empty()) return std::string();
  uint64_t h = 1469598103934665603ull;
  hipDeviceProp_t prop;
  DFMM_HIP(hipGetDeviceProperties(&prop, P.device));
  fnv(h, prop.gcnArchName, std::strlen(prop.gcnArchName));
  fnv(h, &prop.multiProcessorCount, sizeof(prop.multiProcessorCount));
  fnv(h, &nrhs, sizeof(nrhs));
  for (const GGemm* g : gs) {
    const int64_t dims[8] = {g->M, g->K, g->T, g->ngroups, g->nvec, g->split, int64_t(g->acc64), g->prec};
    fnv(h, dims, sizeof(dims));
    fnv(h, g->v0_h.data(), g->v0_h.size() * sizeof(int32_t));
  }
  char name[64];
  std::snprintf(name, sizeof(name), "/dfmm_tune_%016llx.txt", static_cast<unsigned long long>(h));
  return P.tune_dir + name;
}

static bool load_tuning(const std::string& path, std::vector<Launch*>& ls, const std::vector<const GGemm*>& gs,
                        int nrhs, int* fused_nt) {
  if (path.empty()) return false;
  FILE* fp = std::fopen(path.c_str(), "r");
  if (!fp) return false;
  int n = 0;
  bool ok = std::fscanf(fp, "dfmm-tune 4 %d", &n) == 1 && n == int(ls.size());
  std::vector<int> v(4 * size_t(std::max(n, 0)));
  for (int i = 0; ok && i < n; ++i) {
    int* c = &v[4 * size_t(i)];  // tile width, M-slices, operator in LDS, waves
    ok = std::fscanf(fp, "%d %d %d %d", &c[0], &c[1], &c[2], &c[3]) == 4;
    ok = ok && c[0] >= 1 && c[0] <= 4 && c[1] >= 1 && c[1] <= 64 && (c[3] == 2 || c[3] == 4);
  }
  ok = ok && std::fscanf(fp, " fused %d", fused_nt) == 1 &&
       (*fused_nt == 0 || *fused_nt == 1 || *fused_nt == 2 || *fused_nt == 4);
  std::fclose(fp);
  if (!ok) return false;
  for (int i = 0; i < n; ++i) {
    const int* c = &v[4 * size_t(i)];
    if (!gg_fits(*gs[i], c[0], c[1], c[2] != 0, c[3])) return false;
    prepare_cfg(*ls[i], *gs[i], nrhs, c[0], c[1], c[3], c[2] != 0);
  }
  return true;
}

static void save_tuning(const std::string& path, const std::vector<Launch*>& ls, int fused_nt) {
  if (path.empty()) return;
  const std::string tmp = path + ".tmp";
  FILE* fp = std::fopen(tmp.c_str(), "w");
  if (!fp) return;  // the record is an optimisation only
  std::fprintf(fp, "dfmm-tune 4 %d\n", int(ls.size()));
  for (const Launch* L : ls) std::fprintf(fp, "%d %d %d %d\n", L->nt, L->slices, L->alds ? 1 : 0, L->nw);
  std::fprintf(fp, "fused %d\n", fused_nt);
  const bool ok = std::fclose(fp) == 0;
  if (ok) std::rename(tmp.c_str(), path.c_str());
}

// Fused M2L or separate launches: time the tuned separate M2L launches and the
// fused launch at each tile width, each with the reductions of the pair outputs
// (the fused form reduces them after all levels, when they are no longer in
// cache), 3 runs each on the apply stream, and keep the faster form.  The timed
// reductions add into the incoming potentials, which every apply overwrites
// or clears before it adds to them.
static void tune_fused(const dfmm_plan_s& P, int nrhs, const Ws& S, LaunchSet& LS, hipStream_t st) {
  LS.fused.nt = 0;
  bool any = false;
  for (int nt : {1, 2, 4}) any = any || fused_fits(P, nt);
  if (!any) return;
  std::vector<int> level;
  const auto probs = m2l_problems(P, &level);
  hipEvent_t e0, e1;
  DFMM_HIP(hipEventCreate(&e0));
  DFMM_HIP(hipEventCreate(&e1));
  auto timed = [&](const std::function<void()>& run) {
    run();  // warm-up
    DFMM_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < 3; ++r) run();
    DFMM_HIP(hipEventRecord(e1, st));
    DFMM_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    DFMM_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ms;
  };
  auto reduce = [&](size_t i, const float2* Yp) {
    if (level[i] >= 0) {
      const HFLevel& H = P.hf[size_t(level[i])];
      const int RN = H.R * nrhs;
      hipLaunchKernelGGL(k_reduce, dim3(nblocks(H.nin * RN, 256)), dim3(256), 0, st, H.red_start.as<int>(),
                         H.red_idx.as<int>(), Yp, H.nin, RN, 1, S.U[size_t(level[i])].as<float2>());
    } else {
      const int RN = P.lf.R * nrhs;
      hipLaunchKernelGGL(k_reduce, dim3(nblocks(P.lf.nbox * RN, 256)), dim3(256), 0, st,
                         P.lf.red_start.as<int>(), P.lf.red_idx.as<int>(), Yp, P.lf.nbox, RN, 1,
                         S.ulf.as<float2>());
    }
  };
  const float t_sep = timed([&]() {
    for (size_t i = 0; i < probs.size(); ++i) {
      const Launch& L = level[i] >= 0 ? LS.m2l[size_t(level[i])] : LS.lf_m2l;
      const float2* X = level[i] >= 0 ? S.F[size_t(level[i])].as<float2>() : S.flf.as<float2>();
      launch_gemm(L, nrhs, X, S.Y.as<float2>(), st);
      reduce(i, S.Y.as<float2>());
    }
  });
  float best = t_sep;
  int best_nt = 0;
  for (int nt : {1, 2, 4}) {
    if (!fused_fits(P, nt)) continue;
    prepare_fused(P, nrhs, nt, LS.fused);
    const float t = timed([&]() {
      launch_fused(P, S, LS.fused, nrhs, st);
      for (size_t i = 0; i < probs.size(); ++i) reduce(i, S.Y.as<float2>() + LS.fused.yoff[i]);
    });
    if (t < best) {
      best = t;
      best_nt = nt;
    }
  }
  DFMM_HIP(hipEventDestroy(e0));
  DFMM_HIP(hipEventDestroy(e1));
  if (best_nt > 0) prepare_fused(P, nrhs, best_nt, LS.fused);
  else LS.fused = Fused();
}

// Tune the GEMM launches of nrhs right-hand sides on the apply stream.
static void tune_launches(dfmm_plan_s& P, int nrhs, const Ws& S, LaunchSet& LS, hipStream_t st) {
  float2* Y = S.Y.as<float2>();
  std::vector<Launch*> ls;
  std::vector<const GGemm*> gs;
  std::vector<const float2*> xs;
  LS.m2m.resize(P.hf.size());
  LS.l2l.resize(P.hf.size());
  LS.m2l.resize(P.hf.size());
  for (size_t e = 0; e < P.hf.size(); ++e) {
    const float2* Fc = e == 0 ? S.flf.as<float2>() : S.F[e - 1].as<float2>();
    ls.insert(ls.end(), {&LS.m2m[e], &LS.l2l[e], &LS.m2l[e]});
    gs.insert(gs.end(), {&P.hf[e].m2m, &P.hf[e].l2l, &P.hf[e].m2l});
    xs.insert(xs.end(), {Fc, S.U[e].as<float2>(), S.F[e].as<float2>()});
    LS.m2l[e].m2l = true;
  }
  ls.push_back(&LS.lf_m2l);
  gs.push_back(&P.lf.m2l);
  xs.push_back(S.flf.as<float2>());
  LS.lf_m2l.m2l = true;
  const std::string path = tune_path(P, gs, nrhs);
  int fused_nt = 0;
  if (load_tuning(path, ls, gs, nrhs, &fused_nt)) {
    if (fused_nt > 0 && fused_fits(P, fused_nt)) prepare_fused(P, nrhs, fused_nt, LS.fused);
  } else {
    for (size_t i = 0; i < ls.size(); ++i) autotune(*ls[i], *gs[i], nrhs, xs[i], Y, st);
    const char* env = std::getenv("DFMM_AUTOTUNE");
    const bool tune = !(env && env[0] == '0');
    if (tune) tune_fused(P, nrhs, S, LS, st);
    if (tune) save_tuning(path, ls, LS.fused.nt);
  }
  // DFMM_FUSED=0 / 1 forces the separate / fused M2L form (tests of both)
  if (const char* f = std::getenv("DFMM_FUSED")) {
    if (f[0] == '0') LS.fused = Fused();
    else if (f[0] == '1' && LS.fused.nt == 0 && fused_fits(P, 2)) prepare_fused(P, nrhs, 2, LS.fused);
  }
}

// A launch set for nrhs that is not a power of two takes the tuned shapes of
// the largest power of two below it (only its chunk tables are built), so a
// request loop with many batch sizes tunes at most log2(max nrhs) + 1 of them.
static void inherit_launches(dfmm_plan_s& P, int nrhs, const LaunchSet& from, LaunchSet& LS) {
  LS.m2m.resize(P.hf.size());
  LS.l2l.resize(P.hf.size());
  LS.m2l.resize(P.hf.size());
  auto take = [&](Launch& L, const Launch& F, const GGemm& G) {
    prepare_cfg(L, G, nrhs, F.nt, F.slices, F.nw, F.alds);
    L.m2l = F.m2l;
  };
  for (size_t e = 0; e < P.hf.size(); ++e) {
    take(LS.m2m[e], from.m2m[e], P.hf[e].m2m);
    take(LS.l2l[e], from.l2l[e], P.hf[e].l2l);
    take(LS.m2l[e], from.m2l[e], P.hf[e].m2l);
  }
  take(LS.lf_m2l, from.lf_m2l, P.lf.m2l);
  if (from.fused.nt > 0) prepare_fused(P, nrhs, from.fused.nt, LS.fused);
}

static LaunchSet& launch_set(dfmm_plan_s& P, ApplyState& AS, const Ws& S, int nrhs, hipStream_t st) {
  auto it = AS.sets.find(nrhs);
  if (it != AS.sets.end()) return *it->second;
  std::unique_ptr<LaunchSet> ls(new LaunchSet());
  if (use_slot(P, nrhs)) {
    prepare_slot_set(P, nrhs, *ls);
  } else if ((nrhs & (nrhs - 1)) == 0) {
    tune_launches(P, nrhs, S, *ls, st);
  } else {
    // the pair form's shapes from the largest power of two below whose set is
    // in the pair form (1 always is)
    int p2 = 1;
    while (2 * p2 < nrhs) p2 *= 2;
    while (p2 > 1 && use_slot(P, p2)) p2 /= 2;
    const LaunchSet& from = launch_set(P, AS, S, p2, st);
    if (from.slot) tune_launches(P, nrhs, S, *ls, st);  // no pair-form shapes below
    else inherit_launches(P, nrhs, from, *ls);
  }
  return *AS.sets.emplace(nrhs, std::move(ls)).first->second;
}

void run_apply(dfmm_plan_s& P, const ReqTable& R, int nrhs, hipStream_t st, void* ws, size_t ws_bytes,
               bool existing_only) {
  // under stream capture only launches, event records and event waits may be
  // issued: the workspace, the tuning and the side stream must already exist
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  DFMM_HIP(hipStreamIsCapturing(st, &cap));
  const bool capturing = cap != hipStreamCaptureStatusNone;
  const bool own = ws == nullptr;  // plan-owned workspace (dfmm_apply) or the caller's
  if (!P.ws) {
    if (capturing || existing_only)
      throw Error{DFMM_EINVAL, "this apply needs an earlier apply with the same nrhs on the plan"};
    P.ws = new ApplyState();
  }
  ApplyState& AS = *P.ws;
  std::unique_lock<std::mutex> lock(AS.mu);
  if (P.prec == DFMM_PREC_FP64) {  // the float64 pass: its own kernels, everything on st
    if (R.n != 1 || existing_only) throw Error{DFMM_EUNSUPPORTED, "float64 plans take dfmm_apply or dfmm_apply_ws"};
    const size_t need = ws_layout(ws_shape64(P), nrhs, false, 16).total;
    if (!own && ws_bytes < need)
      throw Error{DFMM_EINVAL, "workspace of " + std::to_string(ws_bytes) + " bytes; this apply needs " +
                                   std::to_string(need)};
    if (own) {
      hipStreamCaptureStatus c2 = hipStreamCaptureStatusNone;
      DFMM_HIP(hipStreamIsCapturing(st, &c2));
      if (c2 != hipStreamCaptureStatusNone && (!AS.buf.p || AS.buf.bytes < need))
        throw Error{DFMM_EINVAL, "dfmm_apply under stream capture needs an earlier uncaptured apply"};
      if (c2 != hipStreamCaptureStatusNone) AS.captured = true;
      ensure_workspace(AS, need);
    } else {
      lock.unlock();
    }
    run_apply64(P, reinterpret_cast<const double2*>(R.f[0]), reinterpret_cast<double2*>(R.u[0]), nrhs, st,
                own ? AS.buf.p : ws);
    return;
  }
  const WsLayout L = plan_layout(P, nrhs);
  if (!own && ws_bytes < L.total)
    throw Error{DFMM_EINVAL, "workspace of " + std::to_string(ws_bytes) + " bytes; this apply needs " +
                                 std::to_string(L.total)};
  const bool have_set = AS.sets.count(nrhs) != 0;
  if ((capturing || existing_only) && (!have_set || (own && (!AS.buf.p || AS.buf.bytes < L.total || !AS.side))))
    throw Error{DFMM_EINVAL, "dfmm_apply under stream capture (or without allocation) needs an earlier "
                             "uncaptured apply with the same nrhs"};
  if (own) ensure_workspace(AS, L.total);
  const Ws S = carve(L, own ? AS.buf.p : ws);
  LaunchSet& LS = launch_set(P, AS, S, nrhs, st);
  if (capturing) AS.captured = true;
  // the launch set is immutable from here; applies on caller workspaces run
  // concurrently (the stage timer and the second stream belong to dfmm_apply)
  if (!own) lock.unlock();
  const int64_t N = P.N;
  const int64_t nleaf = P.lf.nleaf;
  const int Rl = P.lf.R;
  const int e_top = int(P.hf.size()) - 1;
  const int* gid = P.leaf_gid.p ? P.leaf_gid.as<int>() : nullptr;  // leaf -> LF vector (adaptive)
  StageTimer* tm = own ? P.timer : nullptr;
  if (tm && (capturing || !tm->begin_apply(st))) tm = nullptr;  // no stage events inside a graph
  auto mark = [&](int stage) {
    if (tm) tm->mark(stage, st);
  };
  // the tiled permutations pay from 16 rhs; the L2T of as many writes tree order
  const bool tiled = nrhs >= 16;
  const dim3 pt_grid(nblocks(N, PT_P), unsigned((nrhs + PT_C - 1) / PT_C));
  if (tiled)
    hipLaunchKernelGGL(k_permute_in_tile, pt_grid, dim3(PT_BS), 0, st, R, S.fs.as<float2>(), P.iperm_d.as<int>(), N,
                       nrhs);
  else
    hipLaunchKernelGGL(k_permute_in, dim3(nblocks(N * nrhs, 256)), dim3(256), 0, st, R, S.fs.as<float2>(),
                       P.perm_d.as<int>(), N, nrhs);
  mark(ST_PERMUTE);
  // the near field needs only the permuted densities: it runs on the plan's
  // second stream while the far-field passes run on st (on st itself when the
  // workspace is the caller's)
  hipStream_t nst = st;
  if (own) {
    AS.ensure_side();
    DFMM_HIP(hipEventRecord(AS.fork, st));
    DFMM_HIP(hipStreamWaitEvent(AS.side, AS.fork, 0));
    nst = AS.side;
    if (tm) tm->side_begin(nst);
  }
#define DFMM_NEAR(PREC, RCV)                                                                                   \
  hipLaunchKernelGGL((k_leaf_eval<PREC, RCV>), dim3(unsigned(nleaf)), dim3(EV_BS), 0, nst, P.pthi.as<float4>(), \
                     P.ptlo.as<float4>(), P.leaf_start.as<int>(), P.near_start.as<int>(), P.near_src.as<int>(),    \
                     S.fs.as<float2>(), nrhs, N, S.unear.as<double2>())
  if (P.precise) {
    if (nrhs == 1) DFMM_NEAR(true, 1); else DFMM_NEAR(true, 8);
  } else if (nrhs >= kNearMfmaMinRhs) {
    const dim3 grid(unsigned(nleaf), unsigned((nrhs + 31) / 32), unsigned((P.max_leaf_pts + NM_TB - 1) / NM_TB));
    const dim3 grid1(unsigned(nleaf), unsigned((nrhs + 15) / 16), grid.z);
#define DFMM_NEARM(NCT, PR, G)                                                                                   \
  hipLaunchKernelGGL((k_near_mfma<NCT, PR>), G, dim3(64 * NM_NW), 0, nst, P.pthi.as<float4>(),               \
                     P.ptlo.as<float4>(), P.leaf_start.as<int>(), P.near_start.as<int>(), P.near_src.as<int>(),   \
                     S.fs.as<float2>(), nrhs, N, S.unear.as<double2>())
    if (P.prec == DFMM_PREC_FP16X3) {
      if (nrhs <= 16) DFMM_NEARM(1, PREC_F16, grid1); else DFMM_NEARM(2, PREC_F16, grid);
    } else if (P.prec == DFMM_PREC_BF16X3) {
      if (nrhs <= 16) DFMM_NEARM(1, PREC_BF16, grid1); else DFMM_NEARM(2, PREC_BF16, grid);
    } else {
      if (nrhs <= 16) DFMM_NEARM(1, 0, grid1); else DFMM_NEARM(2, 0, grid);
    }
#undef DFMM_NEARM
  } else {
    if (nrhs == 1) DFMM_NEAR(false, 1); else DFMM_NEAR(false, 8);
  }
#undef DFMM_NEAR
  if (own) {
    if (tm) tm->side_mark(ST_NEAR, nst);
    DFMM_HIP(hipEventRecord(AS.join, nst));
  } else {
    mark(ST_NEAR);
  }
  if (nrhs == 1)
    hipLaunchKernelGGL(k_s2m<1>, dim3(unsigned(nleaf)), dim3(S2M_BS), 0, st, P.leaf_start.as<int>(),
                       P.lf.V.as<float2>(), S.fs.as<float2>(), Rl, nrhs, gid, S.flf.as<float2>());
  else if (nrhs < 24)
    hipLaunchKernelGGL(k_s2m<8>, dim3(unsigned(nleaf)), dim3(S2M_BS), 0, st, P.leaf_start.as<int>(),
                       P.lf.V.as<float2>(), S.fs.as<float2>(), Rl, nrhs, gid, S.flf.as<float2>());
  else if (size_t(P.max_leaf_pts + 1) * 32 * sizeof(float2) > size_t(kGgDynLds) || Rl % 8 != 0)
    // one pass over the weights for up to 32 right-hand sides
    hipLaunchKernelGGL(k_s2m<32>, dim3(unsigned(nleaf)), dim3(S2M_BS), 0, st, P.leaf_start.as<int>(),
                       P.lf.V.as<float2>(), S.fs.as<float2>(), Rl, nrhs, gid, S.flf.as<float2>());
  else {  // k_s2m_mfma: the leaf's densities of 32 columns in LDS
    const size_t lds = sizeof(float2) * size_t(32) * size_t((P.max_leaf_pts + 1) & ~1);
    ensure_lds_limit(reinterpret_cast<const void*>(&k_s2m_mfma<2>));
    hipLaunchKernelGGL(k_s2m_mfma<2>, dim3(unsigned(nleaf), unsigned((nrhs + 31) / 32)), dim3(64 * S2M_MT_NW),
                       lds, st, P.leaf_start.as<int>(), P.lf.V.as<float2>(), S.fs.as<float2>(), Rl, nrhs, gid,
                       S.flf.as<float2>());
  }
  mark(ST_S2M);
  if (LS.slot) {
    // slot form: M2M fine to coarse; then per level, coarse to fine, one launch
    // sums the M2L pairs and the L2L terms of every incoming slot.  Adaptive
    // trees first run LF-M2M from the deepest LF level up to width 1/2.
    for (int k = int(P.lfd.size()) - 1; k >= 0; --k) {
      const LFDeep& Q = P.lfd[size_t(k)];
      launch_slot(LS.lfd_up[size_t(k)], Q.m2m.A.as<float4>(), S.flf.as<float2>(), Rl, nullptr, nullptr, 0, nrhs,
                  S.flf.as<float2>(), false, st, Q.up_dst.as<int>());
      mark(ST_M2M);
    }
    for (int e = 0; e <= e_top; ++e) {
      const float2* Fc = e == 0 ? S.flf.as<float2>() : S.F[e - 1].as<float2>();
      const int KC = e == 0 ? Rl : P.hf[e - 1].R;
      launch_slot(LS.up[e], P.hf[e].m2m.A.as<float4>(), Fc, KC, nullptr, nullptr, 0, nrhs,
                  S.F[e].as<float2>(), false, st);
      mark(ST_M2M);
    }
    for (int e = e_top; e >= 0; --e) {
      const HFLevel& H = P.hf[e];
      const bool par = e < e_top;
      launch_slot(LS.down[e], H.m2l.A.as<float4>(), S.F[e].as<float2>(), H.R,
                  par ? P.hf[e + 1].l2l.A.as<float4>() : nullptr, par ? S.U[e + 1].as<float2>() : nullptr,
                  par ? P.hf[e + 1].R : 0, nrhs, S.U[e].as<float2>(), true, st);
      mark(ST_M2L);
    }
    launch_slot(LS.lf_down, P.lf.m2l.A.as<float4>(), S.flf.as<float2>(), Rl,
                e_top >= 0 ? P.hf[0].l2l.A.as<float4>() : nullptr, e_top >= 0 ? S.U[0].as<float2>() : nullptr,
                e_top >= 0 ? P.hf[0].R : 0, nrhs, S.ulf.as<float2>(), true, st);
    mark(ST_LF_M2L);
    // adaptive trees: LF-M2L + LF-L2L of each deeper level into its boxes' LF vectors
    for (size_t k = 0; k < P.lfd.size(); ++k) {
      const LFDeep& Q = P.lfd[k];
      launch_slot(LS.lfd_down[k], Q.m2l.A.as<float4>(), S.flf.as<float2>(), Rl, Q.l2l.A.as<float4>(),
                  S.ulf.as<float2>(), Rl, nrhs, S.ulf.as<float2>() + Q.base * nrhs * Rl, true, st);
      mark(ST_LF_M2L);
    }
  }
  // HF-M2M, fine to coarse
  for (int e = 0; e <= e_top && !LS.slot; ++e) {
    HFLevel& H = P.hf[e];
    const float2* Fc = e == 0 ? S.flf.as<float2>() : S.F[e - 1].as<float2>();
    launch_gemm(LS.m2m[e], nrhs, Fc, S.Y.as<float2>(), st);
    int RN = H.R * nrhs;
    if (H.nout > 0)
      hipLaunchKernelGGL(k_reduce, dim3(nblocks(H.nout * RN, 256)), dim3(256), 0, st, H.m2m_rs.as<int>(),
                         H.m2m_ri.as<int>(), S.Y.as<float2>(), H.nout, RN, 0, S.F[e].as<float2>());
    mark(ST_M2M);
  }
  // HF-M2L (+ reduction) then HF-L2L, coarse to fine.  Below the top level the
  // M2L sums are added to what L2L wrote; at the top level the reduction
  // writes every incoming slot itself, so the slots need clearing only when
  // that level has no M2L pairs.
  const bool top_m2l = e_top >= 0 && !LS.slot && LS.m2l[e_top].nchunks > 0;
  if (e_top >= 0 && !top_m2l && !LS.slot) {
    HFLevel& H = P.hf[e_top];
    int64_t n = std::max<int64_t>(1, H.nin) * H.R * nrhs;
    hipLaunchKernelGGL(k_zero, dim3(nblocks(n, 256)), dim3(256), 0, st, S.U[e_top].as<float2>(), n);
    mark(ST_ZERO);
  }
  // fused form: every level's M2L in one launch, each into its own pair scratch
  const bool fused = !LS.slot && LS.fused.nt > 0;
  std::vector<const float2*> ym2l(P.hf.size() + 1, S.Y.as<float2>());  // pair outputs per level (last: LF)
  if (fused) {
    std::vector<int> level;
    const auto probs = m2l_problems(P, &level);
    for (size_t i = 0; i < probs.size(); ++i)
      ym2l[level[i] >= 0 ? size_t(level[i]) : P.hf.size()] = S.Y.as<float2>() + LS.fused.yoff[i];
    launch_fused(P, S, LS.fused, nrhs, st);
    mark(ST_M2L);
  }
  for (int e = e_top; e >= 0 && !LS.slot; --e) {
    HFLevel& H = P.hf[e];
    if (LS.m2l[e].nchunks > 0) {
      if (!fused) {
        launch_gemm(LS.m2l[e], nrhs, S.F[e].as<float2>(), S.Y.as<float2>(), st);
        mark(ST_M2L);
      }
      int RN = H.R * nrhs;
      hipLaunchKernelGGL(k_reduce, dim3(nblocks(H.nin * RN, 256)), dim3(256), 0, st, H.red_start.as<int>(),
                         H.red_idx.as<int>(), ym2l[size_t(e)], H.nin, RN, e == e_top ? 0 : 1,
                         S.U[e].as<float2>());
      mark(ST_REDUCE);
    }
    float2* Uc = e == 0 ? S.ulf.as<float2>() : S.U[e - 1].as<float2>();
    launch_gemm(LS.l2l[e], nrhs, S.U[e].as<float2>(), S.Y.as<float2>(), st);
    int RNc = H.Rc * nrhs;
    if (H.nchild_in > 0)
      hipLaunchKernelGGL(k_reduce, dim3(nblocks(H.nchild_in * RNc, 256)), dim3(256), 0, st, H.l2l_rs.as<int>(),
                         H.l2l_ri.as<int>(), S.Y.as<float2>(), H.nchild_in, RNc, 0, Uc);
    mark(ST_L2L);
  }
  // without HF levels nothing has written the LF incoming slots: the LF
  // reduction writes them itself, or they are cleared if it does not run
  if (e_top < 0 && !LS.slot && LS.lf_m2l.nchunks == 0) {
    int64_t n = P.lf.nbox * Rl * nrhs;
    hipLaunchKernelGGL(k_zero, dim3(nblocks(n, 256)), dim3(256), 0, st, S.ulf.as<float2>(), n);
    mark(ST_ZERO);
  }
  // LF-M2L
  if (!LS.slot && LS.lf_m2l.nchunks > 0) {
    if (!fused) {
      launch_gemm(LS.lf_m2l, nrhs, S.flf.as<float2>(), S.Y.as<float2>(), st);
      mark(ST_LF_M2L);
    }
    int RN = Rl * nrhs;
    hipLaunchKernelGGL(k_reduce, dim3(nblocks(P.lf.nbox * RN, 256)), dim3(256), 0, st, P.lf.red_start.as<int>(),
                       P.lf.red_idx.as<int>(), ym2l[P.hf.size()], P.lf.nbox, RN, e_top >= 0 ? 1 : 0,
                       S.ulf.as<float2>());
    mark(ST_LF_REDUCE);
  }
  if (own) DFMM_HIP(hipStreamWaitEvent(st, AS.join, 0));
  if (Rl > 16 * L2T_QMAX || Rl % 2 != 0) throw Error{DFMM_EUNSUPPORTED, "leaf skeleton rank unsupported by L2T"};
  if (tiled) {
    // k_l2t_mfma: the staged column stride RS is odd (in float2), which spreads
    // the 16 columns a wave reads at one rank over the LDS banks
    const int RS = Rl | 1;
    const int nt = nrhs > 16 ? 2 : 1;
    const size_t lds = sizeof(float2) * size_t(16 * nt) * size_t(RS);
    const dim3 grid(unsigned(nleaf), unsigned((nrhs + 16 * nt - 1) / (16 * nt)),
                    unsigned((P.max_leaf_pts + L2T_MT_TB - 1) / L2T_MT_TB));
    auto kern = nt == 2 ? &k_l2t_mfma<2> : &k_l2t_mfma<1>;
    ensure_lds_limit(reinterpret_cast<const void*>(kern));
    // the potentials in tree order go to fs: the densities there are dead once
    // S2M and the near field (joined above) have run
    hipLaunchKernelGGL(kern, grid, dim3(64 * L2T_MT_NW), lds, st, P.lf.W.as<float2>(), S.ulf.as<float2>(),
                       P.leaf_start.as<int>(), gid, S.unear.as<double2>(), Rl, RS, nrhs, N, S.fs.as<float2>());
    hipLaunchKernelGGL(k_permute_out_tile, pt_grid, dim3(PT_BS), 0, st, R, S.fs.as<const float2>(),
                       P.iperm_d.as<int>(), N, nrhs);
  } else if (nrhs >= 4) {
    const int kc = std::min(nrhs, std::max(1, int((48 << 10) / (sizeof(float2) * Rl))));
    hipLaunchKernelGGL(k_l2t_leaf, dim3(unsigned(nleaf)), dim3(L2T_BS), sizeof(float2) * size_t(kc) * Rl, st,
                       P.lf.W.as<float2>(), S.ulf.as<float2>(), P.leaf_start.as<int>(), gid, S.unear.as<double2>(),
                       P.perm_d.as<int>(), Rl, nrhs, kc, N, R);
  } else {
    hipLaunchKernelGGL(k_l2t, dim3(nblocks(N * 16, L2T_BS)), dim3(L2T_BS), 0, st, P.lf.W.as<float2>(),
                       S.ulf.as<float2>(), P.leaf_of.as<int>(), S.unear.as<double2>(), P.perm_d.as<int>(), Rl, nrhs,
                       N, R);
  }
  mark(ST_LEAF);
  DFMM_HIP(hipGetLastError());
}

// ---- applies without allocation -------------------------------------------------------
// The workspace of dfmm_apply_noalloc: a static device array, one per GPU the
// library runs on, held until the process ends.  In host code `scratch` names a
// host-side stand-in, not the device memory: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static void* scratch_ptr(int device) {
  static std::mutex mu;
  static std::map<int, void*> ptr;  // device ordinal -> address of that device's array
  std::lock_guard<std::mutex> lock(mu);
  auto it = ptr.find(device);
  if (it != ptr.end()) return it->second;
  void* p = nullptr;
  DFMM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error{DFMM_EDEVICE, "no device address for the static workspace"};
  ptr.emplace(device, p);
  return p;
}

void run_apply_noalloc(dfmm_plan_s& P, const ReqTable& R, int nrhs, hipStream_t st) {
  const size_t need = workspace_bytes(P, nrhs);
  if (need > kNoAllocBytes)
    throw Error{DFMM_EINVAL, "this apply needs a workspace of " + std::to_string(need) +
                                 " bytes; the static workspace holds " + std::to_string(kNoAllocBytes)};
  run_apply(P, R, nrhs, st, scratch_ptr(P.device), kNoAllocBytes, true);
}

// ---- plan-time leaf weights ---------------------------------------------------------
void build_leaf_weights(dfmm_plan_s& P, const std::vector<double>& sorted_pts, const std::vector<double>& DT,
                        const std::vector<int32_t>& ra, const std::vector<int32_t>& sk_of) {
  const int R = P.lf.R;
  if (int64_t(sk_of.size()) != P.lf.nleaf || DT.size() != size_t(2) * R * R * ra.size())
    throw Error{DFMM_EINVAL, "leaf weight tables of the wrong size"};
  for (int32_t k : sk_of)
    if (k < 0 || k >= int32_t(ra.size())) throw Error{DFMM_EINVAL, "leaf skeleton index out of range"};
  for (int32_t r : ra)
    if (r < 1 || r > R) throw Error{DFMM_EINVAL, "LF skeleton rank out of range"};
  DevBuf dp, dt, dra, dsk;
  dp.upload(sorted_pts);
  dt.upload(DT);
  dra.upload(ra);
  dsk.upload(sk_of);
  const bool f64 = P.prec == DFMM_PREC_FP64;
  const size_t es = f64 ? sizeof(double2) : sizeof(float2);
  P.lf.V.alloc(es * size_t(P.N) * R);
  P.lf.W.alloc(es * size_t(P.N) * R);
  if (f64)
    hipLaunchKernelGGL(k_leaf_weights<double2>, dim3(unsigned(P.lf.nleaf)), dim3(LW_BS), sizeof(double2) * R, 0,
                       dp.as<double>(), P.leaf_start.as<int>(), P.leaf_center.as<float4>(), P.lf.a64.as<double4>(),
                       dt.as<double2>(), dra.as<int>(), dsk.as<int>(), R, P.lf.V.as<double2>(),
                       P.lf.W.as<double2>());
  else
    hipLaunchKernelGGL(k_leaf_weights<float2>, dim3(unsigned(P.lf.nleaf)), dim3(LW_BS), sizeof(double2) * R, 0,
                       dp.as<double>(), P.leaf_start.as<int>(), P.leaf_center.as<float4>(), P.lf.a64.as<double4>(),
                       dt.as<double2>(), dra.as<int>(), dsk.as<int>(), R, P.lf.V.as<float2>(), P.lf.W.as<float2>());
  DFMM_HIP(hipGetLastError());
  DFMM_HIP(hipDeviceSynchronize());
}

// ---- stage timer -------------------------------------------------------------------
bool StageTimer::begin_apply(hipStream_t st) {
  const size_t i = book.begin_apply();
  if (i == StageBook::kNone) return false;
  DFMM_HIP(hipEventRecord(pool[i], st));
  return true;
}

void StageTimer::mark(int st_id, hipStream_t st) {
  const size_t i = book.mark(st_id);
  if (i != StageBook::kNone) DFMM_HIP(hipEventRecord(pool[i], st));
}

void StageTimer::side_begin(hipStream_t side) {
  const size_t i = book.side_begin();
  if (i != StageBook::kNone) DFMM_HIP(hipEventRecord(pool[i], side));
}

void StageTimer::side_mark(int st_id, hipStream_t side) {
  const size_t i = book.side_mark(st_id);
  if (i != StageBook::kNone) DFMM_HIP(hipEventRecord(pool[i], side));
}

void StageTimer::collect(double* ms, int64_t* launches) {
  // the events carry no system-scope fence: wait for the device, then read them
  if (book.used > 0) DFMM_HIP(hipDeviceSynchronize());
  book.collect(ms, launches, ST_COUNT, [&](size_t a, size_t b) {
    float t = 0.f;
    DFMM_HIP(hipEventElapsedTime(&t, pool[a], pool[b]));
    return t;
  });
}

StageTimer::StageTimer(int applies) : book(size_t(applies) * kPerApply, kPerApply) {
  pool.resize(size_t(applies) * kPerApply);
  // timing-only events: without the system-scope release fence, recording one
  // does not write back the L2 between the launches it separates
  for (auto& e : pool) DFMM_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
}

StageTimer::~StageTimer() {
  for (auto e : pool) (void)hipEventDestroy(e);
}

}  // namespace dfmm
