// The evaluation pass in float64 (plans of precision DFMM_PREC_FP64), for
// end-to-end accuracies down to 1e-8 and below, where the float32 vectors of
// the other plans set the floor (about 1e-7).  Same steps as apply.hip
// (Algorithm 1 plus the near-field sum), all in float64 / complex128:
// densities and potentials, leaf weights, equivalent check potentials, the
// translation operators (GEMMs on v_mfma_f64_16x16x4f64, slot form for every
// number of right-hand sides) and the near-field sum with float64 sin / cos.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <set>
#include <string>

#include "internal.hpp"

namespace dfmm {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

inline unsigned nblk(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

__global__ void k_permute_in64(const double2* __restrict__ f, double2* __restrict__ fs, const int* __restrict__ perm,
                               int64_t N, int nrhs) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N * nrhs) return;
  const int64_t s = i / nrhs;
  const int k = int(i % nrhs);
  fs[i] = f[int64_t(k) * N + perm[s]];
}

// Leaf S2M: chk[b][k][p] = sum_{j in leaf b} V[j][p] fs[j][k]; one block per leaf,
// threads over check points, sources in order.
constexpr int S64_BS = 128;
__global__ void __launch_bounds__(S64_BS) k_s2m64(const int* __restrict__ lstart, const double2* __restrict__ V,
                                                   const double2* __restrict__ fs, int R, int nrhs,
                                                   double2* __restrict__ clf) {
  const int b = blockIdx.x;
  const int s0 = lstart[b], s1 = lstart[b + 1];
  for (int k = 0; k < nrhs; ++k)
    for (int p = threadIdx.x; p < R; p += S64_BS) {
      double re = 0.0, im = 0.0;
      for (int j = s0; j < s1; ++j) {
        const double2 v = V[int64_t(j) * R + p], x = fs[int64_t(j) * nrhs + k];
        re = fma(v.x, x.x, fma(-v.y, x.y, re));
        im = fma(v.x, x.y, fma(v.y, x.x, im));
      }
      clf[(int64_t(b) * nrhs + k) * R + p] = make_double2(re, im);
    }
}

// Near-field sum in float64: one block of 64 threads per leaf; the adjacent
// leaves' points (separations from the hi / lo float parts, formed in float64)
// and densities are staged in LDS a chunk at a time; G = exp(2 pi i r) / r with
// the phase reduced in float64 and sin / cos of it in float64.
constexpr int N64_BS = 64;
constexpr int N64_CHUNK = 128;
constexpr int N64_RC = 4;  // right-hand sides per pass
__global__ void __launch_bounds__(N64_BS) k_near64(const float4* __restrict__ phi, const float4* __restrict__ plo,
                                                    const int* __restrict__ lstart, const int* __restrict__ nstart,
                                                    const int* __restrict__ nsrc, const double2* __restrict__ fs,
                                                    int nrhs, int64_t N, double2* __restrict__ unear) {
  __shared__ double sx[N64_CHUNK], sy[N64_CHUNK], sz[N64_CHUNK];
  __shared__ double2 sf[N64_CHUNK * N64_RC];
  __shared__ int nb_beg[64], nb_off[65];
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  const int s0 = lstart[b], s1 = lstart[b + 1];
  const int n0 = nstart[b];
  const int nn = min(nstart[b + 1] - n0, 64);  // adjacent leaves (at most 27)
  {
    int beg = 0, cnt = 0;
    if (lane < nn) {
      const int A = nsrc[n0 + lane];
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
  for (int k0 = 0; k0 < nrhs; k0 += N64_RC) {
    const int nk = min(N64_RC, nrhs - k0);
    for (int t0 = s0; t0 < s1; t0 += N64_BS) {
      const int t = t0 + lane;
      const bool act = t < s1;
      const int tt = act ? t : s0;
      const float4 th = phi[tt], tq = plo[tt];
      const double tx = double(th.x) + double(tq.x), ty = double(th.y) + double(tq.y),
                   tz = double(th.z) + double(tq.z);
      double ar[N64_RC], ai[N64_RC];
#pragma unroll
      for (int k = 0; k < N64_RC; ++k) ar[k] = ai[k] = 0.0;
      for (int base = 0; base < total; base += N64_CHUNK) {
        const int fill = min(N64_CHUNK, total - base);
        __syncthreads();
        for (int i = lane; i < fill; i += N64_BS) {
          const int g = base + i;
          int q = 0;  // the neighbour holding element g: largest q with nb_off[q] <= g
          for (int step = 16; step > 0; step >>= 1)
            if (q + step < nn && nb_off[q + step] <= g) q += step;
          const int j = nb_beg[q] + (g - nb_off[q]);
          const float4 h = phi[j], l = plo[j];
          sx[i] = double(h.x) + double(l.x);
          sy[i] = double(h.y) + double(l.y);
          sz[i] = double(h.z) + double(l.z);
          for (int k = 0; k < N64_RC; ++k)
            sf[i * N64_RC + k] = k < nk ? fs[int64_t(j) * nrhs + k0 + k] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int i = 0; i < fill; ++i) {
          const double dx = tx - sx[i], dy = ty - sy[i], dz = tz - sz[i];
          const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
          if (r2 == 0.0) continue;  // coincident points contribute nothing
          const double r = sqrt(r2);
          double sn, cs;
          sincospi(2.0 * (r - rint(r)), &sn, &cs);
          const double ri = 1.0 / r;
          const double gr = cs * ri, gi = sn * ri;
#pragma unroll
          for (int k = 0; k < N64_RC; ++k) {
            const double2 x = sf[i * N64_RC + k];
            ar[k] = fma(gr, x.x, fma(-gi, x.y, ar[k]));
            ai[k] = fma(gr, x.y, fma(gi, x.x, ai[k]));
          }
        }
      }
      if (act)
        for (int k = 0; k < nk; ++k) unear[int64_t(k0 + k) * N + t] = make_double2(ar[k], ai[k]);
    }
  }
}

// Slot-form translation GEMM in float64: a workgroup of 4 waves owns one output
// slot and 16 of its right-hand sides; wave w holds the 16-row M-tiles
// w, w + 4, ... (up to MT of them) as float64 MFMA accumulators across all
// terms.  Per term the source columns are staged in LDS, then every tile runs
// its k-steps on v_mfma_f64_16x16x4f64 with the operator fragments read from
// memory one step ahead.  Complex as interleaved real, as in the float32
// engine: real row 2q of the operator is (Re, -Im), row 2q + 1 is (Im, Re).
struct Slot64Args {
  const int* order;
  const int* t0;
  const int* gm;
  const int4* terms;  // (operator double4 offset, source vector, K | kind << 14, 0)
  const double4* A0;
  const double4* A1;
  const double2* X0;
  const double2* X1;
  int KX0, KX1;
  int M;
  int cpg;
  int S;      // LDS column stride in double4
};

template <int MT>
__global__ void __launch_bounds__(256) k_slot64(const Slot64Args a, int nrhs, double2* __restrict__ Y) {
  extern __shared__ double4 xs64[];  // 16 columns x S double4
  const int tid = int(threadIdx.x);
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int j = lane & 15, kr = lane >> 4;
  const bool odd = (j & 1) != 0;
  const int chunk = int(blockIdx.x);
  const int g = a.order[chunk / a.cpg];
  const int c0 = (chunk % a.cpg) * 16;
  const int nc = min(16, nrhs - c0);
  const int tb = a.t0[g], te = a.t0[g + 1];
  const int nM = a.gm[g] / 8;
  const int S = a.S;
  v4d acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int i = tb; i < te; ++i) {
    const int4 e = a.terms[i];
    const int kind = (e.z >> 14) & 1;
    const int Kg = e.z & 0xFFF;
    const int KX = kind ? a.KX1 : a.KX0;
    const double4* A = (kind ? a.A1 : a.A0) + e.x;
    const double2* X = (kind ? a.X1 : a.X0) + (int64_t(e.y) * nrhs + c0) * KX;
    const int Q4 = Kg / 8;          // k-steps: 8 complex k each (4 quarters x 2)
    __syncthreads();                // the previous term's columns are consumed
    // column c: its first Kg complex entries as Kg / 2 double4, in order (quarter
    // kr of the k range starts at double4 kr Q4)
    for (int idx = tid; idx < 16 * (Kg / 2); idx += 256) {
      const int col = idx / (Kg / 2), q = idx - col * (Kg / 2);
      double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
      if (col < nc) {
        const double2* p = X + int64_t(col) * KX + 2 * q;
        const double2 u0 = p[0], u1 = p[1];
        v = make_double4(u0.x, u0.y, u1.x, u1.y);
      }
      xs64[col * S + q] = v;
    }
    __syncthreads();
    const double4* bcol = xs64 + j * S + kr * Q4;
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      const int m = wave + 4 * t;
      if (m < nM) {  // wave-uniform
        const double4* ap = A + int64_t(m) * Q4 * 32 + (j >> 1) * 4 + kr;
        double4 v = ap[0];
        for (int s = 0; s < Q4; ++s) {
          const double4 vn = ap[min(s + 1, Q4 - 1) * 32];  // next step's fragment, in flight
          const double4 b = bcol[s];
          const double f0 = odd ? v.y : v.x, f1 = odd ? v.x : -v.y, f2 = odd ? v.w : v.z, f3 = odd ? v.z : -v.w;
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(f0, b.x, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(f1, b.y, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(f2, b.z, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(f3, b.w, acc[t], 0, 0, 0);
          v = vn;
        }
      }
    }
  }
  // v_mfma_f64_16x16x4f64 leaves real row kr + 4 r of the tile (column j) in
  // register r of lane (j, kr): even kr hold the real parts of complex rows
  // kr / 2 + 2 r, odd kr the imaginary parts of the same rows, so lane (j, kr)
  // with kr even takes the imaginary parts from lane (j, kr + 1) and writes
  // its four complex rows
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const int m = wave + 4 * t;
    const v4d o = m < nM ? acc[t] : v4d{0.0, 0.0, 0.0, 0.0};
    double im[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) im[r] = __shfl_xor(o[r], 16, 64);
    if (j < nc && (kr & 1) == 0 && m < a.M / 8) {
      double2* yp = Y + (int64_t(g) * nrhs + c0 + j) * a.M + 8 * m + (kr >> 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) yp[2 * r] = make_double2(o[r], im[r]);
    }
  }
}

// L2T and the output: u[k][perm[t]] = sum_q W[t][q] U_LF[leaf(t)][k][q] + unear[k][t].
__global__ void k_l2t64(const double2* __restrict__ W, const double2* __restrict__ ulf, const int* __restrict__ leaf_of,
                        const double2* __restrict__ unear, const int* __restrict__ perm, int R, int nrhs, int64_t N,
                        double2* __restrict__ u) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N * nrhs) return;
  const int k = int(i / N);
  const int64_t t = i % N;
  const double2* w = W + t * R;
  const double2* x = ulf + (int64_t(leaf_of[t]) * nrhs + k) * R;
  double re = 0.0, im = 0.0;
  for (int q = 0; q < R; ++q) {
    const double2 a = w[q], b = x[q];
    re = fma(a.x, b.x, fma(-a.y, b.y, re));
    im = fma(a.x, b.y, fma(a.y, b.x, im));
  }
  const double2 nf = unear[int64_t(k) * N + t];
  u[int64_t(k) * N + perm[t]] = make_double2(re + nf.x, im + nf.y);
}

// tiles per wave of the largest group
int slot64_mt(const SlotGemm& S) { return (S.M / 8 + 3) / 4; }

constexpr int kLds64 = 159 * 1024;  // dynamic LDS limit set on the float64 slot kernels

template <int MT>
void launch_slot64_t(const SlotGemm& S, const Slot64Args& a, int nrhs, double2* Y, hipStream_t st) {
  const size_t lds = sizeof(double4) * 16 * size_t(a.S);
  static std::mutex mu;
  static std::set<int> done;  // devices on which the attribute is set
  int dev = 0;
  DFMM_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!done.count(dev)) {
      DFMM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_slot64<MT>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, kLds64));
      done.insert(dev);
    }
  }
  hipLaunchKernelGGL(k_slot64<MT>, dim3(unsigned(S.ngroups * a.cpg)), dim3(256), lds, st, a, nrhs, Y);
}

void launch_slot64(const SlotGemm& S, const double4* A0, const double2* X0, int KX0, const double4* A1,
                   const double2* X1, int KX1, int nrhs, double2* Y, hipStream_t st) {
  if (S.ngroups == 0) return;
  if (S.split2 || S.Kmax % 8 != 0) throw Error{DFMM_EUNSUPPORTED, "float64 slot GEMM: bad operator packing"};
  const int cpg = (nrhs + 15) / 16;
  Slot64Args a{S.order.as<int>(), S.t0.as<int>(), S.gm.as<int>(), S.terms.as<int4>(), A0, A1 ? A1 : A0, X0,
               X1 ? X1 : X0, KX0, X1 ? KX1 : KX0, S.M, cpg, S.Kmax / 2 + 1};
  const int mt = slot64_mt(S);
  if (sizeof(double4) * 16 * size_t(a.S) > size_t(kLds64))
    throw Error{DFMM_EUNSUPPORTED, "skeleton rank too large for the float64 slot GEMM"};
  if (mt <= 2) launch_slot64_t<2>(S, a, nrhs, Y, st);
  else if (mt <= 4) launch_slot64_t<4>(S, a, nrhs, Y, st);
  else if (mt <= 8) launch_slot64_t<8>(S, a, nrhs, Y, st);
  else throw Error{DFMM_EUNSUPPORTED, "skeleton rank too large for the float64 slot GEMM"};
}

}  // namespace

void run_apply64(dfmm_plan_s& P, const double2* f, double2* u, int nrhs, hipStream_t st, void* ws) {
  const WsLayout L = ws_layout(ws_shape64(P), nrhs, false, 16);
  if (!ws) throw Error{DFMM_EINVAL, "no workspace"};
  char* b = static_cast<char*>(ws);
  double2* fs = reinterpret_cast<double2*>(b + L.fs);
  double2* unear = reinterpret_cast<double2*>(b + L.unear);
  double2* flf = reinterpret_cast<double2*>(b + L.flf);
  double2* ulf = reinterpret_cast<double2*>(b + L.ulf);
  std::vector<double2*> F, U;
  for (size_t e = 0; e < L.F.size(); ++e) {
    F.push_back(reinterpret_cast<double2*>(b + L.F[e]));
    U.push_back(reinterpret_cast<double2*>(b + L.U[e]));
  }
  const int64_t N = P.N, nleaf = P.lf.nleaf;
  const int Rl = P.lf.R, e_top = int(P.hf.size()) - 1;
  hipLaunchKernelGGL(k_permute_in64, dim3(nblk(N * nrhs, 256)), dim3(256), 0, st, f, fs, P.perm_d.as<int>(), N, nrhs);
  hipLaunchKernelGGL(k_near64, dim3(unsigned(nleaf)), dim3(N64_BS), 0, st, P.pthi.as<float4>(), P.ptlo.as<float4>(),
                     P.leaf_start.as<int>(), P.near_start.as<int>(), P.near_src.as<int>(), fs, nrhs, N, unear);
  hipLaunchKernelGGL(k_s2m64, dim3(unsigned(nleaf)), dim3(S64_BS), 0, st, P.leaf_start.as<int>(),
                     P.lf.V.as<double2>(), fs, Rl, nrhs, flf);
  for (int e = 0; e <= e_top; ++e) {
    const double2* Fc = e == 0 ? flf : F[size_t(e - 1)];
    const int KC = e == 0 ? Rl : P.hf[size_t(e - 1)].R;
    launch_slot64(P.hf[size_t(e)].up, P.hf[size_t(e)].m2m.A.as<double4>(), Fc, KC, nullptr, nullptr, 0, nrhs,
                  F[size_t(e)], st);
  }
  for (int e = e_top; e >= 0; --e) {
    const HFLevel& H = P.hf[size_t(e)];
    const bool par = e < e_top;
    launch_slot64(H.down, H.m2l.A.as<double4>(), F[size_t(e)], H.R,
                  par ? P.hf[size_t(e + 1)].l2l.A.as<double4>() : nullptr, par ? U[size_t(e + 1)] : nullptr,
                  par ? P.hf[size_t(e + 1)].R : 0, nrhs, U[size_t(e)], st);
  }
  launch_slot64(P.lf.down, P.lf.m2l.A.as<double4>(), flf, Rl, e_top >= 0 ? P.hf[0].l2l.A.as<double4>() : nullptr,
                e_top >= 0 ? U[0] : nullptr, e_top >= 0 ? P.hf[0].R : 0, nrhs, ulf, st);
  hipLaunchKernelGGL(k_l2t64, dim3(nblk(N * nrhs, 256)), dim3(256), 0, st, P.lf.W.as<double2>(), ulf,
                     P.leaf_of.as<int>(), unear, P.perm_d.as<int>(), Rl, nrhs, N, u);
  DFMM_HIP(hipGetLastError());
}

WsShape ws_shape64(const dfmm_plan_s& P) {
  WsShape z;
  z.N = P.N;
  z.nleaf = P.lf.nleaf;
  z.Rlf = P.lf.R;
  for (const auto& H : P.hf) {
    z.nout.push_back(H.nout);
    z.nin.push_back(H.nin);
    z.R.push_back(H.R);
  }
  z.pair_rows = 0;
  return z;
}

}  // namespace dfmm
