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
#include <cstring>

#include "internal.hpp"

namespace dfmm {

namespace {

constexpr int RC = 4;  // right-hand sides handled per pass of a kernel

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ void cfma(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x));
  acc.y = fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y));
}

// G for a separation (dx, dy, dz) in float32: e^{2 pi i r} / r, 0 at r = 0.
__device__ __forceinline__ float2 green32(float dx, float dy, float dz) {
  float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  if (r2 == 0.0f) return make_float2(0.0f, 0.0f);
  float ri = rsqrtf(r2);
  float r = r2 * ri;
  float s, c;
  sincospif(2.0f * r, &s, &c);
  return make_float2(c * ri, s * ri);
}

inline unsigned nblocks(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

// ---- permutation into Morton order ------------------------------------------
__global__ void k_permute_in(const float2* __restrict__ f, float2* __restrict__ fs,
                             const int* __restrict__ perm, int64_t N, int nrhs) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N * nrhs) return;
  int64_t s = i / nrhs;
  int k = int(i % nrhs);
  fs[i] = f[int64_t(k) * N + perm[s]];
}

// ---- leaf S2M: outgoing check potentials at c_B + a_p ---------------------------
// One block per leaf; threads over check points.  LDS holds a chunk of the
// leaf's points (local coordinates) and densities.  The check-to-equivalent
// matrix D_LF is folded into the operators that read these potentials.
constexpr int S2M_BS = 128;
__global__ void __launch_bounds__(S2M_BS) k_s2m(const float4* __restrict__ phi, const float4* __restrict__ plo,
                                                 const int* __restrict__ lstart, const float4* __restrict__ lcen,
                                                 const float2* __restrict__ fs, const float4* __restrict__ a_lf,
                                                 int R, int Ra, int nrhs, float2* __restrict__ clf) {
  __shared__ float4 xs[S2M_BS];
  __shared__ float2 fv[S2M_BS * RC];
  const int b = blockIdx.x;
  const int s0 = lstart[b], s1 = lstart[b + 1];
  const float4 c = lcen[b];
  for (int k0 = 0; k0 < nrhs; k0 += RC) {
    const int nk = min(RC, nrhs - k0);
    for (int p0 = 0; p0 < R; p0 += S2M_BS) {
      int p = p0 + threadIdx.x;
      float2 acc[RC];
#pragma unroll
      for (int k = 0; k < RC; ++k) acc[k] = make_float2(0.f, 0.f);
      float4 ap = p < Ra ? a_lf[p] : make_float4(0.f, 0.f, 0.f, 0.f);
      for (int j0 = s0; j0 < s1; j0 += S2M_BS) {
        __syncthreads();
        int j = j0 + threadIdx.x;
        if (j < s1) {
          float4 h = phi[j], l = plo[j];
          xs[threadIdx.x] = make_float4((h.x - c.x) + l.x, (h.y - c.y) + l.y, (h.z - c.z) + l.z, 0.f);
          for (int k = 0; k < nk; ++k) fv[threadIdx.x * RC + k] = fs[int64_t(j) * nrhs + k0 + k];
        }
        __syncthreads();
        int nj = min(S2M_BS, s1 - j0);
        if (p < Ra) {
          for (int t = 0; t < nj; ++t) {
            float4 x = xs[t];
            float2 g = green32(ap.x - x.x, ap.y - x.y, ap.z - x.z);
#pragma unroll
            for (int k = 0; k < RC; ++k)
              if (k < nk) cfma(acc[k], g, fv[t * RC + k]);
          }
        }
      }
      if (p < R)
        for (int k = 0; k < nk; ++k) clf[(int64_t(b) * R + p) * nrhs + k0 + k] = acc[k];
    }
  }
}

// ---- HF-M2M: F[slot] = sum_o M[dir, o] Fchild[child_o] ------------------------
constexpr int M2M_BS = 128;
__global__ void __launch_bounds__(M2M_BS) k_m2m(const int* __restrict__ child, const int* __restrict__ opb,
                                                 const float2* __restrict__ M, const float2* __restrict__ Fc,
                                                 int R, int Rc, int nrhs, float2* __restrict__ F) {
  extern __shared__ float2 xs[];  // 8 * Rc * RC
  const int64_t i = blockIdx.x;
  const int base = opb[i];
  for (int k0 = 0; k0 < nrhs; k0 += RC) {
    const int nk = min(RC, nrhs - k0);
    __syncthreads();
    for (int t = threadIdx.x; t < 8 * Rc * RC; t += M2M_BS) {
      int o = t / (Rc * RC), rem = t % (Rc * RC), p = rem / RC, k = rem % RC;
      int c = child[8 * i + o];
      xs[t] = (c >= 0 && k < nk) ? Fc[(int64_t(c) * Rc + p) * nrhs + k0 + k] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < R; q += M2M_BS) {
      float2 acc[RC];
#pragma unroll
      for (int k = 0; k < RC; ++k) acc[k] = make_float2(0.f, 0.f);
      for (int o = 0; o < 8; ++o) {
        if (child[8 * i + o] < 0) continue;
        const float2* Mo = M + (int64_t(base + o) * R + q) * Rc;
        const float2* xo = xs + o * Rc * RC;
        for (int p = 0; p < Rc; ++p) {
          float2 m = Mo[p];
#pragma unroll
          for (int k = 0; k < RC; ++k) cfma(acc[k], m, xo[p * RC + k]);
        }
      }
      for (int k = 0; k < nk; ++k) F[(i * R + q) * nrhs + k0 + k] = acc[k];
    }
  }
}

// ---- M2L grouped by offset: Y[pos] = T[g] F[src[pos]] ---------------------------
// One block per (group, chunk of 64 columns); a column is (pair, rhs).  The
// source vectors of the chunk sit in LDS as [row][column]; T is read from
// global memory (one row per wave step, uniform across the wave).
constexpr int M2L_BS = 256;
constexpr int M2L_COLS = 32;
__global__ void __launch_bounds__(M2L_BS) k_m2l(const int* __restrict__ gstart, const int* __restrict__ src,
                                                 const float2* __restrict__ T, const float2* __restrict__ F,
                                                 int R, int nrhs, const int* __restrict__ chunk_grp,
                                                 const int* __restrict__ chunk_col0, float2* __restrict__ Y) {
  extern __shared__ float2 xs[];  // R * M2L_COLS
  const int g = chunk_grp[blockIdx.x];
  const int64_t c0 = chunk_col0[blockIdx.x];
  const int64_t p0 = gstart[g], p1 = gstart[g + 1];
  const int64_t ncol = (p1 - p0) * nrhs;
  const int nc = int(min<int64_t>(M2L_COLS, ncol - c0));
  for (int t = threadIdx.x; t < R * M2L_COLS; t += M2L_BS) {
    int row = t / M2L_COLS, col = t % M2L_COLS;
    float2 v = make_float2(0.f, 0.f);
    if (col < nc) {
      int64_t cc = c0 + col;
      int64_t pos = p0 + cc / nrhs;
      int k = int(cc % nrhs);
      v = F[(int64_t(src[pos]) * R + row) * nrhs + k];
    }
    xs[t] = v;
  }
  __syncthreads();
  const int col = threadIdx.x % M2L_COLS;
  const int rb = threadIdx.x / M2L_COLS;
  const float2* Tg = T + int64_t(g) * R * R;
  for (int q = rb; q < R; q += M2L_BS / M2L_COLS) {
    float2 acc = make_float2(0.f, 0.f);
    const float2* Tq = Tg + int64_t(q) * R;
    for (int p = 0; p < R; ++p) cfma(acc, Tq[p], xs[p * M2L_COLS + col]);
    if (col < nc) {
      int64_t cc = c0 + col;
      int64_t pos = p0 + cc / nrhs;
      int k = int(cc % nrhs);
      Y[(pos * R + q) * nrhs + k] = acc;
    }
  }
}

// ---- U[slot] += sum of Y over the pairs of the slot ------------------------------
__global__ void k_reduce(const int* __restrict__ rs, const int* __restrict__ ri, const float2* __restrict__ Y,
                         int64_t nslot, int RN, float2* __restrict__ U) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nslot * RN) return;
  int64_t s = t / RN;
  int e = int(t % RN);
  float2 acc = U[t];
  for (int j = rs[s]; j < rs[s + 1]; ++j) {
    float2 y = Y[int64_t(ri[j]) * RN + e];
    acc.x += y.x;
    acc.y += y.y;
  }
  U[t] = acc;
}

// ---- HF-L2L: Uc[child] = sum_t Mdn[op_t] U[par_t] ----------------------------------
constexpr int L2L_BS = 128;
__global__ void __launch_bounds__(L2L_BS) k_l2l(const int* __restrict__ par, const int* __restrict__ op,
                                                 int terms, const float2* __restrict__ M,
                                                 const float2* __restrict__ U, int R, int Rc, int nrhs,
                                                 float2* __restrict__ Uc) {
  extern __shared__ float2 xs[];  // terms * R * RC
  const int64_t i = blockIdx.x;
  for (int k0 = 0; k0 < nrhs; k0 += RC) {
    const int nk = min(RC, nrhs - k0);
    __syncthreads();
    for (int t = threadIdx.x; t < terms * R * RC; t += L2L_BS) {
      int tt = t / (R * RC), rem = t % (R * RC), s = rem / RC, k = rem % RC;
      int pp = par[i * terms + tt];
      xs[t] = (pp >= 0 && k < nk) ? U[(int64_t(pp) * R + s) * nrhs + k0 + k] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < Rc; q += L2L_BS) {
      float2 acc[RC];
#pragma unroll
      for (int k = 0; k < RC; ++k) acc[k] = make_float2(0.f, 0.f);
      for (int tt = 0; tt < terms; ++tt) {
        int o = op[i * terms + tt];
        if (o < 0) continue;
        const float2* Mo = M + (int64_t(o) * Rc + q) * R;  // row q of Mdn[o] (Rc x R)
        const float2* xo = xs + tt * R * RC;
        for (int s = 0; s < R; ++s) {
          float2 m = Mo[s];
#pragma unroll
          for (int k = 0; k < RC; ++k) cfma(acc[k], m, xo[s * RC + k]);
        }
      }
      for (int k = 0; k < nk; ++k) Uc[(i * Rc + q) * nrhs + k0 + k] = acc[k];
    }
  }
}

// ---- leaf evaluation: L2T plus the near-field sum, written in user order ----------
// One block per leaf, one thread per target point (looping if the leaf holds
// more points than threads).  L2T runs in float64: g = D_LF^T U_LF[leaf] (the
// incoming equivalent charges at c + a_p, large and mutually cancelling) and
// the kernel values G(x, c + a_p).  The near-field sum evaluates G in float32
// on hi/lo point differences and accumulates in float64.
constexpr int EV_BS = 64;
__device__ __forceinline__ void green64(double dx, double dy, double dz, double& re, double& im) {
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  double s, c;
  sincospi(2.0 * r, &s, &c);
  double ri = 1.0 / r;
  re = c * ri;
  im = s * ri;
}

__global__ void __launch_bounds__(EV_BS) k_leaf_eval(const float4* __restrict__ phi, const float4* __restrict__ plo,
                                                      const int* __restrict__ lstart, const float4* __restrict__ lcen,
                                                      const int* __restrict__ nstart, const int* __restrict__ nsrc,
                                                      const float2* __restrict__ fs, const double4* __restrict__ a_lf,
                                                      const double2* __restrict__ Dm, const float2* __restrict__ ulf,
                                                      int R, int Ra, int nrhs, int64_t N, const int* __restrict__ perm,
                                                      float2* __restrict__ u) {
  __shared__ float4 sh[EV_BS], sl[EV_BS];
  __shared__ float2 fv[EV_BS * RC];
  extern __shared__ double2 g[];  // R * RC
  const int b = blockIdx.x;
  const int s0 = lstart[b], s1 = lstart[b + 1];
  const float4 c = lcen[b];
  for (int k0 = 0; k0 < nrhs; k0 += RC) {
    const int nk = min(RC, nrhs - k0);
    __syncthreads();
    for (int p = threadIdx.x; p < R; p += EV_BS) {
      double gr[RC], gi[RC];
#pragma unroll
      for (int k = 0; k < RC; ++k) gr[k] = gi[k] = 0.0;
      for (int q = 0; q < R; ++q) {
        double2 d = Dm[q * R + p];  // (D^T)[p][q]
#pragma unroll
        for (int k = 0; k < RC; ++k)
          if (k < nk) {
            float2 v = ulf[(int64_t(b) * R + q) * nrhs + k0 + k];
            gr[k] += d.x * double(v.x) - d.y * double(v.y);
            gi[k] += d.x * double(v.y) + d.y * double(v.x);
          }
      }
      for (int k = 0; k < RC; ++k) g[p * RC + k] = make_double2(gr[k], gi[k]);
    }
    __syncthreads();
    for (int t0 = s0; t0 < s1; t0 += EV_BS) {
      const int t = t0 + threadIdx.x;
      const bool act = t < s1;
      float4 th = act ? phi[t] : make_float4(0.f, 0.f, 0.f, 0.f);
      float4 tl = act ? plo[t] : make_float4(0.f, 0.f, 0.f, 0.f);
      double ar[RC], ai[RC];
#pragma unroll
      for (int k = 0; k < RC; ++k) ar[k] = ai[k] = 0.0;
      // L2T in float64
      {
        double lx = (double(th.x) - double(c.x)) + double(tl.x);
        double ly = (double(th.y) - double(c.y)) + double(tl.y);
        double lz = (double(th.z) - double(c.z)) + double(tl.z);
        for (int p = 0; p < Ra; ++p) {  // padded check points carry g = 0
          double4 ap = a_lf[p];
          double re, im;
          green64(lx - ap.x, ly - ap.y, lz - ap.z, re, im);
#pragma unroll
          for (int k = 0; k < RC; ++k) {
            double2 gg = g[p * RC + k];
            ar[k] += re * gg.x - im * gg.y;
            ai[k] += re * gg.y + im * gg.x;
          }
        }
      }
      // near field over adjacent leaves (self included)
      for (int a = nstart[b]; a < nstart[b + 1]; ++a) {
        const int A = nsrc[a];
        const int q0 = lstart[A], q1 = lstart[A + 1];
        for (int j0 = q0; j0 < q1; j0 += EV_BS) {
          __syncthreads();
          int j = j0 + threadIdx.x;
          if (j < q1) {
            sh[threadIdx.x] = phi[j];
            sl[threadIdx.x] = plo[j];
            for (int k = 0; k < nk; ++k) fv[threadIdx.x * RC + k] = fs[int64_t(j) * nrhs + k0 + k];
          }
          __syncthreads();
          const int nj = min(EV_BS, q1 - j0);
          for (int jj = 0; jj < nj; ++jj) {
            float4 h = sh[jj], l = sl[jj];
            float dx = (th.x - h.x) + (tl.x - l.x);
            float dy = (th.y - h.y) + (tl.y - l.y);
            float dz = (th.z - h.z) + (tl.z - l.z);
            float2 gg = green32(dx, dy, dz);
#pragma unroll
            for (int k = 0; k < RC; ++k) {
              if (k < nk) {
                float2 fk = fv[jj * RC + k];
                ar[k] += double(gg.x * fk.x - gg.y * fk.y);
                ai[k] += double(gg.x * fk.y + gg.y * fk.x);
              }
            }
          }
        }
      }
      if (act) {
        int64_t o = perm[t];
        for (int k = 0; k < nk; ++k) u[int64_t(k0 + k) * N + o] = make_float2(float(ar[k]), float(ai[k]));
      }
    }
  }
}

__global__ void k_zero(float2* __restrict__ p, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_float2(0.f, 0.f);
}

struct Chunks {
  DevBuf grp, col0;
  int64_t n = 0;
};

}  // namespace

// Column chunks of the grouped M2L for a given nrhs (host-side bookkeeping).
static void make_chunks(const std::vector<int32_t>& gstart, int nrhs, std::vector<int32_t>& grp,
                        std::vector<int32_t>& col0) {
  grp.clear();
  col0.clear();
  for (size_t g = 0; g + 1 < gstart.size(); ++g) {
    int64_t ncol = int64_t(gstart[g + 1] - gstart[g]) * nrhs;
    for (int64_t c = 0; c < ncol; c += M2L_COLS) {
      grp.push_back(int32_t(g));
      col0.push_back(int32_t(c));
    }
  }
}

struct ApplyState {
  int nrhs = 0;
  std::vector<std::unique_ptr<DevBuf>> F, U;  // per HF level
  DevBuf fs, flf, ulf, Y;
  DevBuf lf_cg, lf_cc;
  int64_t lf_nch = 0;
  std::vector<std::unique_ptr<DevBuf>> cg, cc;
  std::vector<int64_t> nch;
  std::vector<hipEvent_t> ev;
  ~ApplyState() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

void destroy_apply_state(ApplyState* s) { delete s; }

static void ensure_workspace(dfmm_plan_s& P, int nrhs, ApplyState& S) {
  if (S.nrhs == nrhs) return;
  S.nrhs = nrhs;
  int64_t N = P.N;
  S.fs.alloc(sizeof(float2) * N * nrhs);
  S.flf.alloc(sizeof(float2) * P.lf.nleaf * P.lf.R * nrhs);
  S.ulf.alloc(sizeof(float2) * P.lf.nleaf * P.lf.R * nrhs);
  int64_t ymax = P.lf.npairs * P.lf.R;
  S.F.clear();
  S.U.clear();
  S.cg.clear();
  S.cc.clear();
  S.nch.clear();
  for (auto& H : P.hf) {
    S.F.emplace_back(new DevBuf());
    S.U.emplace_back(new DevBuf());
    S.F.back()->alloc(sizeof(float2) * std::max<int64_t>(1, H.nout) * H.R * nrhs);
    S.U.back()->alloc(sizeof(float2) * std::max<int64_t>(1, H.nin) * H.R * nrhs);
    ymax = std::max<int64_t>(ymax, H.npairs * H.R);
  }
  S.Y.alloc(sizeof(float2) * std::max<int64_t>(1, ymax) * nrhs);
  std::vector<int32_t> grp, col0;
  for (size_t e = 0; e < P.hf.size(); ++e) {
    make_chunks(P.hf[e].gs_h, nrhs, grp, col0);
    S.cg.emplace_back(new DevBuf());
    S.cc.emplace_back(new DevBuf());
    S.cg.back()->upload(grp);
    S.cc.back()->upload(col0);
    S.nch.push_back(int64_t(grp.size()));
  }
  make_chunks(P.lf.gs_h, nrhs, grp, col0);
  S.lf_cg.upload(grp);
  S.lf_cc.upload(col0);
  S.lf_nch = int64_t(grp.size());
}

void run_apply(dfmm_plan_s& P, const void* fv, void* uv, int nrhs, hipStream_t st) {
  if (!P.ws) P.ws = new ApplyState();
  ApplyState& S = *P.ws;
  ensure_workspace(P, nrhs, S);
  const float2* f = static_cast<const float2*>(fv);
  float2* u = static_cast<float2*>(uv);
  const int64_t N = P.N;
  const int64_t nleaf = P.lf.nleaf;
  const int Rl = P.lf.R;
  const int e_top = int(P.hf.size()) - 1;
  bool timing = P.timing;
  if (timing && S.ev.empty()) {
    S.ev.resize(10);
    for (auto& e : S.ev) DFMM_HIP(hipEventCreate(&e));
  }
  auto mark = [&](int i) {
    if (timing) DFMM_HIP(hipEventRecord(S.ev[i], st));
  };
  mark(0);
  hipLaunchKernelGGL(k_permute_in, dim3(nblocks(N * nrhs, 256)), dim3(256), 0, st, f, S.fs.as<float2>(),
                     P.perm_d.as<int>(), N, nrhs);
  mark(1);
  hipLaunchKernelGGL(k_s2m, dim3(unsigned(nleaf)), dim3(S2M_BS), 0, st, P.pthi.as<float4>(), P.ptlo.as<float4>(),
                     P.leaf_start.as<int>(), P.leaf_center.as<float4>(), S.fs.as<float2>(), P.lf.a.as<float4>(), Rl,
                     P.lf.r, nrhs, S.flf.as<float2>());
  mark(2);
  // HF-M2M, fine to coarse
  for (int e = 0; e <= e_top; ++e) {
    HFLevel& H = P.hf[e];
    if (H.nout == 0) continue;
    const float2* Fc = e == 0 ? S.flf.as<float2>() : S.F[e - 1]->as<float2>();
    hipLaunchKernelGGL(k_m2m, dim3(unsigned(H.nout)), dim3(M2M_BS), sizeof(float2) * 8 * H.Rc * RC, st,
                       H.m2m_child.as<int>(), H.m2m_op.as<int>(), H.Mup.as<float2>(), Fc, H.R, H.Rc, nrhs,
                       S.F[e]->as<float2>());
  }
  mark(3);
  // HF-M2L then HF-L2L, coarse to fine
  if (e_top >= 0) {
    HFLevel& H = P.hf[e_top];
    int64_t n = std::max<int64_t>(1, H.nin) * H.R * nrhs;
    hipLaunchKernelGGL(k_zero, dim3(nblocks(n, 256)), dim3(256), 0, st, S.U[e_top]->as<float2>(), n);
  }
  for (int e = e_top; e >= 0; --e) {
    HFLevel& H = P.hf[e];
    if (S.nch[e] > 0) {
      hipLaunchKernelGGL(k_m2l, dim3(unsigned(S.nch[e])), dim3(M2L_BS), sizeof(float2) * H.R * M2L_COLS, st,
                         H.grp_start.as<int>(), H.pair_src.as<int>(), H.T.as<float2>(), S.F[e]->as<float2>(), H.R,
                         nrhs, S.cg[e]->as<int>(), S.cc[e]->as<int>(), S.Y.as<float2>());
      int RN = H.R * nrhs;
      hipLaunchKernelGGL(k_reduce, dim3(nblocks(H.nin * RN, 256)), dim3(256), 0, st, H.red_start.as<int>(),
                         H.red_idx.as<int>(), S.Y.as<float2>(), H.nin, RN, S.U[e]->as<float2>());
    }
    float2* Uc = e == 0 ? S.ulf.as<float2>() : S.U[e - 1]->as<float2>();
    int64_t nchild = H.nchild_in;
    if (nchild > 0)
      hipLaunchKernelGGL(k_l2l, dim3(unsigned(nchild)), dim3(L2L_BS), sizeof(float2) * H.l2l_terms * H.R * RC, st,
                         H.l2l_par.as<int>(), H.l2l_op.as<int>(), H.l2l_terms, H.Mdn.as<float2>(),
                         S.U[e]->as<float2>(), H.R, H.Rc, nrhs, Uc);
  }
  if (e_top < 0) {
    int64_t n = nleaf * Rl * nrhs;
    hipLaunchKernelGGL(k_zero, dim3(nblocks(n, 256)), dim3(256), 0, st, S.ulf.as<float2>(), n);
  }
  mark(4);
  // LF-M2L
  if (S.lf_nch > 0) {
    hipLaunchKernelGGL(k_m2l, dim3(unsigned(S.lf_nch)), dim3(M2L_BS), sizeof(float2) * Rl * M2L_COLS, st,
                       P.lf.grp_start.as<int>(), P.lf.pair_src.as<int>(), P.lf.T.as<float2>(), S.flf.as<float2>(),
                       Rl, nrhs, S.lf_cg.as<int>(), S.lf_cc.as<int>(), S.Y.as<float2>());
    int RN = Rl * nrhs;
    hipLaunchKernelGGL(k_reduce, dim3(nblocks(nleaf * RN, 256)), dim3(256), 0, st, P.lf.red_start.as<int>(),
                       P.lf.red_idx.as<int>(), S.Y.as<float2>(), nleaf, RN, S.ulf.as<float2>());
  }
  mark(5);
  hipLaunchKernelGGL(k_leaf_eval, dim3(unsigned(nleaf)), dim3(EV_BS), sizeof(double2) * Rl * RC, st,
                     P.pthi.as<float4>(), P.ptlo.as<float4>(), P.leaf_start.as<int>(), P.leaf_center.as<float4>(),
                     P.near_start.as<int>(), P.near_src.as<int>(), S.fs.as<float2>(), P.lf.a64.as<double4>(),
                     P.lf.D64.as<double2>(), S.ulf.as<float2>(), Rl, P.lf.r, nrhs, N, P.perm_d.as<int>(), u);
  mark(6);
  DFMM_HIP(hipGetLastError());
  if (timing) {
    DFMM_HIP(hipEventSynchronize(S.ev[6]));
    P.stage_ms.assign(6, 0.0);
    for (int i = 0; i < 6; ++i) {
      float ms = 0.f;
      DFMM_HIP(hipEventElapsedTime(&ms, S.ev[i], S.ev[i + 1]));
      P.stage_ms[i] = ms;
    }
  }
}

}  // namespace dfmm
