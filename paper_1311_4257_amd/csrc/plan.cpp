// Plan construction: octree, interaction lists, wedges, needed directions and
// translation tables (Section 2.2, Algorithm 1), resident on the device.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <thread>
#include <tuple>

#include "geometry.hpp"
#include "internal.hpp"

namespace dfmm {

void build_tree_device(dfmm_plan_s& P, const double* points, int64_t N, double K, Tree& T, DevTree& DT);

namespace {

template <class F>
void parallel_for(int64_t n, F&& fn) {
  unsigned hc = std::thread::hardware_concurrency();
  int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hc ? hc : 1, 16));
  nt = std::min<int64_t>(nt, n);
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> th;
  for (int64_t t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (int64_t i = next++; i < n; i = next++) fn(i);
    });
  for (auto& x : th) x.join();
}

// G(x, y) in float64 (zero at coincidence).
inline void green64(double dx, double dy, double dz, double* re, double* im) {
  double r = std::sqrt(dx * dx + dy * dy + dz * dz);
  if (r == 0.0) {
    *re = *im = 0.0;
    return;
  }
  *re = std::cos(2.0 * M_PI * r) / r;
  *im = std::sin(2.0 * M_PI * r) / r;
}

int pad8(int r) { return (r + 7) / 8 * 8; }

}  // namespace

// Fragment order of an M x K complex operator for the MFMA kernel: for M-tile
// m (8 complex rows), step s4 (K / 8 of them), row-in-tile ql (8) and K quarter
// kr (4), one float4 holds the two complex entries (q, p0) and (q, p0 + 1) with
// q = 8 m + ql and p0 = kr K / 4 + 2 s4.
void pack_operator(const double* Tc, int M, int K, float* out) {
  int nm = M / 8, ns = K / 8;
  for (int m = 0; m < nm; ++m)
    for (int s4 = 0; s4 < ns; ++s4)
      for (int ql = 0; ql < 8; ++ql)
        for (int kr = 0; kr < 4; ++kr) {
          int q = 8 * m + ql, p0 = kr * (K / 4) + 2 * s4;
          float* o = out + 4 * ((((size_t(m) * ns + s4) * 8 + ql) * 4) + kr);
          o[0] = float(Tc[2 * (size_t(q) * K + p0)]);
          o[1] = float(Tc[2 * (size_t(q) * K + p0) + 1]);
          o[2] = float(Tc[2 * (size_t(q) * K + p0 + 1)]);
          o[3] = float(Tc[2 * (size_t(q) * K + p0 + 1) + 1]);
        }
}

void pack_operator64(const double* Tc, int M, int K, double* out) {
  int nm = M / 8, ns = K / 8;
  for (int m = 0; m < nm; ++m)
    for (int s4 = 0; s4 < ns; ++s4)
      for (int ql = 0; ql < 8; ++ql)
        for (int kr = 0; kr < 4; ++kr) {
          int q = 8 * m + ql, p0 = kr * (K / 4) + 2 * s4;
          double* o = out + 4 * ((((size_t(m) * ns + s4) * 8 + ql) * 4) + kr);
          o[0] = Tc[2 * (size_t(q) * K + p0)];
          o[1] = Tc[2 * (size_t(q) * K + p0) + 1];
          o[2] = Tc[2 * (size_t(q) * K + p0 + 1)];
          o[3] = Tc[2 * (size_t(q) * K + p0 + 1) + 1];
        }
}

namespace {
// Packed operators of one launch, float32 (fragment order of the float32 and
// 16-bit engines) or float64 (float64 plans); entries at the same offsets.
struct OpStore {
  bool f64;
  std::vector<float> f;
  std::vector<double> d;
  OpStore(bool f64_, size_t n) : f64(f64_) {
    if (f64) d.assign(n, 0.0);
    else f.assign(n, 0.0f);
  }
  void pack(const double* T, int M, int K, int split, size_t off) {
    if (f64) pack_operator64(T, M, K, d.data() + off);
    else pack_operator_split(T, M, K, split, f.data() + off);
  }
  void upload(DevBuf& b) {
    if (f64) b.upload(d);
    else b.upload(f);
  }
};
}  // namespace

void pack_operator_split(const double* Tc, int M, int K, int split, float* out) {
  if (split == 1) {
    pack_operator(Tc, M, K, out);
    return;
  }
  std::vector<double> T2(size_t(2) * M * 2 * K);
  for (int q = 0; q < M; ++q)
    for (int p = 0; p < K; ++p)
      for (int c = 0; c < 2; ++c) {
        const double v = Tc[2 * (size_t(q) * K + p) + c];
        const double hi = double(float(v));
        T2[2 * (size_t(q) * 2 * K + p) + c] = hi;
        T2[2 * (size_t(q) * 2 * K + K + p) + c] = v - hi;
      }
  pack_operator(T2.data(), M, 2 * K, out);
}

// float32 -> IEEE binary16 bits, round to nearest even (subnormals kept; the
// callers scale every value below 2^14, so there is no overflow)
static uint16_t f32_to_f16(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  const uint32_t sign = (x >> 16) & 0x8000u;
  x &= 0x7FFFFFFFu;
  if (x >= 0x477FF000u) return uint16_t(sign | 0x7C00u);  // rounds past 65504: infinity
  if (x < 0x38800000u) {                                   // below 2^-14: subnormal or zero
    if (x <= 0x33000000u) return uint16_t(sign);           // <= 2^-25 rounds to zero
    const uint32_t mant = (x & 0x7FFFFFu) | 0x800000u;
    const int shift = 126 - int(x >> 23);                  // value = mant 2^(e - 150) = m 2^-24
    uint32_t m = mant >> shift;
    const uint32_t rem = mant & ((1u << shift) - 1u), half = 1u << (shift - 1);
    if (rem > half || (rem == half && (m & 1u))) ++m;
    return uint16_t(sign | m);
  }
  uint32_t r = x - 0x38000000u;  // rebias the exponent from 127 to 15
  r += 0xFFFu + ((r >> 13) & 1u);
  return uint16_t(sign | (r >> 13));
}

static float f16_to_f32(uint16_t h) {
  const uint32_t sign = uint32_t(h & 0x8000u) << 16, e = (h >> 10) & 0x1Fu, m = h & 0x3FFu;
  float v;
  if (e == 0) v = std::ldexp(float(m), -24);
  else v = std::ldexp(float(m | 0x400u), int(e) - 25);
  uint32_t b;
  std::memcpy(&b, &v, 4);
  b |= sign;
  std::memcpy(&v, &b, 4);
  return v;
}

// float32 -> bfloat16 bits, round to nearest even (finite inputs)
static uint16_t f32_to_bf16(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  x += 0x7FFFu + ((x >> 16) & 1u);
  return uint16_t(x >> 16);
}

static float bf16_to_f32(uint16_t h) {
  const uint32_t b = uint32_t(h) << 16;
  float v;
  std::memcpy(&v, &b, 4);
  return v;
}

void to_half_ops(std::vector<float>& A, int64_t nops, int64_t stride, int prec, std::vector<int32_t>& aexp) {
  aexp.assign(size_t(nops), 0);
  parallel_for(nops, [&](int64_t i) {
    float* a = A.data() + size_t(i) * size_t(stride);
    int e = 0;
    if (prec == DFMM_PREC_FP16X3) {
      float mx = 0.0f;
      for (int64_t k = 0; k < stride; ++k) mx = std::max(mx, std::fabs(a[k]));
      if (mx > 0.0f) {
        int E = 0;
        (void)std::frexp(mx, &E);  // mx < 2^E
        e = 14 - E;
      }
    }
    aexp[size_t(i)] = e;
    for (int64_t k = 0; k < stride; k += 4) {
      uint16_t hi[4], lo[4];
      for (int c = 0; c < 4; ++c) {
        const float v = std::ldexp(a[k + c], e);
        if (prec == DFMM_PREC_FP16X3) {
          hi[c] = f32_to_f16(v);
          lo[c] = f32_to_f16(v - f16_to_f32(hi[c]));
        } else {
          hi[c] = f32_to_bf16(v);
          lo[c] = f32_to_bf16(v - bf16_to_f32(hi[c]));
        }
      }
      const uint32_t w[4] = {uint32_t(hi[0]) | uint32_t(hi[1]) << 16, uint32_t(hi[2]) | uint32_t(hi[3]) << 16,
                             uint32_t(lo[0]) | uint32_t(lo[1]) << 16, uint32_t(lo[2]) | uint32_t(lo[3]) << 16};
      std::memcpy(a + k, w, 16);
    }
  });
}

void build_slot_gemm(SlotGemm& S, int M, int64_t ngroups, const std::vector<int32_t>& gM,
                     const std::vector<SlotTerm>& terms, const SlotKind kinds[2], int kx_max) {
  S.M = M;
  S.KXmax = kx_max;
  S.split2 = false;
  S.ngroups = ngroups;
  S.nterms = int64_t(terms.size());
  S.flops[0] = S.flops[1] = 0.0;
  // terms grouped by destination, each group in the order given
  std::vector<int32_t> cnt(size_t(ngroups) + 1, 0);
  for (const SlotTerm& t : terms) {
    if (t.dst < 0 || t.dst >= ngroups) throw Error{DFMM_EINVAL, "slot term outside its launch"};
    ++cnt[size_t(t.dst) + 1];
  }
  for (int64_t g = 0; g < ngroups; ++g) cnt[size_t(g) + 1] += cnt[size_t(g)];
  std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1), tab(size_t(4) * terms.size());
  int kmax = 8;
  for (const SlotTerm& t : terms) {
    const SlotKind& k = kinds[t.kind];
    if (!k.G) throw Error{DFMM_EINVAL, "slot term of a kind without operators"};
    const int64_t aoff = k.G->aoff_h[size_t(t.op)];
    const int kp = k.G->kpk_h[size_t(t.op)];
    if (aoff > INT32_MAX || kp >= (1 << 12) || k.split > 3)
      throw Error{DFMM_EUNSUPPORTED, "operator table too large for the slot-form GEMM"};
    int32_t* e = &tab[size_t(4) * size_t(pos[size_t(t.dst)]++)];
    e[0] = int32_t(aoff);
    e[1] = t.src;
    e[2] = kp | (k.split << 12) | (t.kind << 14);
    e[3] = 0;
    kmax = std::max(kmax, kp);
    S.split2 = S.split2 || k.split != 1;
    S.flops[t.kind] += k.G->opflops[size_t(t.op)];
  }
  S.Kmax = kmax;
  S.max_terms = 0;
  for (int64_t g = 0; g < ngroups; ++g) S.max_terms = std::max(S.max_terms, cnt[size_t(g) + 1] - cnt[size_t(g)]);
  // launch order: the groups with the most terms first (the long ones start
  // early and the launch ends on short ones)
  std::vector<int32_t> order(static_cast<size_t>(ngroups));
  for (int64_t g = 0; g < ngroups; ++g) order[size_t(g)] = int32_t(g);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return cnt[size_t(a) + 1] - cnt[size_t(a)] > cnt[size_t(b) + 1] - cnt[size_t(b)];
  });
  S.order.upload(order);
  S.t0.upload(cnt);
  S.gm.upload(gM);
  S.terms.upload(tab);
}

// Device bytes held by a plan (every table and operator array; the apply
// workspace is separate).
static size_t gg_bytes(const GGemm& G) {
  return G.aexp.bytes + G.A.bytes + G.aoff.bytes + G.gmk.bytes + G.ops.bytes + G.v0.bytes + G.vsrc.bytes +
         G.vdst.bytes;
}
static size_t slot_bytes(const SlotGemm& S) { return S.order.bytes + S.t0.bytes + S.gm.bytes + S.terms.bytes; }
size_t plan_device_bytes(const dfmm_plan_s& P) {
  size_t b = P.pthi.bytes + P.ptlo.bytes + P.perm_d.bytes + P.leaf_start.bytes + P.leaf_of.bytes +
             P.leaf_center.bytes + P.near_start.bytes + P.near_src.bytes;
  b += P.lf.a.bytes + P.lf.a64.bytes + P.lf.V.bytes + P.lf.W.bytes + gg_bytes(P.lf.m2l) + P.lf.red_start.bytes +
       P.lf.red_idx.bytes + slot_bytes(P.lf.down);
  for (const HFLevel& H : P.hf)
    b += gg_bytes(H.m2m) + gg_bytes(H.l2l) + gg_bytes(H.m2l) + H.m2m_rs.bytes + H.m2m_ri.bytes + H.l2l_rs.bytes +
         H.l2l_ri.bytes + H.red_start.bytes + H.red_idx.bytes + slot_bytes(H.up) + slot_bytes(H.down);
  return b;
}

void build_plan(dfmm_plan_s& P, const double* points, int64_t N, double K,
                const OpSetImpl* (*get_ops)(void* ctx, int w_needed), void* ctx) {
  auto t0 = std::chrono::steady_clock::now();
  P.N = N;
  P.K = K;
  Tree T;
  DevTree DT;
  build_tree_device(P, points, N, K, T, DT);
  const int D = T.D;
  P.D = D;
  dfmm_info& info = P.info;
  std::memset(&info, 0, sizeof(info));
  const bool fp64 = P.prec == DFMM_PREC_FP64;  // float64 operators and vectors
  const bool half = P.prec == DFMM_PREC_FP16X3 || P.prec == DFMM_PREC_BF16X3;
  info.N = N;
  info.K = K;
  info.depth = D;

  // ---- exports of the tree --------------------------------------------------
  P.perm = T.perm;
  P.boxes.assign(D + 1, {});
  for (int l = 0; l <= D; ++l) {
    const auto& L = T.lv[l];
    auto& v = P.boxes[l];
    for (size_t b = 0; b < L.key.size(); ++b) {
      v.insert(v.end(), {L.cx[b], L.cy[b], L.cz[b], L.start[b], L.end[b]});
    }
    info.boxes[l] = int64_t(L.key.size());
  }

  // ---- interaction lists on every level -------------------------------------
  std::vector<std::vector<PairRec>> pairs(D + 1);
  std::vector<DevBuf> pair_fields(D + 1);
  std::vector<int64_t> npairs(D + 1, 0);
  P.pairs.assign(D + 1, {});
  int l_top = -1;
  for (int l = 1; l <= D; ++l) {
    pairs[l] = level_pairs_device(DT, D, l, pair_fields[l]);
    npairs[l] = int64_t(pairs[l].size());
    auto& v = P.pairs[l];
    for (auto& r : pairs[l]) v.insert(v.end(), {r.B, r.A, int64_t(r.din), int64_t(r.dout), 0});
    info.pairs[l] = int64_t(pairs[l].size());
    std::set<std::tuple<int64_t, int64_t, int64_t>> offs;
    for (auto& r : pairs[l]) offs.insert({r.nx, r.ny, r.nz});
    info.offsets[l] = int64_t(offs.size());
    if (l < D && !pairs[l].empty() && l_top < 0) l_top = l;
  }
  int e_top = l_top >= 0 ? (D - 1 - l_top) : -1;
  P.w_top = e_top >= 0 ? (1 << e_top) : 0;
  info.w_top = P.w_top;
  info.nlevels_hf = e_top + 1;
  const OpSetImpl& ops = *get_ops(ctx, std::max(1, P.w_top));
  info.tau = ops.tau;
  if (e_top >= 0 && (1 << e_top) > ops.w_hi)
    throw Error{DFMM_EUNSUPPORTED, "tree needs HF width " + std::to_string(1 << e_top) +
                                       " but the operator set stops at " + std::to_string(ops.w_hi)};

  // ---- near-field lists -------------------------------------------------------
  const auto& LL = T.lv[D];
  int64_t nleaf = int64_t(LL.key.size());
  std::vector<int32_t> near_start, near_src;
  near_lists_device(DT, D, near_start, near_src);
  for (int64_t b = 0; b < nleaf; ++b)
    for (int32_t j = near_start[b]; j < near_start[b + 1]; ++j) {
      const int64_t a = near_src[j];
      P.near.push_back(b);
      P.near.push_back(a);
      info.near_point_pairs += (LL.end[b] - LL.start[b]) * (LL.end[a] - LL.start[a]);
    }
  info.near_pairs = int64_t(near_src.size());
  P.near_start.upload(near_start);
  P.near_src.upload(near_src);

  // ---- needed directions (top-down closure) ----------------------------------
  P.out_slots.assign(D + 1, {});
  P.in_slots.assign(D + 1, {});
  std::vector<SlotIndex> OS, IS;
  slot_closure_device(DT, D, e_top >= 0 ? l_top : -1, pair_fields, npairs, OS, IS);
  if (e_top >= 0) {
    for (int l = l_top; l < D; ++l) {
      for (auto& s : OS[l].list) P.out_slots[l].insert(P.out_slots[l].end(), {s.first, int64_t(s.second)});
      for (auto& s : IS[l].list) P.in_slots[l].insert(P.in_slots[l].end(), {s.first, int64_t(s.second)});
      info.out_slots[l] = int64_t(OS[l].list.size());
      info.in_slots[l] = int64_t(IS[l].list.size());
    }
  }

  // ---- LF level tables ------------------------------------------------------------
  const Skel& sl = ops.lf;
  int Rlf = pad8(sl.r);
  P.lf.R = Rlf;
  P.lf.r = sl.r;
  P.lf.nleaf = nleaf;
  info.rank[D] = Rlf;
  {
    std::vector<float> a4(size_t(4) * Rlf, 0.0f);
    std::vector<double> a64(size_t(4) * Rlf, 0.0), DT(size_t(2) * Rlf * Rlf, 0.0);
    for (int i = 0; i < sl.r; ++i)
      for (int k = 0; k < 3; ++k) {
        a4[4 * i + k] = float(sl.a[3 * i + k]);
        a64[4 * i + k] = sl.a[3 * i + k];
      }
    for (int q = 0; q < sl.r; ++q)
      for (int p = 0; p < sl.r; ++p) {  // DT[p][q] = D[q][p]
        DT[2 * (size_t(p) * Rlf + q)] = sl.D[2 * (size_t(q) * sl.r + p)];
        DT[2 * (size_t(p) * Rlf + q) + 1] = sl.D[2 * (size_t(q) * sl.r + p) + 1];
      }
    P.lf.a.upload(a4);
    P.lf.a64.upload(a64);
    build_leaf_weights(P, T.pts, DT);
  }

  // M2L of one level: pairs grouped by offset n; one operator per group,
  // G(b^{l_in}, n w + b^{l_out}) D^{l_out} (maps outgoing check potentials of A to
  // incoming check potentials of B); the pair outputs are summed per in-slot.
  auto build_m2l = [&](const std::vector<PairRec>& pr, double w, int R,
                       const std::vector<const Skel*>& skin, const SlotIndex* osl, const SlotIndex* isl,
                       int64_t nin, GGemm& G, DevBuf& rs, DevBuf& ri, int64_t& ngroups, double& flops,
                       int split, std::vector<SlotTerm>& sterms) {
    // algorithmic bytes: each group's operator once (complex64, unpadded), each
    // source slot read once and each target slot read and written once, per rhs
    double& bytes_op = info.bytes_m2l_op;
    double& bytes_vec = info.bytes_m2l_vec;
    {
      std::set<std::pair<int64_t, int>> srcs, tgts;
      for (const PairRec& r : pr) {
        srcs.insert({r.A, r.dout});
        tgts.insert({r.B, r.din});
      }
      for (const auto& s : srcs) bytes_vec += 8.0 * skin[s.second < 0 ? 0 : s.second]->r;
      for (const auto& t : tgts) bytes_vec += 16.0 * skin[t.second < 0 ? 0 : t.second]->r;
    }
    std::map<std::tuple<int64_t, int64_t, int64_t>, std::vector<int64_t>> g;
    for (size_t i = 0; i < pr.size(); ++i) g[{pr[i].nx, pr[i].ny, pr[i].nz}].push_back(int64_t(i));
    ngroups = int64_t(g.size());
    std::vector<int32_t> v0(1, 0), vsrc, opsv, pos_of(pr.size());
    std::vector<std::tuple<int64_t, int64_t, int64_t>> keys;
    std::vector<int64_t> rep;
    flops = 0.0;
    for (auto& kv : g) {
      keys.push_back(kv.first);
      rep.push_back(kv.second.front());
      {
        const PairRec& r0 = pr[kv.second.front()];
        bytes_op += 8.0 * skin[r0.din < 0 ? 0 : r0.din]->r * skin[r0.dout < 0 ? 0 : r0.dout]->r;
      }
      opsv.push_back(int32_t(keys.size() - 1));
      for (int64_t i : kv.second) {
        const PairRec& r = pr[i];
        pos_of[i] = int32_t(vsrc.size());
        vsrc.push_back(int32_t(osl ? osl->at(r.A, r.dout) : r.A));
        sterms.push_back({int32_t(isl ? isl->at(r.B, r.din) : r.B), int32_t(keys.size() - 1), vsrc.back(), 0});
        flops += 8.0 * skin[r.din < 0 ? 0 : r.din]->r * skin[r.dout < 0 ? 0 : r.dout]->r;
      }
      v0.push_back(int32_t(vsrc.size()));
    }
    std::vector<std::vector<int32_t>> per(nin);
    for (size_t i = 0; i < pr.size(); ++i) {
      const PairRec& r = pr[i];
      per[isl ? isl->at(r.B, r.din) : r.B].push_back(pos_of[i]);
    }
    std::vector<int32_t> rstart(1, 0), ridx;
    for (auto& v : per) {
      std::sort(v.begin(), v.end());
      ridx.insert(ridx.end(), v.begin(), v.end());
      rstart.push_back(int32_t(ridx.size()));
    }
    std::vector<int32_t> vdst(vsrc.size());
    for (size_t i = 0; i < vdst.size(); ++i) vdst[i] = int32_t(i);
    const int RK = kpad(R, P.prec);  // packed K of every operator of the launch
    OpStore At(fp64, size_t(2) * R * RK * split * ngroups);
    std::vector<int32_t> gmk(size_t(2) * ngroups);
    std::vector<int64_t> aoff(ngroups);
    parallel_for(ngroups, [&](int64_t gi) {
      const PairRec& r = pr[rep[gi]];
      const Skel* si = skin[r.din < 0 ? 0 : r.din];
      const Skel* so = skin[r.dout < 0 ? 0 : r.dout];
      double sx = double(std::get<0>(keys[gi])) * w, sy = double(std::get<1>(keys[gi])) * w,
             sz = double(std::get<2>(keys[gi])) * w;
      const int Mg = pad8(si->r), Kg = pad8(so->r);
      gmk[2 * gi] = Mg;
      gmk[2 * gi + 1] = Kg * split;
      aoff[gi] = int64_t(gi) * R * RK * split / 2;
      const int Kp = kpad(Kg, P.prec);
      std::vector<double> G(size_t(2) * so->r), T(size_t(2) * Mg * Kp, 0.0);
      for (int q = 0; q < si->r; ++q) {
        for (int p = 0; p < so->r; ++p)
          green64(si->b[3 * q] - (sx + so->b[3 * p]), si->b[3 * q + 1] - (sy + so->b[3 * p + 1]),
                  si->b[3 * q + 2] - (sz + so->b[3 * p + 2]), &G[2 * p], &G[2 * p + 1]);
        for (int j = 0; j < so->r; ++j) {
          double re = 0.0, im = 0.0;
          for (int p = 0; p < so->r; ++p) {
            double gr = G[2 * p], gi2 = G[2 * p + 1];
            double dr = so->D[2 * (size_t(p) * so->r + j)], di = so->D[2 * (size_t(p) * so->r + j) + 1];
            re += gr * dr - gi2 * di;
            im += gr * di + gi2 * dr;
          }
          T[2 * (size_t(q) * Kp + j)] = re;
          T[2 * (size_t(q) * Kp + j) + 1] = im;
        }
      }
      At.pack(T.data(), Mg, Kp, split, size_t(2) * R * RK * split * gi);
    });
    if (half) {
      std::vector<int32_t> aexp;
      to_half_ops(At.f, ngroups, int64_t(2) * R * RK * split, P.prec, aexp);
      G.aexp.upload(aexp);
    }
    G.prec = P.prec;
    G.M = R;
    G.K = R;
    G.T = 1;
    G.split = split;
    G.acc64 = P.precise;
    G.ngroups = ngroups;
    G.nvec = int64_t(vsrc.size());
    G.nops = ngroups;
    At.upload(G.A);
    G.aoff.upload(aoff);
    G.gmk.upload(gmk);
    G.ops.upload(opsv);
    G.v0.upload(v0);
    G.v0_h = v0;
    G.vsrc.upload(vsrc);
    G.vdst.upload(vdst);
    G.aoff_h = aoff;
    G.kpk_h.resize(size_t(ngroups));
    G.opflops.resize(size_t(ngroups));
    for (int64_t gi = 0; gi < ngroups; ++gi) {
      G.kpk_h[size_t(gi)] = kpad(gmk[2 * gi + 1] / split, P.prec) * split;
      const PairRec& r = pr[rep[gi]];
      G.opflops[size_t(gi)] = 8.0 * skin[r.din < 0 ? 0 : r.din]->r * skin[r.dout < 0 ? 0 : r.dout]->r;
    }
    rs.upload(rstart);
    ri.upload(ridx);
  };

  // slot-form term lists: M2L pairs and L2L terms of the leaves and of every HF level
  std::vector<SlotTerm> lf_terms;
  std::vector<std::vector<SlotTerm>> down_terms(size_t(e_top + 1)), up_terms(size_t(e_top + 1));
  {
    std::vector<const Skel*> s1{&sl};
    P.lf.npairs = int64_t(pairs[D].size());
    build_m2l(pairs[D], 0.5, Rlf, s1, nullptr, nullptr, nleaf, P.lf.m2l, P.lf.red_start, P.lf.red_idx,
              P.lf.ngroups, P.lf.flops, 1, lf_terms);
    info.flops_m2l_lf = P.lf.flops;
    info.flops_m2l_level[D] = P.lf.flops;
  }

  // ---- HF levels ----------------------------------------------------------------
  // precise plans split the directional operators into float32 hi + lo parts
  const int hf_split = P.precise ? 2 : 1;
  P.hf.clear();
  P.hf.resize(e_top + 1);
  for (int e = e_top; e >= 0; --e) {
    HFLevel& H = P.hf[e];
    int l = D - 1 - e;
    int64_t w = int64_t(1) << e;
    H.l = l;
    H.e = e;
    const auto& sk = ops.hf[e];
    int rmax = 0;
    for (auto& s : sk) rmax = std::max(rmax, s.r);
    H.R = pad8(rmax);
    info.rank[l] = H.R;
    std::vector<const Skel*> child_sk;
    if (e == 0) {
      H.Rc = Rlf;
    } else {
      int rc = 0;
      for (auto& s : ops.hf[e - 1]) rc = std::max(rc, s.r);
      H.Rc = pad8(rc);
      for (auto& s : ops.hf[e - 1]) child_sk.push_back(&s);
    }
    H.nout = int64_t(OS[l].list.size());
    H.nin = int64_t(IS[l].list.size());
    H.npairs = int64_t(pairs[l].size());
    const auto& L = T.lv[l];
    const auto& C = T.lv[l + 1];

    // Per (dir, octant): upward G(a^{w,l} - delta_o, b^c) D^c (R x Rc) maps the
    // child's outgoing check potentials to the parent's; downward
    // G(b^c + delta_o, a^{w,l}) (D^{w,l})^T (Rc x R) maps the parent's incoming
    // check potentials to the child's (c = the child skeleton of wedge l).
    int ndir = int(6 * w * w);
    const int KU = kpad(H.Rc, P.prec), KD = kpad(H.R, P.prec);  // packed K of the up / down operators
    OpStore Mu(fp64, size_t(2) * ndir * 8 * H.R * KU * hf_split);
    OpStore Md(fp64, size_t(2) * ndir * 8 * H.Rc * KD * hf_split);
    std::vector<char> dir_used(ndir, 0);
    for (auto& s : OS[l].list) dir_used[s.second] = 1;
    for (auto& s : IS[l].list) dir_used[s.second] = 1;
    std::vector<int32_t> op_ms(size_t(ndir) * 8, 8), op_mc(size_t(ndir) * 8, 8);  // padded ranks per op
    std::vector<double> op_fl(size_t(ndir) * 8, 0.0);  // 8 r_s r_c per op (unpadded)
    double wc = double(w) / 2.0;
    parallel_for(int64_t(ndir) * 8, [&](int64_t id) {
      int d = int(id / 8), o = int(id % 8);
      if (!dir_used[d]) return;
      const Skel& s = sk[d];
      const Skel& c = e == 0 ? sl : *child_sk[direction_down(d, w)];
      double dx = ((o & 1) - 0.5) * wc, dy = (((o >> 1) & 1) - 0.5) * wc, dz = (((o >> 2) & 1) - 0.5) * wc;
      std::vector<double> G(size_t(2) * s.r * c.r);
      for (int p = 0; p < s.r; ++p)
        for (int j = 0; j < c.r; ++j)
          green64(s.a[3 * p] - dx - c.b[3 * j], s.a[3 * p + 1] - dy - c.b[3 * j + 1],
                  s.a[3 * p + 2] - dz - c.b[3 * j + 2], &G[2 * (size_t(p) * c.r + j)],
                  &G[2 * (size_t(p) * c.r + j) + 1]);
      const int Ms = pad8(s.r), Mc = pad8(c.r);
      op_ms[id] = Ms;
      op_mc[id] = Mc;
      op_fl[id] = 8.0 * s.r * c.r;
      const int Kpu = kpad(Mc, P.prec), Kpd = kpad(Ms, P.prec);
      std::vector<double> up(size_t(2) * Ms * Kpu, 0.0), dn(size_t(2) * Mc * Kpd, 0.0);
      for (int p = 0; p < s.r; ++p)
        for (int k = 0; k < c.r; ++k) {  // (G D^c)[p][k]
          double re = 0.0, im = 0.0;
          for (int j = 0; j < c.r; ++j) {
            double gr = G[2 * (size_t(p) * c.r + j)], gi = G[2 * (size_t(p) * c.r + j) + 1];
            double dr = c.D[2 * (size_t(j) * c.r + k)], di = c.D[2 * (size_t(j) * c.r + k) + 1];
            re += gr * dr - gi * di;
            im += gr * di + gi * dr;
          }
          up[2 * (size_t(p) * Kpu + k)] = re;
          up[2 * (size_t(p) * Kpu + k) + 1] = im;
        }
      for (int j = 0; j < c.r; ++j)
        for (int q = 0; q < s.r; ++q) {  // (G^T D^T)[j][q] = sum_p G[p][j] D[q][p]
          double re = 0.0, im = 0.0;
          for (int p = 0; p < s.r; ++p) {
            double gr = G[2 * (size_t(p) * c.r + j)], gi = G[2 * (size_t(p) * c.r + j) + 1];
            double dr = s.D[2 * (size_t(q) * s.r + p)], di = s.D[2 * (size_t(q) * s.r + p) + 1];
            re += gr * dr - gi * di;
            im += gr * di + gi * dr;
          }
          dn[2 * (size_t(j) * Kpd + q)] = re;
          dn[2 * (size_t(j) * Kpd + q) + 1] = im;
        }
      Mu.pack(up.data(), Ms, Kpu, hf_split, size_t(2) * id * H.R * KU * hf_split);
      Md.pack(dn.data(), Mc, Kpd, hf_split, size_t(2) * id * H.Rc * KD * hf_split);
    });

    // HF-M2M and HF-L2L as pair lists: one pair per (parent slot, child), grouped
    // by the (wedge, octant) operator it uses; the GEMM writes one output per
    // pair and a reduction sums the pairs of each destination slot.
    auto finish_pairs = [&](GGemm& G, std::vector<std::vector<std::pair<int32_t, int32_t>>>& by_op, int M,
                            int K, int64_t nops, int64_t ndst, DevBuf& rs, DevBuf& ri, int64_t& npairs,
                            const std::vector<int32_t>& opM, const std::vector<int32_t>& opK) {
      // by_op[op] = list of (source vector, destination slot)
      std::vector<int32_t> v0(1, 0), vsrc, vdst, opsv, gmk;
      std::vector<int64_t> aoff(nops);
      for (int64_t op = 0; op < nops; ++op) aoff[op] = op * int64_t(M) * kpad(K, P.prec) * hf_split / 2;
      std::vector<std::vector<int32_t>> per(ndst);
      for (int64_t op = 0; op < int64_t(by_op.size()); ++op) {
        if (by_op[op].empty()) continue;
        opsv.push_back(int32_t(op));
        gmk.push_back(opM[op]);
        gmk.push_back(opK[op] * hf_split);
        for (auto& sd : by_op[op]) {
          per[sd.second].push_back(int32_t(vsrc.size()));
          vsrc.push_back(sd.first);
          vdst.push_back(int32_t(vdst.size()));
        }
        v0.push_back(int32_t(vsrc.size()));
      }
      std::vector<int32_t> rstart(1, 0), ridx;
      for (auto& v : per) {
        ridx.insert(ridx.end(), v.begin(), v.end());
        rstart.push_back(int32_t(ridx.size()));
      }
      G.M = M;
      G.K = K;
      G.T = 1;
      G.split = hf_split;
      G.acc64 = P.precise;
      G.prec = P.prec;
      G.ngroups = int64_t(v0.size()) - 1;
      G.nvec = int64_t(vsrc.size());
      G.nops = nops;
      G.aoff.upload(aoff);
      G.gmk.upload(gmk);
      G.ops.upload(opsv);
      G.v0.upload(v0);
      G.v0_h = v0;
      G.vsrc.upload(vsrc);
      G.vdst.upload(vdst);
      G.aoff_h = aoff;
      G.kpk_h.resize(size_t(nops));
      for (int64_t op = 0; op < nops; ++op) G.kpk_h[size_t(op)] = kpad(opK[size_t(op)], P.prec) * hf_split;
      G.opflops = op_fl;
      rs.upload(rstart);
      ri.upload(ridx);
      npairs = G.nvec;
    };
    {
      std::vector<std::vector<std::pair<int32_t, int32_t>>> by_op(size_t(ndir) * 8);
      for (int64_t i = 0; i < H.nout; ++i) {
        auto [b, d] = OS[l].list[i];
        for (int64_t c = L.cbeg[b]; c < L.cend[b]; ++c) {
          int32_t src = int32_t(e == 0 ? c : OS[l + 1].at(c, direction_down(d, w)));
          by_op[size_t(d) * 8 + C.octant[c]].push_back({src, int32_t(i)});
          up_terms[size_t(e)].push_back({int32_t(i), int32_t(size_t(d) * 8 + C.octant[c]), src, 0});
        }
      }
      if (half) {
        std::vector<int32_t> aexp;
        to_half_ops(Mu.f, int64_t(ndir) * 8, int64_t(2) * H.R * KU * hf_split, P.prec, aexp);
        H.m2m.aexp.upload(aexp);
      }
      Mu.upload(H.m2m.A);
      finish_pairs(H.m2m, by_op, H.R, H.Rc, int64_t(ndir) * 8, H.nout, H.m2m_rs, H.m2m_ri, H.m2m_npairs, op_ms,
                   op_mc);
    }
    {
      std::vector<std::vector<std::pair<int32_t, int32_t>>> by_op(size_t(ndir) * 8);
      if (e == 0) {
        H.nchild_in = nleaf;
        for (int64_t c = 0; c < nleaf; ++c) {
          int64_t p = C.parent[c];
          for (int d = 0; d < 6; ++d) {
            int64_t sidx = IS[l].at(p, d);
            if (sidx >= 0) {
              by_op[size_t(d) * 8 + C.octant[c]].push_back({int32_t(sidx), int32_t(c)});
              lf_terms.push_back({int32_t(c), int32_t(size_t(d) * 8 + C.octant[c]), int32_t(sidx), 1});
            }
          }
        }
      } else {
        int64_t wc_i = w / 2;
        H.nchild_in = int64_t(IS[l + 1].list.size());
        for (int64_t i = 0; i < H.nchild_in; ++i) {
          auto [c, dc] = IS[l + 1].list[i];
          int64_t p = C.parent[c];
          int64_t face = dc / (wc_i * wc_i), rem = dc % (wc_i * wc_i);
          int64_t ci = rem / wc_i, cj = rem % wc_i;
          for (int di = 0; di < 2; ++di)
            for (int dj = 0; dj < 2; ++dj) {
              int d = int((face * w + 2 * ci + di) * w + 2 * cj + dj);
              int64_t sidx = IS[l].at(p, d);
              if (sidx >= 0) {
                by_op[size_t(d) * 8 + C.octant[c]].push_back({int32_t(sidx), int32_t(i)});
                down_terms[size_t(e - 1)].push_back({int32_t(i), int32_t(size_t(d) * 8 + C.octant[c]),
                                                     int32_t(sidx), 1});
              }
            }
        }
      }
      // algorithmic bytes of the L2L terms: each (wedge, octant) operator used
      // once (complex64, unpadded: 8 r_c r_s bytes, the same number as its
      // flops) and each parent incoming slot read once per rhs
      {
        std::set<int32_t> parents;
        for (int64_t op = 0; op < int64_t(by_op.size()); ++op) {
          if (by_op[size_t(op)].empty()) continue;
          info.bytes_l2l_op += op_fl[size_t(op)];
          for (auto& sd : by_op[size_t(op)]) parents.insert(sd.first);
        }
        for (int32_t sidx : parents) info.bytes_l2l_vec += 8.0 * sk[size_t(IS[l].list[size_t(sidx)].second)].r;
      }
      if (half) {
        std::vector<int32_t> aexp;
        to_half_ops(Md.f, int64_t(ndir) * 8, int64_t(2) * H.Rc * KD * hf_split, P.prec, aexp);
        H.l2l.aexp.upload(aexp);
      }
      Md.upload(H.l2l.A);
      finish_pairs(H.l2l, by_op, H.Rc, H.R, int64_t(ndir) * 8, H.nchild_in, H.l2l_rs, H.l2l_ri, H.l2l_npairs,
                   op_mc, op_ms);
    }
    // M2L
    std::vector<const Skel*> sp;
    for (auto& s : sk) sp.push_back(&s);
    build_m2l(pairs[l], double(w), H.R, sp, &OS[l], &IS[l], H.nin, H.m2l, H.red_start, H.red_idx, H.ngroups,
              H.flops, hf_split, down_terms[size_t(e)]);
    info.flops_m2l_hf += H.flops;
    info.flops_m2l_level[l] = H.flops;
  }
  // algorithmic flops of the tree transfers per right-hand side (8 r_out r_in per term)
  for (int e = 0; e <= e_top; ++e) {
    for (const SlotTerm& t : up_terms[size_t(e)]) info.flops_m2m += P.hf[size_t(e)].m2m.opflops[size_t(t.op)];
    for (const SlotTerm& t : down_terms[size_t(e)])
      if (t.kind == 1) info.flops_l2l += P.hf[size_t(e + 1)].l2l.opflops[size_t(t.op)];
  }
  for (const SlotTerm& t : lf_terms)
    if (t.kind == 1) info.flops_l2l += P.hf[0].l2l.opflops[size_t(t.op)];

  // ---- slot-form tables (fast float32 plans; used from 16 right-hand sides) -------
  if ((!P.precise && P.prec == DFMM_PREC_FP32) || fp64) {
    auto slot_m = [&](int l, int64_t n, bool in) {  // padded rows of each slot's skeleton
      std::vector<int32_t> gm(static_cast<size_t>(n));
      const int e = D - 1 - l;
      for (int64_t i = 0; i < n; ++i)
        gm[size_t(i)] = pad8(ops.hf[e][(in ? IS[l] : OS[l]).list[size_t(i)].second].r);
      return gm;
    };
    for (int e = 0; e <= e_top; ++e) {
      HFLevel& H = P.hf[size_t(e)];
      const int l = H.l;
      SlotKind up[2] = {{&H.m2m, hf_split}, {nullptr, 1}};
      build_slot_gemm(H.up, H.R, H.nout, slot_m(l, H.nout, false), up_terms[size_t(e)], up,
                      e == 0 ? Rlf : P.hf[size_t(e - 1)].R);
      SlotKind dn[2] = {{&H.m2l, hf_split}, {e < e_top ? &P.hf[size_t(e + 1)].l2l : nullptr, hf_split}};
      build_slot_gemm(H.down, H.R, H.nin, slot_m(l, H.nin, true), down_terms[size_t(e)], dn,
                      std::max(H.R, e < e_top ? P.hf[size_t(e + 1)].R : 0));
    }
    SlotKind dn[2] = {{&P.lf.m2l, 1}, {e_top >= 0 ? &P.hf[0].l2l : nullptr, hf_split}};
    build_slot_gemm(P.lf.down, Rlf, nleaf, std::vector<int32_t>(size_t(nleaf), Rlf), lf_terms, dn,
                    std::max(Rlf, e_top >= 0 ? P.hf[0].R : 0));
  }

  info.device_bytes = int64_t(plan_device_bytes(P));
  auto t1 = std::chrono::steady_clock::now();
  P.plan_seconds = std::chrono::duration<double>(t1 - t0).count();
  info.plan_seconds = P.plan_seconds;
}

}  // namespace dfmm
