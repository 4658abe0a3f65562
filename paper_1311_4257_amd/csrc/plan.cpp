// Plan construction: octree, interaction lists, wedges, needed directions and
// translation tables (Section 2.2, Algorithm 1), resident on the device.
#include <algorithm>
#include <array>
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

void build_tree_device(dfmm_plan_s& P, const double* points, int64_t N, double K, Tree& T, DevTree& DT,
                       int extra);

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

// ---- adaptive low-frequency tree (Section 2.2) ---------------------------------
// The device box tables cover every level down to the sort depth, boxes under
// leaves included.  A box of level l > D exists when its parent exists and is
// split; a box of width <= 1/2 is split when it holds more than leaf_max points
// and is above the deepest level.  Kept boxes keep the Morton order.
struct AdaptiveLevels {
  int D = 0, Dmax = 0;
  std::vector<std::vector<int64_t>> box;    // per level (index l - D): device-table index of each kept box
  std::vector<std::vector<char>> split;     // per kept box: it has children
  std::vector<std::vector<int64_t>> par;    // per kept box of level > D: kept index of the parent
  std::vector<std::vector<int64_t>> c0, c1; // per kept box: range of its kept children one level down
  std::vector<int64_t> base;                // LF vector index of the first kept box of each level
  std::vector<std::map<std::tuple<int64_t, int64_t, int64_t>, int64_t>> at;  // coordinates -> kept index
};

AdaptiveLevels adaptive_levels(const Tree& T, int D, int leaf_max) {
  AdaptiveLevels A;
  A.D = A.Dmax = D;
  const int Dk = int(T.lv.size()) - 1;
  std::vector<int64_t> kprev;  // device index of level l - 1 -> kept index (-1: not kept)
  for (int l = D; l <= Dk; ++l) {
    const auto& L = T.lv[size_t(l)];
    const int64_t nu = int64_t(L.key.size());
    std::vector<int64_t> kidx(size_t(nu), -1), box, par;
    std::vector<char> sp;
    for (int64_t u = 0; u < nu; ++u) {
      int64_t pk = -1;
      if (l > D) {
        pk = kprev[size_t(L.parent[size_t(u)])];
        if (pk < 0 || !A.split.back()[size_t(pk)]) continue;
      }
      kidx[size_t(u)] = int64_t(box.size());
      box.push_back(u);
      par.push_back(pk);
      sp.push_back(char(l < Dk && L.end[size_t(u)] - L.start[size_t(u)] > leaf_max));
    }
    if (box.empty()) break;
    const bool any_split = std::any_of(sp.begin(), sp.end(), [](char c) { return c != 0; });
    A.box.push_back(std::move(box));
    A.split.push_back(std::move(sp));
    A.par.push_back(std::move(par));
    A.Dmax = l;
    kprev = std::move(kidx);
    if (!any_split) break;
  }
  const int nl = A.Dmax - D + 1;
  A.c0.assign(size_t(nl), {});
  A.c1.assign(size_t(nl), {});
  A.base.assign(size_t(nl), 0);
  A.at.assign(size_t(nl), {});
  int64_t base = 0;
  for (int k = 0; k < nl; ++k) {
    const size_t nb = A.box[size_t(k)].size();
    A.base[size_t(k)] = base;
    base += int64_t(nb);
    A.c0[size_t(k)].assign(nb, 0);
    A.c1[size_t(k)].assign(nb, 0);
    const auto& L = T.lv[size_t(D + k)];
    for (size_t b = 0; b < nb; ++b) {
      const int64_t u = A.box[size_t(k)][b];
      A.at[size_t(k)][{L.cx[size_t(u)], L.cy[size_t(u)], L.cz[size_t(u)]}] = int64_t(b);
    }
    if (k > 0) {  // children of a box are consecutive in the Morton order
      for (size_t c = 0; c < nb; ++c) {
        const int64_t p = A.par[size_t(k)][c];
        if (A.c1[size_t(k - 1)][size_t(p)] == 0) A.c0[size_t(k - 1)][size_t(p)] = int64_t(c);
        A.c1[size_t(k - 1)][size_t(p)] = int64_t(c) + 1;
      }
    }
  }
  return A;
}

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
    if (aoff > INT32_MAX || kp >= (1 << 12) || kp < 8 || kp % 8 != 0 || k.split > 3)
      throw Error{DFMM_EUNSUPPORTED, "operator table too large for the slot-form GEMM"};
    int32_t* e = &tab[size_t(4) * size_t(pos[size_t(t.dst)]++)];
    e[0] = int32_t(aoff);
    e[1] = t.src;
    e[2] = kp | (k.split << 12) | (t.kind << 14);
    // column staging divides a thread's index (< 2^11) by the term's float4 per
    // column (kp / 2 < 2^11): the quotient is (idx * e[3]) >> 23 exactly for
    // e[3] = ceil(2^23 / (kp / 2)), since idx times the rounding excess is < 2^23
    e[3] = int32_t(((1u << 23) + uint32_t(kp / 2) - 1) / uint32_t(kp / 2));
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
  size_t b = P.pthi.bytes + P.ptlo.bytes + P.perm_d.bytes + P.iperm_d.bytes + P.leaf_start.bytes + P.leaf_of.bytes +
             P.leaf_center.bytes + P.near_start.bytes + P.near_src.bytes;
  b += P.lf.a.bytes + P.lf.a64.bytes + P.lf.V.bytes + P.lf.W.bytes + gg_bytes(P.lf.m2l) + P.lf.red_start.bytes +
       P.lf.red_idx.bytes + slot_bytes(P.lf.down);
  for (const HFLevel& H : P.hf)
    b += gg_bytes(H.m2m) + gg_bytes(H.l2l) + gg_bytes(H.m2l) + H.m2m_rs.bytes + H.m2m_ri.bytes + H.l2l_rs.bytes +
         H.l2l_ri.bytes + H.red_start.bytes + H.red_idx.bytes + slot_bytes(H.up) + slot_bytes(H.down);
  b += P.leaf_gid.bytes;
  for (const LFDeep& Q : P.lfd)
    b += gg_bytes(Q.m2l) + gg_bytes(Q.m2m) + gg_bytes(Q.l2l) + Q.red_start.bytes + Q.red_idx.bytes +
         slot_bytes(Q.up) + slot_bytes(Q.down) + Q.up_dst.bytes;
  return b;
}

void build_plan(dfmm_plan_s& P, const double* points, int64_t N, double K,
                const OpSetImpl* (*get_ops)(void* ctx, int w_needed),
                const std::vector<Skel>* (*get_lf_deep)(void* ctx, int n), void* ctx) {
  auto t0 = std::chrono::steady_clock::now();
  P.N = N;
  P.K = K;
  Tree T;
  DevTree DT;
  const bool adaptive = P.leaf_max > 0;
  build_tree_device(P, points, N, K, T, DT, adaptive ? P.lf_levels : 0);
  const int D = T.D;
  P.D = D;
  dfmm_info& info = P.info;
  std::memset(&info, 0, sizeof(info));
  const bool fp64 = P.prec == DFMM_PREC_FP64;  // float64 operators and vectors
  const bool half = P.prec == DFMM_PREC_FP16X3 || P.prec == DFMM_PREC_BF16X3;
  info.N = N;
  info.K = K;
  info.depth = D;
  info.depth_max = D;

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
  const int64_t nD = int64_t(LL.key.size());  // boxes of width 1/2
  int64_t nleaf = nD;
  std::vector<int32_t> near_start, near_src;
  AdaptiveLevels AL;
  int nl = 1;                                        // LF levels D .. D + nl - 1
  std::vector<int64_t> leaf_lv;                      // adaptive: LF level index of each leaf
  std::vector<std::vector<PairRec>> dpairs;          // adaptive: M2L pairs of the levels below D
  if (!adaptive) {
    near_lists_device(DT, D, near_start, near_src);
    for (int64_t b = 0; b < nleaf; ++b)
      for (int32_t j = near_start[b]; j < near_start[b + 1]; ++j) {
        const int64_t a = near_src[j];
        P.near.push_back(b);
        P.near.push_back(a);
        info.near_point_pairs += (LL.end[b] - LL.start[b]) * (LL.end[a] - LL.start[a]);
      }
    P.nlfbox = nD;
  } else {
    // adaptive low-frequency part (Section 2.2), built on the host from the
    // device box tables: kept boxes, leaves in point order, their LF vectors
    AL = adaptive_levels(T, D, P.leaf_max);
    nl = AL.Dmax - D + 1;
    auto coords = [&](int l, int64_t u) {
      const auto& L = T.lv[size_t(l)];
      return std::array<int64_t, 3>{L.cx[size_t(u)], L.cy[size_t(u)], L.cz[size_t(u)]};
    };
    struct LeafRec {
      int64_t k, b, s, e;  // LF level index, kept box, point range
    };
    std::vector<LeafRec> lv;
    std::vector<std::vector<int64_t>> leaf_at(static_cast<size_t>(nl));
    for (int k = 0; k < nl; ++k) {
      const auto& L = T.lv[size_t(D + k)];
      leaf_at[size_t(k)].assign(AL.box[size_t(k)].size(), -1);
      for (size_t b = 0; b < AL.box[size_t(k)].size(); ++b)
        if (!AL.split[size_t(k)][b]) {
          const int64_t u = AL.box[size_t(k)][b];
          lv.push_back({k, int64_t(b), L.start[size_t(u)], L.end[size_t(u)]});
        }
    }
    std::sort(lv.begin(), lv.end(), [](const LeafRec& a, const LeafRec& b) { return a.s < b.s; });
    nleaf = int64_t(lv.size());
    std::vector<int64_t> lstart(static_cast<size_t>(nleaf));
    for (int64_t i = 0; i < nleaf; ++i) {
      leaf_at[size_t(lv[size_t(i)].k)][size_t(lv[size_t(i)].b)] = i;
      lstart[size_t(i)] = lv[size_t(i)].s;
    }
    P.nlfbox = AL.base.back() + int64_t(AL.box.back().size());
    std::vector<int32_t> ls, gid, lof(static_cast<size_t>(N));
    std::vector<float> lc(size_t(4) * size_t(nleaf), 0.0f);
    int mx = 0;
    P.leaves.clear();
    for (int64_t i = 0; i < nleaf; ++i) {
      const LeafRec& r = lv[size_t(i)];
      const int l = D + int(r.k);
      const int64_t g = AL.base[size_t(r.k)] + r.b;
      ls.push_back(int32_t(r.s));
      gid.push_back(int32_t(g));
      const auto c = coords(l, AL.box[size_t(r.k)][size_t(r.b)]);
      const double w = K / std::ldexp(1.0, l);
      for (int t = 0; t < 3; ++t) lc[size_t(4 * i + t)] = float((double(c[size_t(t)]) + 0.5) * w - K / 2.0);
      mx = std::max<int>(mx, int(r.e - r.s));
      for (int64_t j = r.s; j < r.e; ++j) lof[size_t(j)] = int32_t(g);
      P.leaves.insert(P.leaves.end(), {int64_t(l), r.b, r.s, r.e});
      leaf_lv.push_back(r.k);
    }
    ls.push_back(int32_t(N));
    P.leaf_start.upload(ls);
    P.leaf_gid.upload(gid);
    P.leaf_center.upload(lc);
    P.leaf_of.upload(lof);
    P.max_leaf_pts = mx;
    // near field: leaves whose boxes at the coarser of their two levels are
    // adjacent (or equal); the finer leaves under an adjacent split box are the
    // leaves whose first point lies in that box's point range
    near_start.push_back(0);
    for (int64_t i = 0; i < nleaf; ++i) {
      const LeafRec& B = lv[size_t(i)];
      const int lb = D + int(B.k);
      const auto cb = coords(lb, AL.box[size_t(B.k)][size_t(B.b)]);
      std::vector<int32_t> src;
      for (int la = D; la <= lb; ++la) {
        const int sh = lb - la, ka = la - D;
        for (int dx = -1; dx <= 1; ++dx)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
              auto it = AL.at[size_t(ka)].find({(cb[0] >> sh) + dx, (cb[1] >> sh) + dy, (cb[2] >> sh) + dz});
              if (it != AL.at[size_t(ka)].end() && !AL.split[size_t(ka)][size_t(it->second)])
                src.push_back(int32_t(leaf_at[size_t(ka)][size_t(it->second)]));
            }
      }
      const auto& L = T.lv[size_t(lb)];
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            auto it = AL.at[size_t(B.k)].find({cb[0] + dx, cb[1] + dy, cb[2] + dz});
            if (it == AL.at[size_t(B.k)].end() || !AL.split[size_t(B.k)][size_t(it->second)]) continue;
            const int64_t u = AL.box[size_t(B.k)][size_t(it->second)];
            auto lo = std::lower_bound(lstart.begin(), lstart.end(), L.start[size_t(u)]);
            auto hi = std::lower_bound(lstart.begin(), lstart.end(), L.end[size_t(u)]);
            for (auto q = lo; q != hi; ++q) src.push_back(int32_t(q - lstart.begin()));
          }
      std::sort(src.begin(), src.end());
      for (int32_t a : src) {
        near_src.push_back(a);
        P.near.push_back(i);
        P.near.push_back(a);
        info.near_point_pairs += (B.e - B.s) * (lv[size_t(a)].e - lv[size_t(a)].s);
      }
      near_start.push_back(int32_t(near_src.size()));
    }
    // M2L pairs of the levels below D: the kept children of the boxes adjacent
    // to the parent that are not adjacent themselves (the classical V-list),
    // sorted by (B, A)
    dpairs.assign(size_t(nl), {});
    for (int k = 1; k < nl; ++k) {
      const int l = D + k;
      for (size_t b = 0; b < AL.box[size_t(k)].size(); ++b) {
        const auto cB = coords(l, AL.box[size_t(k)][b]);
        const int64_t p = AL.par[size_t(k)][b];
        const auto cP = coords(l - 1, AL.box[size_t(k - 1)][size_t(p)]);
        std::vector<int64_t> cand;
        for (int dx = -1; dx <= 1; ++dx)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
              auto it = AL.at[size_t(k - 1)].find({cP[0] + dx, cP[1] + dy, cP[2] + dz});
              if (it == AL.at[size_t(k - 1)].end()) continue;
              for (int64_t c = AL.c0[size_t(k - 1)][size_t(it->second)]; c < AL.c1[size_t(k - 1)][size_t(it->second)]; ++c)
                cand.push_back(c);
            }
        std::sort(cand.begin(), cand.end());
        for (int64_t c : cand) {
          const auto cA = coords(l, AL.box[size_t(k)][size_t(c)]);
          const int64_t nx = cA[0] - cB[0], ny = cA[1] - cB[1], nz = cA[2] - cB[2];
          if (std::max({std::abs(nx), std::abs(ny), std::abs(nz)}) > 1)
            dpairs[size_t(k)].push_back(PairRec{int64_t(b), c, nx, ny, nz, -1, -1});
        }
      }
    }
    // exports and counts of the levels below D
    P.boxes.resize(size_t(D + nl));
    P.pairs.resize(size_t(D + nl));
    for (int k = 1; k < nl; ++k) {
      const int l = D + k;
      const auto& L = T.lv[size_t(l)];
      auto& v = P.boxes[size_t(l)];
      for (int64_t u : AL.box[size_t(k)])
        v.insert(v.end(), {L.cx[size_t(u)], L.cy[size_t(u)], L.cz[size_t(u)], L.start[size_t(u)], L.end[size_t(u)]});
      auto& pv = P.pairs[size_t(l)];
      std::set<std::tuple<int64_t, int64_t, int64_t>> offs;
      for (const PairRec& r : dpairs[size_t(k)]) {
        pv.insert(pv.end(), {r.B, r.A, -1, -1, 0});
        offs.insert({r.nx, r.ny, r.nz});
      }
      if (l < 32) {
        info.boxes[l] = int64_t(AL.box[size_t(k)].size());
        info.pairs[l] = int64_t(dpairs[size_t(k)].size());
        info.offsets[l] = int64_t(offs.size());
      }
    }
    info.depth_max = D + nl - 1;
  }
  info.leaves = nleaf;
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
  // One skeleton per LF width: 1/2, and 1/4, 1/8, ... below it in an adaptive
  // tree.  Every LF vector has the row stride of the largest rank.
  const Skel& sl = ops.lf;
  std::vector<const Skel*> lsk{&sl};
  if (nl > 1) {
    const std::vector<Skel>* deep = get_lf_deep(ctx, nl - 1);
    for (int k = 1; k < nl; ++k) lsk.push_back(&(*deep)[size_t(k - 1)]);
  }
  int rmax = 0;
  for (const Skel* q : lsk) rmax = std::max(rmax, q->r);
  int Rlf = pad8(rmax);
  P.lf.R = Rlf;
  P.lf.r = sl.r;
  P.lf.nleaf = nleaf;
  P.lf.nbox = nD;
  for (int k = 0; k < nl && D + k < 32; ++k) info.rank[D + k] = k == 0 ? Rlf : pad8(lsk[size_t(k)]->r);
  {
    const int nsk = int(lsk.size());
    std::vector<float> a4(size_t(4) * Rlf, 0.0f);
    std::vector<double> a64(size_t(4) * Rlf * nsk, 0.0), DT(size_t(2) * Rlf * Rlf * nsk, 0.0);
    std::vector<int32_t> ra(static_cast<size_t>(nsk));
    for (int i = 0; i < sl.r; ++i)
      for (int k = 0; k < 3; ++k) a4[4 * i + k] = float(sl.a[3 * i + k]);
    for (int t = 0; t < nsk; ++t) {  // skeleton t: check points and D^T at offsets t R, t R R
      const Skel& q = *lsk[size_t(t)];
      ra[size_t(t)] = q.r;
      for (int i = 0; i < q.r; ++i)
        for (int k = 0; k < 3; ++k) a64[size_t(4) * (size_t(t) * Rlf + i) + k] = q.a[3 * i + k];
      double* dt = DT.data() + size_t(2) * Rlf * Rlf * t;
      for (int c = 0; c < q.r; ++c)
        for (int p = 0; p < q.r; ++p) {  // DT[p][c] = D[c][p]
          dt[2 * (size_t(p) * Rlf + c)] = q.D[2 * (size_t(c) * q.r + p)];
          dt[2 * (size_t(p) * Rlf + c) + 1] = q.D[2 * (size_t(c) * q.r + p) + 1];
        }
    }
    P.lf.a.upload(a4);
    P.lf.a64.upload(a64);
    std::vector<int32_t> sk_of(static_cast<size_t>(nleaf), 0);
    for (size_t i = 0; i < leaf_lv.size(); ++i) sk_of[i] = int32_t(leaf_lv[i]);
    build_leaf_weights(P, T.pts, DT, ra, sk_of);
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
    build_m2l(pairs[D], 0.5, Rlf, s1, nullptr, nullptr, nD, P.lf.m2l, P.lf.red_start, P.lf.red_idx,
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
        H.nchild_in = nD;
        for (int64_t c = 0; c < nD; ++c) {
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

  // ---- LF levels below D (adaptive trees) ---------------------------------------
  // Per level: the M2L operators of its offsets with its own skeleton, and the
  // 8 octant operators to the level above, in the folded forms of the HF levels
  // (child width w, delta_o = (o - 1/2) w): LF-M2M G(a_P - delta_o, b_C) D_C,
  // LF-L2L G(b_C + delta_o, a_P) D_P^T.
  auto build_lf_transfer = [&](const Skel& sp, const Skel& sc, double wc, GGemm& up, GGemm& dn) {
    const int RK = kpad(Rlf, P.prec);
    const size_t per = size_t(2) * Rlf * RK;  // storage of one operator
    OpStore Au(fp64, per * 8), Ad(fp64, per * 8);
    const int Mp = pad8(sp.r), Mc = pad8(sc.r);
    const int Kpu = kpad(Mc, P.prec), Kpd = kpad(Mp, P.prec);
    parallel_for(8, [&](int64_t o) {
      const double dx = ((o & 1) - 0.5) * wc, dy = (((o >> 1) & 1) - 0.5) * wc, dz = (((o >> 2) & 1) - 0.5) * wc;
      std::vector<double> G(size_t(2) * sp.r * sc.r);  // G[p][j] = G(a_P[p] - delta_o, b_C[j])
      for (int p = 0; p < sp.r; ++p)
        for (int j = 0; j < sc.r; ++j)
          green64(sp.a[3 * p] - dx - sc.b[3 * j], sp.a[3 * p + 1] - dy - sc.b[3 * j + 1],
                  sp.a[3 * p + 2] - dz - sc.b[3 * j + 2], &G[2 * (size_t(p) * sc.r + j)],
                  &G[2 * (size_t(p) * sc.r + j) + 1]);
      std::vector<double> U(size_t(2) * Mp * Kpu, 0.0), Dn(size_t(2) * Mc * Kpd, 0.0);
      for (int p = 0; p < sp.r; ++p)
        for (int k = 0; k < sc.r; ++k) {  // (G D_C)[p][k]
          double re = 0.0, im = 0.0;
          for (int j = 0; j < sc.r; ++j) {
            const double gr = G[2 * (size_t(p) * sc.r + j)], gi = G[2 * (size_t(p) * sc.r + j) + 1];
            const double dr = sc.D[2 * (size_t(j) * sc.r + k)], di = sc.D[2 * (size_t(j) * sc.r + k) + 1];
            re += gr * dr - gi * di;
            im += gr * di + gi * dr;
          }
          U[2 * (size_t(p) * Kpu + k)] = re;
          U[2 * (size_t(p) * Kpu + k) + 1] = im;
        }
      for (int j = 0; j < sc.r; ++j)
        for (int q = 0; q < sp.r; ++q) {  // (G^T D_P^T)[j][q] = sum_p G[p][j] D_P[q][p]
          double re = 0.0, im = 0.0;
          for (int p = 0; p < sp.r; ++p) {
            const double gr = G[2 * (size_t(p) * sc.r + j)], gi = G[2 * (size_t(p) * sc.r + j) + 1];
            const double dr = sp.D[2 * (size_t(q) * sp.r + p)], di = sp.D[2 * (size_t(q) * sp.r + p) + 1];
            re += gr * dr - gi * di;
            im += gr * di + gi * dr;
          }
          Dn[2 * (size_t(j) * Kpd + q)] = re;
          Dn[2 * (size_t(j) * Kpd + q) + 1] = im;
        }
      Au.pack(U.data(), Mp, Kpu, 1, per * size_t(o));
      Ad.pack(Dn.data(), Mc, Kpd, 1, per * size_t(o));
    });
    for (GGemm* g : {&up, &dn}) {
      const bool isup = g == &up;
      g->prec = P.prec;
      g->M = Rlf;
      g->K = Rlf;
      g->T = 1;
      g->split = 1;
      g->nops = 8;
      g->aoff_h.resize(8);
      g->kpk_h.assign(8, isup ? Kpu : Kpd);
      g->opflops.assign(8, 8.0 * sp.r * sc.r);
      for (int o = 0; o < 8; ++o) g->aoff_h[size_t(o)] = int64_t(o) * Rlf * RK / 2;
    }
    Au.upload(up.A);
    Ad.upload(dn.A);
  };
  std::vector<std::vector<SlotTerm>> deep_m2l_terms(static_cast<size_t>(nl));
  P.lfd.clear();
  P.lfd.resize(size_t(nl > 1 ? nl - 1 : 0));
  for (int k = 1; k < nl; ++k) {
    LFDeep& Q = P.lfd[size_t(k - 1)];
    const int l = D + k;
    const double w = K / std::ldexp(1.0, l);
    const Skel& sc = *lsk[size_t(k)];
    Q.l = l;
    Q.r = sc.r;
    Q.nb = int64_t(AL.box[size_t(k)].size());
    Q.base = AL.base[size_t(k)];
    Q.npairs = int64_t(dpairs[size_t(k)].size());
    std::vector<const Skel*> s1{&sc};
    build_m2l(dpairs[size_t(k)], w, Rlf, s1, nullptr, nullptr, Q.nb, Q.m2l, Q.red_start, Q.red_idx, Q.ngroups,
              Q.flops, 1, deep_m2l_terms[size_t(k)]);
    info.flops_m2l_lf += Q.flops;
    if (l < 32) info.flops_m2l_level[l] = Q.flops;
    build_lf_transfer(*lsk[size_t(k - 1)], sc, w, Q.m2m, Q.l2l);
  }

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
    build_slot_gemm(P.lf.down, Rlf, nD, std::vector<int32_t>(size_t(nD), Rlf), lf_terms, dn,
                    std::max(Rlf, e_top >= 0 ? P.hf[0].R : 0));
    // adaptive levels below D.  LF-M2M: a group per split box of level l - 1
    // (written at its LF vector through up_dst), a term per child.  Downward: a
    // group per box of level l: its M2L pairs (kind 0, sources at their LF
    // vectors) and its parent's incoming potentials (kind 1)
    for (int k = 1; k < nl; ++k) {
      LFDeep& Q = P.lfd[size_t(k - 1)];
      const auto& Lc = T.lv[size_t(D + k)];
      std::vector<SlotTerm> up_t;
      std::vector<int32_t> up_dst;
      for (size_t p = 0; p < AL.box[size_t(k - 1)].size(); ++p) {
        if (!AL.split[size_t(k - 1)][p]) continue;
        const int32_t g = int32_t(up_dst.size());
        up_dst.push_back(int32_t(AL.base[size_t(k - 1)] + int64_t(p)));
        for (int64_t c = AL.c0[size_t(k - 1)][p]; c < AL.c1[size_t(k - 1)][p]; ++c)
          up_t.push_back({g, int32_t(Lc.octant[size_t(AL.box[size_t(k)][size_t(c)])]),
                          int32_t(Q.base + c), 0});
      }
      Q.nsplit = int64_t(up_dst.size());
      SlotKind uk[2] = {{&Q.m2m, 1}, {nullptr, 1}};
      build_slot_gemm(Q.up, Rlf, Q.nsplit, std::vector<int32_t>(up_dst.size(), pad8(lsk[size_t(k - 1)]->r)), up_t,
                      uk, Rlf);
      Q.up_dst.upload(up_dst);
      std::vector<SlotTerm> dn_t;
      for (const SlotTerm& t : deep_m2l_terms[size_t(k)])
        dn_t.push_back({t.dst, t.op, int32_t(Q.base + t.src), 0});
      for (int64_t b = 0; b < Q.nb; ++b)
        dn_t.push_back({int32_t(b), int32_t(Lc.octant[size_t(AL.box[size_t(k)][size_t(b)])]),
                        int32_t(AL.base[size_t(k - 1)] + AL.par[size_t(k)][size_t(b)]), 1});
      SlotKind dk[2] = {{&Q.m2l, 1}, {&Q.l2l, 1}};
      build_slot_gemm(Q.down, Rlf, Q.nb, std::vector<int32_t>(size_t(Q.nb), pad8(Q.r)), dn_t, dk, Rlf);
      for (const SlotTerm& t : up_t) info.flops_m2m += Q.m2m.opflops[size_t(t.op)];
      for (int64_t b = 0; b < Q.nb; ++b) info.flops_l2l += Q.l2l.opflops[0];
    }
  }

  info.device_bytes = int64_t(plan_device_bytes(P));
  auto t1 = std::chrono::steady_clock::now();
  P.plan_seconds = std::chrono::duration<double>(t1 - t0).count();
  info.plan_seconds = P.plan_seconds;
}

}  // namespace dfmm
