// Internal declarations shared by the host sources of libdfmm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dfmm.h"
#include "stagebook.hpp"
#include "workspace.hpp"

namespace dfmm {

// ---- errors ----------------------------------------------------------------
void set_error(const std::string& msg);
struct Error {
  int code;
  std::string msg;
};
#define DFMM_HIP(call)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::dfmm::Error{e_ == hipErrorOutOfMemory ? DFMM_ENOMEM : DFMM_EDEVICE,         \
                          std::string(#call) + ": " + hipGetErrorString(e_)};              \
  } while (0)

// ---- skeletons (Eq. 2) -------------------------------------------------------
struct Skel {
  int r = 0;
  std::vector<double> a, b;  // r x 3, box-centred frame
  std::vector<double> D;     // r x r complex, row-major, interleaved
};

}  // namespace dfmm

struct dfmm_opset_s {
  double tau = 0.0;
  int w_hi = 1;
  std::vector<std::vector<dfmm::Skel>> hf;  // [log2 w][dir]
  dfmm::Skel lf;
  std::vector<dfmm::Skel> lf_deep;  // low-frequency widths 1/4, 1/8, ... (adaptive trees)
};

namespace dfmm {
using OpSetImpl = dfmm_opset_s;
void build_opset(OpSetImpl& set);
bool save_opset(const OpSetImpl& set, const std::string& path);
bool load_opset(OpSetImpl& set, const std::string& path);
// Skeletons of the LF widths 1/4, ..., 2^-(1 + n) (Eq. 2, one per width): extends
// set.lf_deep to n entries from set.lf; cached as a file of its own.
void build_lf_deep(OpSetImpl& set, int n);
bool save_lf_deep(const OpSetImpl& set, const std::string& path);
bool load_lf_deep(OpSetImpl& set, const std::string& path, int n);
constexpr int kMaxLfLevels = 6;  // LF levels below width 1/2 an adaptive tree may reach

// ---- device buffers ---------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t n) {
    release();
    if (n == 0) n = 16;
    DFMM_HIP(hipMalloc(&p, n));
    bytes = n;
  }
  template <class T>
  void upload(const std::vector<T>& v) {
    alloc(v.size() * sizeof(T));
    if (!v.empty()) DFMM_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// ---- grouped gather GEMM (the MFMA engine of M2M, M2L and L2L) ---------------
// Vectors are complex64, one per (slot, rhs), stored [slot][rhs][row].  A
// launch computes, for every vector column v of every group g,
//   Y[vdst[v]] = sum_{t < T} A[ops[g T + t]] X[vsrc[v T + t]]
// (a term with source -1 contributes nothing).  Each operator is an M x K
// complex matrix (M, K multiples of 8) stored in MFMA fragment order, see
// pack_operator().
struct GGemm {
  int M = 0, K = 0, T = 1;   // vector strides (rows of Y and of X vectors); per-group sizes <= these
  int split = 1;             // 2: each operator is [T_hi | T_lo] (K doubled) and every source
                             // vector is read twice, so the float32 rounding of T cancels
  bool acc64 = false;        // float64 partial sums every two k-steps (precise plans)
  int prec = 0;              // DFMM_PREC_*: FP16X3 / BF16X3 hold A as 16-bit hi + lo pairs, K padded
                             // to 16 (kpad), one power-of-two scale exponent per operator (aexp)
  DevBuf aexp;               // int32[nops] (FP16X3)
  int64_t ngroups = 0, nvec = 0, nops = 0;
  DevBuf A;                  // operators in fragment order, op i at float4 offset aoff[i]
  DevBuf aoff;               // int64[nops]
  DevBuf gmk;                // int32[ngroups][2]: (M_g, K_g) of the group's operators, multiples of 8
  DevBuf ops;                // int32[ngroups][T]
  DevBuf v0;                 // int32[ngroups + 1]: vector range of each group
  DevBuf vsrc;               // int32[nvec][T]
  DevBuf vdst;               // int32[nvec]
  std::vector<int32_t> v0_h; // host copy of v0 (work chunking)
  std::vector<int64_t> aoff_h;  // host copy of aoff, per operator index
  std::vector<int32_t> kpk_h;   // packed K of each operator index (split doubling included)
  std::vector<double> opflops;  // 8 r_out r_in of each operator index (unpadded ranks)
};

// ---- slot-form GEMM (many right-hand sides) ------------------------------------
// Every output vector (a "group": an out-slot for M2M, an in-slot or a leaf for
// the downward pass) sums its own terms in a fixed order,
//   Y[g] = sum_t A_kind[op_t] X_kind[src_t],
// with float64 sums across terms, so no pair outputs are stored and no
// reduction pass runs.  A term is one pair of the pair form: a child of an M2M
// slot, an M2L pair or a parent wedge of an L2L slot.  Kind 0 / 1 selects one of
// two (operator array, source vectors) pairs, so a level's M2L pairs (kind 0)
// and its L2L terms (kind 1) are summed by one launch into its incoming slots.
struct SlotTerm {
  int32_t dst, op, src, kind;
};
struct SlotGemm {
  int M = 0;                 // row stride of the output vectors (padded rank)
  int Kmax = 8;              // largest packed K of any term (LDS column length)
  int KXmax = 8;             // largest row stride of the source vectors (set by the plan)
  bool split2 = false;       // some term has split operators (not handled by the slot kernel)
  int64_t ngroups = 0, nterms = 0;
  int max_terms = 0;
  double flops[2] = {0, 0};  // 8 r_dst r_src per term and rhs by kind (unpadded ranks)
  DevBuf order;              // int32[ngroups]: launch order, groups with more terms first
  DevBuf t0;                 // int32[ngroups + 1]: term range of each group
  DevBuf gm;                 // int32[ngroups]: padded rows M_g of the group's operators
  DevBuf terms;              // int32[nterms][4]: (operator float4 offset, source vector,
                             //   packed K | split << 12 | kind << 14, 0)
};
// Host view of one kind's operators: float4 offset and packed K (split doubling
// included) of every operator index, and the split factor.
struct SlotKind {
  const GGemm* G = nullptr;  // aoff_h, kpk_h and opflops of the operators (null: no terms of this kind)
  int split = 1;
};
// Term lists -> device tables; terms of a group keep the order given.
void build_slot_gemm(SlotGemm& S, int M, int64_t ngroups, const std::vector<int32_t>& gM,
                     const std::vector<SlotTerm>& terms, const SlotKind kinds[2], int kx_max);

// Pack an M x K complex matrix (row-major, interleaved float64) into the
// fragment order read by the GEMM kernel.
void pack_operator(const double* Tc, int M, int K, float* out);
// pack_operator of T (split = 1) or of [T_hi | T_lo] (split = 2), T_hi the float32
// rounding of T and T_lo that of the remainder; out holds 2 M K split floats
void pack_operator_split(const double* Tc, int M, int K, int split, float* out);
// K of a packed operator: a multiple of 16 for the 16-bit MFMA (two k-steps per instruction)
inline int kpad(int K, int prec) {
  return (prec == DFMM_PREC_FP16X3 || prec == DFMM_PREC_BF16X3) ? (K + 15) / 16 * 16 : K;
}
// pack_operator in float64: the same fragment order, double4 in place of float4
void pack_operator64(const double* Tc, int M, int K, double* out);
// Convert nops packed float32 operators (stride floats apart) in place to the
// hi + lo 16-bit format of prec: each float4 slot (re0, im0, re1, im1) becomes
// four 32-bit words (hi re0 | hi im0), (hi re1 | hi im1), (lo re0 | lo im0),
// (lo re1 | lo im1), low half first.  FP16X3 first scales operator i by
// 2^aexp[i] so that its largest entry is below 2^14.
void to_half_ops(std::vector<float>& A, int64_t nops, int64_t stride, int prec, std::vector<int32_t>& aexp);

// ---- one HF level of the plan -------------------------------------------------
struct HFLevel {
  int l = 0;      // tree level
  int e = 0;      // log2 of the width
  int R = 0;      // padded skeleton size (multiple of 8)
  int Rc = 0;     // padded skeleton size of the child level (LF at e = 0)
  int64_t nout = 0, nin = 0, npairs = 0, ngroups = 0, nchild_in = 0;
  double flops = 0.0;  // 8 r_in r_out over pairs (unpadded ranks)
  GGemm m2m;           // (parent out-slot, child) pair outputs, grouped by (wedge, octant)
  DevBuf m2m_rs, m2m_ri;  // CSR of pair outputs per out-slot
  int64_t m2m_npairs = 0;
  GGemm l2l;           // (child in-slot, parent in-slot) pair outputs, grouped by (wedge, octant)
  DevBuf l2l_rs, l2l_ri;  // CSR of pair outputs per child in-slot (or leaf at e = 0)
  int64_t l2l_npairs = 0;
  GGemm m2l;           // pair outputs <- source out-slots, grouped by offset
  DevBuf red_start;    // int32[nin + 1]: CSR of pair outputs per in-slot
  DevBuf red_idx;      // int32[npairs]
  SlotGemm up;         // slot form of M2M: out-slots <- children
  SlotGemm down;       // slot form of M2L + L2L: in-slots <- M2L pairs, parent wedges
};

struct LFLevel {
  int R = 0;           // padded rank (multiple of 8): the row stride of every LF vector
  int r = 0;           // rank of the width-1/2 LF skeleton
  int64_t nleaf = 0;   // leaves (S2M, L2T and the near field run over them)
  int64_t nbox = 0;    // boxes of width 1/2 (LF-M2L of that level; = nleaf in a uniform tree)
  int64_t npairs = 0, ngroups = 0;
  double flops = 0.0;
  DevBuf a;            // float4[R]  check points a_LF (box frame)
  DevBuf a64;          // double4[R] the same in float64
  DevBuf V;            // float2[N][R]: S2M weights G(c + a_p, x_j) per sorted point
  DevBuf W;            // float2[N][R]: L2T weights sum_p G(x_j, c + a_p) D_LF[q][p]
  GGemm m2l;
  DevBuf red_start, red_idx;
  SlotGemm down;       // slot form of LF-M2L + L2L into the leaves
};

// One low-frequency level below width 1/2 of an adaptive tree (Section 2.2):
// its boxes are the children of the split boxes of the level above; it has its
// own skeleton (LF-M2L operators per offset) and the octant operators that
// connect it to the level above (LF-M2M up, LF-L2L down).
struct LFDeep {
  int l = 0;                 // tree level
  int r = 0;                 // rank of this width's skeleton
  int64_t nb = 0;            // boxes of this level
  int64_t base = 0;          // LF vector index of the first of them
  int64_t npairs = 0, ngroups = 0, nsplit = 0;  // M2L pairs and offsets; split boxes of level l - 1
  double flops = 0.0;        // M2L flops (8 r r per pair)
  GGemm m2l;                 // LF-M2L operators, one per offset
  GGemm m2m;                 // 8 octant operators G(a_P - delta_o, b_C) D_C: parent <- child
  GGemm l2l;                 // 8 octant operators G(b_C + delta_o, a_P) D_P^T: child <- parent
  DevBuf red_start, red_idx; // pair-form CSR of the M2L (built with the operators, unused)
  SlotGemm up;               // LF-M2M: the split boxes of level l - 1 <- their children
  DevBuf up_dst;             // int32[nsplit]: LF vector index of each of those parents
  SlotGemm down;             // LF-M2L pairs + LF-L2L term of every box of this level
};

// Octree with one table per level, boxes in Morton order (host copy).
struct Tree {
  int D = 0;                                 // leaf level (leaf width 1/2)
  std::vector<int64_t> perm;                 // sorted position -> original index
  std::vector<double> pts;                   // sorted points, N x 3
  struct Lv {
    std::vector<int64_t> key;                // Morton key at this level, ascending
    std::vector<int64_t> cx, cy, cz;         // integer box coordinates
    std::vector<int64_t> start, end;         // sorted point range
    std::vector<int64_t> parent, octant;     // parent index at level l-1, octant in it
    std::vector<int64_t> cbeg, cend;         // children range at level l+1
  };
  std::vector<Lv> lv;
};

// One interaction pair B <- A at a level: offset n = i_A - i_B and the wedges
// l_in = dir(n), l_out = dir(-n) (-1 at the leaf level).
struct PairRec {
  int64_t B, A, nx, ny, nz;
  int din, dout;
};

// Needed (box, wedge) slots of one level: dense index box * ndir + wedge -> slot
// (or -1), and the slots in (box, wedge) order.
struct SlotIndex {
  int ndir = 0;
  std::vector<int64_t> dense;
  std::vector<std::pair<int64_t, int>> list;
  int64_t at(int64_t b, int d) const { return dense[size_t(b * ndir + d)]; }
};

// Device box tables (int32 except the keys), built from the sorted point keys.
struct DevLevel {
  int64_t nb = 0;
  DevBuf key, start, end, cx, cy, cz, parent, cbeg, cend;
};
struct DevTree {
  std::vector<DevLevel> lv;
  std::vector<DevBuf> incl;  // per level: inclusive box count at each sorted point
};
void build_levels_device(const unsigned long long* sorted_key, int64_t N, int D, Tree& T, DevTree& DT);
// radix.hip: stable LSD radix sort of 64-bit keys (and int values) over the key
// bits [0, end_bit) into separate outputs, and int32 prefix sums (null stream)
void sort_pairs_u64(const unsigned long long* kin, unsigned long long* kout, const int* vin, int* vout, int64_t n,
                    int end_bit);
void sort_keys_u64(const unsigned long long* kin, unsigned long long* kout, int64_t n, int end_bit);
void scan_incl(const int* in, int* out, int64_t n);
void scan_excl(const int* in, int* out, int64_t n);
// I^B of every box of level l, sorted by (B, A); `fields` keeps the device copy
// ([np][7] int32: B, A, nx, ny, nz, l_in, l_out).
std::vector<PairRec> level_pairs_device(const DevTree& DT, int D, int l, DevBuf& fields);
void near_lists_device(const DevTree& DT, int D, std::vector<int32_t>& start, std::vector<int32_t>& src);
void slot_closure_device(const DevTree& DT, int D, int l_top, const std::vector<DevBuf>& fields,
                         const std::vector<int64_t>& npairs, std::vector<SlotIndex>& OS, std::vector<SlotIndex>& IS);

struct ApplyState;
void destroy_apply_state(ApplyState* s);

// Stages reported by dfmm_stage_times (same order as in include/dfmm.h).
enum { ST_PERMUTE = 0, ST_S2M, ST_M2M, ST_M2L, ST_REDUCE, ST_L2L, ST_LF_M2L, ST_LF_REDUCE, ST_LEAF,
       ST_ZERO, ST_NEAR, ST_COUNT };

// HIP events recorded on the apply stream after every launch, for a bounded
// number of applies; no host synchronisation until collect().
struct StageTimer {
  static constexpr size_t kPerApply = 64;
  std::vector<hipEvent_t> pool;
  StageBook book;                   // which event closes which stage interval
  explicit StageTimer(int applies);
  ~StageTimer();
  bool begin_apply(hipStream_t st);
  void mark(int stage, hipStream_t st);            // interval since the previous apply-stream event
  void side_begin(hipStream_t side);               // opens an interval on the side stream
  void side_mark(int stage, hipStream_t side);     // closes it
  void collect(double* ms, int64_t* launches);  // sums per stage (ST_COUNT entries), then resets
};
// The requests of one apply: batch columns k0[r] .. k0[r + 1] - 1 (the last
// request up to nrhs) are request r's right-hand sides, read from f[r] and
// written to u[r] (each [nrhs_r][N], caller's point order).  Passed by value
// as a kernel argument.
constexpr int kMaxBatch = DFMM_MAX_BATCH;
struct ReqTable {
  const float2* f[kMaxBatch];
  float2* u[kMaxBatch];
  int k0[kMaxBatch];
  int n;
};
// ws: the caller's workspace of ws_bytes (>= workspace_bytes(P, nrhs); everything
// then runs on st, and calls may overlap) or null (the plan-owned workspace, the
// near field on the plan's second stream).  existing_only: use only what an
// earlier apply with this nrhs prepared (no allocation, no tuning).
void run_apply(dfmm_plan_s& P, const ReqTable& R, int nrhs, hipStream_t st, void* ws, size_t ws_bytes,
               bool existing_only);
size_t workspace_bytes(const dfmm_plan_s& P, int nrhs);
// dfmm_apply_noalloc: run_apply on the static device workspace (kNoAllocBytes),
// with the launch shapes an earlier apply of this nrhs prepared.
constexpr size_t kNoAllocBytes = size_t(DFMM_NOALLOC_MAX_BYTES);
void run_apply_noalloc(dfmm_plan_s& P, const ReqTable& R, int nrhs, hipStream_t st);
size_t plan_device_bytes(const dfmm_plan_s& P);
// float64 plans: the whole pass in complex128 on a caller-sized workspace
// (ws_layout(ws_shape64(P), nrhs, false, 16))
WsShape ws_shape64(const dfmm_plan_s& P);
void run_apply64(dfmm_plan_s& P, const double2* f, double2* u, int nrhs, hipStream_t st, void* ws);
// S2M and L2T weights of every sorted point (float64, then stored in the plan's
// precision).  DT holds D^T of each LF skeleton at R x R offsets, P.lf.a64 its
// check points at R offsets; ra the skeletons' ranks, sk_of the skeleton of each leaf.
void build_leaf_weights(dfmm_plan_s& P, const std::vector<double>& sorted_pts, const std::vector<double>& DT,
                        const std::vector<int32_t>& ra, const std::vector<int32_t>& sk_of);
void build_plan(dfmm_plan_s& P, const double* points, int64_t N, double K,
                const OpSetImpl* (*get_ops)(void* ctx, int w_needed),
                const std::vector<Skel>* (*get_lf_deep)(void* ctx, int n), void* ctx);

}  // namespace dfmm

struct dfmm_plan_s {
  int device = 0;
  int64_t N = 0;
  double K = 0.0;
  int D = 0;       // leaf level
  int w_top = 0;
  bool precise = false;  // eps < 1e-5: float64 near-field distances, split HF operators
  int prec = 0;          // DFMM_PREC_*: arithmetic of the translation GEMMs
  double plan_seconds = 0.0;
  std::string tune_dir;  // where GEMM launch choices are kept (empty: not kept)
  dfmm_info info{};
  // host copies of structures for export
  std::vector<int64_t> perm;
  std::vector<std::vector<int64_t>> boxes;   // per level: nb x 5
  std::vector<std::vector<int64_t>> pairs;   // per level: np x 5 sorted (B, A)
  std::vector<int64_t> near;                 // np x 2
  std::vector<std::vector<int64_t>> out_slots, in_slots;  // per level: ns x 2
  // device
  dfmm::DevBuf pthi, ptlo;       // float4[N] sorted points (hi, lo split)
  dfmm::DevBuf perm_d;           // int32[N]: tree position -> caller's index
  dfmm::DevBuf iperm_d;          // int32[N]: caller's index -> tree position
  dfmm::DevBuf leaf_start;       // int32[nleaf + 1]
  dfmm::DevBuf leaf_of;          // int32[N]: leaf of each sorted point
  dfmm::DevBuf leaf_center;      // float4[nleaf]
  dfmm::DevBuf near_start, near_src;  // CSR over leaves
  int max_leaf_pts = 0;
  // adaptive low-frequency tree (leaf_max > 0): boxes of width <= 1/2 split while
  // they hold more than leaf_max points, down to lf_levels levels below 1/2
  int leaf_max = 0, lf_levels = 0;
  int64_t nlfbox = 0;            // LF vectors (flf / ulf): every box of width <= 1/2
  dfmm::DevBuf leaf_gid;         // int32[nleaf]: LF vector of each leaf (adaptive; empty = identity)
  std::vector<dfmm::LFDeep> lfd; // levels D + 1 .. of an adaptive tree
  std::vector<int64_t> leaves;   // export: nleaf x 4 (level, box, first point, end point)
  dfmm::LFLevel lf;
  std::vector<dfmm::HFLevel> hf;  // index e (log2 w), 0 .. e_top
  // apply workspace (owned; see apply.hip)
  struct dfmm::ApplyState* ws = nullptr;
  // stage timing (null when disabled)
  dfmm::StageTimer* timer = nullptr;
};
