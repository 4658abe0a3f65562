// C ABI of libdfmm (declarations and contracts in include/dfmm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <sys/stat.h>

#include "internal.hpp"

namespace dfmm {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

template <class F>
int guarded(F&& fn) {
  try {
    set_error("");
    return fn();
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(DFMM_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(DFMM_EINVAL, e.what());
  } catch (...) {
    return fail(DFMM_EINVAL, "unknown error");
  }
}

// Makes `dev` current for its lifetime and restores the caller's device after,
// also when the call fails with an exception.
class DeviceScope {
 public:
  explicit DeviceScope(int dev) {
    DFMM_HIP(hipGetDevice(&prev_));
    if (prev_ != dev) DFMM_HIP(hipSetDevice(dev));
    switched_ = prev_ != dev;
  }
  ~DeviceScope() {
    if (switched_) (void)hipSetDevice(prev_);
  }
  DeviceScope(const DeviceScope&) = delete;
  DeviceScope& operator=(const DeviceScope&) = delete;

 private:
  int prev_ = 0;
  bool switched_ = false;
};

bool is_pow2(double K) {
  if (!(K >= 1.0) || !(K <= 1048576.0)) return false;
  double r = std::round(K);
  if (r != K) return false;
  int64_t k = int64_t(r);
  return (k & (k - 1)) == 0;
}

// Per-skeleton truncation tau for an end-to-end relative L2 target eps,
// calibrated against the direct sum.  The end-to-end error is a multiple of
// tau that grows with the far field's share of the potential: at tau = 1.5e-5
// it was 5.5-6.5 tau on spheres (81-163 points per square wavelength) and the
// K = 32 4:2:1 ellipsoid with 262,144 points, but 8.9 tau on the same
// ellipsoid with 131,072 points, so tau = 0.1 eps.  Below 1e-5 the float32
// translations (~4e-7 with split operators and float64 partial sums) also take
// a share of the budget: at tau = 5e-8 the K = 16 sphere gave 7.6e-7 and the
// 131,072-point ellipsoid 1.07e-6, so tau = 0.03 eps there.
double tau_for_eps(double eps) { return eps >= 1e-5 ? 0.1 * eps : 0.03 * eps; }
// Float64 plans: the same rule, but not below 1e-9.  The skeletons' middle
// factors D = G(X, b)^+ G(X, Y) G(a, Y)^+ are formed in float64 from matrices of
// condition ~1/tau; on fresh samples Eq. 2 then holds to about 7 tau at
// tau = 1e-6, 20 tau at 1e-8, 6e-8 at 1e-9, and worse again below (3e-7 at
// 1e-10, 4e-6 at 1e-11), so tighter tau buys nothing.
double tau_for_eps64(double eps) { return std::max(tau_for_eps(eps), 1e-9); }

// Directions of width w: w = 1, 2, 4, ... -> 6 w^2 (*e = log2 w); the LF
// widths w = 1/2, 1/4, ..., 2^-(1 + kMaxLfLevels) -> 1 (*e = -1 - log2(1/(2w))).
int dir_count(double w, int* e) {
  for (int k = 0; k <= kMaxLfLevels; ++k)
    if (w == std::ldexp(0.5, -k)) {
      *e = -1 - k;
      return 1;
    }
  if (!(w >= 1.0)) return -1;
  int ee = 0;
  while (std::ldexp(1.0, ee) < w) ++ee;
  if (std::ldexp(1.0, ee) != w) return -1;
  *e = ee;
  return 6 << (2 * ee);
}

std::string cache_path(const char* dir, double tau, int w_hi) {
  char buf[128];
  std::snprintf(buf, sizeof(buf), "/dfmm_opset_tau%.3e_w%d_v2.bin", tau, w_hi);
  return std::string(dir) + buf;
}

std::string lf_deep_path(const char* dir, double tau) {
  char buf[128];
  std::snprintf(buf, sizeof(buf), "/dfmm_lfdeep_tau%.3e_v1.bin", tau);
  return std::string(dir) + buf;
}

struct PlanCtx {
  const dfmm_options* opt;
  std::unique_ptr<OpSetImpl> owned;
  const OpSetImpl* used = nullptr;
};

// The skeletons of the LF widths 1/4 .. 2^-(1 + n) for an adaptive plan: from
// the caller's set (which must hold them), else built once and cached.
const std::vector<Skel>* plan_lf_deep(void* vctx, int n) {
  PlanCtx& c = *static_cast<PlanCtx*>(vctx);
  if (c.opt->opset) {
    const auto& v = c.opt->opset->lf_deep;
    if (int(v.size()) < n) throw Error{DFMM_EINVAL, "operator set lacks the deeper LF skeletons"};
    for (int i = 0; i < n; ++i)
      if (v[size_t(i)].r < 1) throw Error{DFMM_EINVAL, "operator set has unset deeper LF skeletons"};
    return &v;
  }
  OpSetImpl& s = *c.owned;
  if (int(s.lf_deep.size()) >= n) return &s.lf_deep;
  const char* dir = c.opt->cache_dir ? c.opt->cache_dir : std::getenv("DFMM_CACHE_DIR");
  if (dir && load_lf_deep(s, lf_deep_path(dir, s.tau), n)) return &s.lf_deep;
  build_lf_deep(s, kMaxLfLevels);
  if (dir) {
    ::mkdir(dir, 0755);
    (void)save_lf_deep(s, lf_deep_path(dir, s.tau));
  }
  return &s.lf_deep;
}

const OpSetImpl* plan_ops(void* vctx, int w_needed) {
  PlanCtx& c = *static_cast<PlanCtx*>(vctx);
  if (c.opt->opset) {
    c.used = c.opt->opset;
    return c.used;
  }
  const bool fp64 = c.opt->precision == DFMM_PREC_FP64;
  double tau = c.opt->tol_factor > 0.0 ? c.opt->tol_factor * c.opt->eps
                                       : (fp64 ? tau_for_eps64(c.opt->eps) : tau_for_eps(c.opt->eps));
  int w_hi = 1;
  while (w_hi < w_needed) w_hi *= 2;
  const char* dir = c.opt->cache_dir ? c.opt->cache_dir : std::getenv("DFMM_CACHE_DIR");
  c.owned.reset(new OpSetImpl());
  if (dir) {
    for (int w = w_hi; w <= 64; w *= 2)
      if (load_opset(*c.owned, cache_path(dir, tau, w)) && c.owned->tau == tau) {
        c.used = c.owned.get();
        return c.used;
      }
  }
  c.owned.reset(new OpSetImpl());
  c.owned->tau = tau;
  c.owned->w_hi = w_hi;
  build_opset(*c.owned);
  if (dir) {
    ::mkdir(dir, 0755);
    (void)save_opset(*c.owned, cache_path(dir, tau, w_hi));
  }
  c.used = c.owned.get();
  return c.used;
}

}  // namespace
}  // namespace dfmm

using namespace dfmm;

extern "C" {

const char* dfmm_status_string(int s) {
  switch (s) {
    case DFMM_OK: return "DFMM_OK";
    case DFMM_EINVAL: return "DFMM_EINVAL";
    case DFMM_EDOMAIN: return "DFMM_EDOMAIN";
    case DFMM_EUNSUPPORTED: return "DFMM_EUNSUPPORTED";
    case DFMM_ENOMEM: return "DFMM_ENOMEM";
    case DFMM_EDEVICE: return "DFMM_EDEVICE";
    case DFMM_EIO: return "DFMM_EIO";
    default: return "DFMM_UNKNOWN";
  }
}

const char* dfmm_last_error(void) { return g_last_error.c_str(); }

int dfmm_opset_build(double tau, int w_hi, const char* cache_dir, dfmm_opset_t* out) {
  return guarded([&]() {
    if (!out) return fail(DFMM_EINVAL, "null output pointer");
    *out = nullptr;
    if (!(tau > 0.0 && tau < 1.0)) return fail(DFMM_EINVAL, "tau must be in (0, 1)");
    if (w_hi < 1 || w_hi > 64 || (w_hi & (w_hi - 1))) return fail(DFMM_EINVAL, "w_hi must be a power of two in [1, 64]");
    std::unique_ptr<OpSetImpl> s(new OpSetImpl());
    if (cache_dir && load_opset(*s, cache_path(cache_dir, tau, w_hi)) && s->tau == tau && s->w_hi == w_hi) {
      *out = s.release();
      return int(DFMM_OK);
    }
    s.reset(new OpSetImpl());
    s->tau = tau;
    s->w_hi = w_hi;
    build_opset(*s);
    if (cache_dir) {
      ::mkdir(cache_dir, 0755);
      (void)save_opset(*s, cache_path(cache_dir, tau, w_hi));
    }
    *out = s.release();
    return int(DFMM_OK);
  });
}

int dfmm_opset_create(double tau, int w_hi, dfmm_opset_t* out) {
  return guarded([&]() {
    if (!out) return fail(DFMM_EINVAL, "null output pointer");
    if (w_hi < 1 || w_hi > 64 || (w_hi & (w_hi - 1))) return fail(DFMM_EINVAL, "w_hi must be a power of two in [1, 64]");
    std::unique_ptr<OpSetImpl> s(new OpSetImpl());
    s->tau = tau;
    s->w_hi = w_hi;
    int emax = 0;
    while ((1 << emax) < w_hi) ++emax;
    s->hf.assign(emax + 1, {});
    for (int e = 0; e <= emax; ++e) s->hf[e].assign(size_t(6) << (2 * e), Skel());
    *out = s.release();
    return int(DFMM_OK);
  });
}

static Skel* find_skel(dfmm_opset_t set, double w, int dir) {
  int e = 0;
  int n = dir_count(w, &e);
  if (n < 0 || dir < 0 || dir >= n) return nullptr;
  if (e == -1) return &set->lf;
  if (e < -1) {  // a deeper LF width: the set grows to hold it
    const size_t k = size_t(-1 - e);
    if (set->lf_deep.size() < k) set->lf_deep.resize(k);
    return &set->lf_deep[k - 1];
  }
  if (e >= int(set->hf.size())) return nullptr;
  return &set->hf[e][dir];
}

int dfmm_opset_set(dfmm_opset_t set, double w, int dir, int r, const double* a, const double* b,
                   const double* D) {
  return guarded([&]() {
    if (!set || !a || !b || !D || r < 1 || r > 4096) return fail(DFMM_EINVAL, "bad argument");
    Skel* s = find_skel(set, w, dir);
    if (!s) return fail(DFMM_EINVAL, "no such width / direction in this set");
    s->r = r;
    s->a.assign(a, a + 3 * size_t(r));
    s->b.assign(b, b + 3 * size_t(r));
    s->D.assign(D, D + 2 * size_t(r) * r);
    return int(DFMM_OK);
  });
}

int dfmm_opset_get(dfmm_opset_t set, double w, int dir, int* r, double* a, double* b, double* D) {
  return guarded([&]() {
    if (!set || !r) return fail(DFMM_EINVAL, "bad argument");
    int e = 0;
    if (dir_count(w, &e) == 1 && e < -1 && size_t(-1 - e) > set->lf_deep.size())
      return fail(DFMM_EINVAL, "no such width / direction in this set");
    Skel* s = find_skel(set, w, dir);
    if (!s) return fail(DFMM_EINVAL, "no such width / direction in this set");
    *r = s->r;
    if (a) std::memcpy(a, s->a.data(), sizeof(double) * s->a.size());
    if (b) std::memcpy(b, s->b.data(), sizeof(double) * s->b.size());
    if (D) std::memcpy(D, s->D.data(), sizeof(double) * s->D.size());
    return int(DFMM_OK);
  });
}

int dfmm_opset_info(dfmm_opset_t set, double* tau, int* w_hi) {
  if (!set) return fail(DFMM_EINVAL, "null set");
  if (tau) *tau = set->tau;
  if (w_hi) *w_hi = set->w_hi;
  return DFMM_OK;
}

int dfmm_opset_save(dfmm_opset_t set, const char* path) {
  return guarded([&]() {
    if (!set || !path) return fail(DFMM_EINVAL, "bad argument");
    if (!save_opset(*set, path)) return fail(DFMM_EIO, std::string("cannot write ") + path);
    return int(DFMM_OK);
  });
}

int dfmm_opset_load(const char* path, dfmm_opset_t* out) {
  return guarded([&]() {
    if (!path || !out) return fail(DFMM_EINVAL, "bad argument");
    std::unique_ptr<OpSetImpl> s(new OpSetImpl());
    if (!load_opset(*s, path)) return fail(DFMM_EIO, std::string("cannot read ") + path);
    *out = s.release();
    return int(DFMM_OK);
  });
}

void dfmm_opset_destroy(dfmm_opset_t set) { delete set; }

void dfmm_options_default(dfmm_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->eps = 1e-4;
  opt->device = -1;
}

int dfmm_plan(const double* points, int64_t N, double K, double eps, dfmm_plan_t* out) {
  dfmm_options o;
  dfmm_options_default(&o);
  o.eps = eps;
  return dfmm_plan_ex(points, N, K, &o, out);
}

int dfmm_plan_ex(const double* points, int64_t N, double K, const dfmm_options* opt, dfmm_plan_t* out) {
  return guarded([&]() {
    if (!out) return fail(DFMM_EINVAL, "null output pointer");
    *out = nullptr;
    if (!points || !opt) return fail(DFMM_EINVAL, "null points or options");
    if (N < 1 || N > (int64_t(1) << 31) - 1) return fail(DFMM_EINVAL, "N must be in [1, 2^31 - 1]");
    if (!is_pow2(K)) return fail(DFMM_EUNSUPPORTED, "K must be a power of two in [1, 2^20]");
    const bool fp64 = opt->precision == DFMM_PREC_FP64;
    if (!opt->opset && !(opt->eps >= (fp64 ? 1e-8 : 1e-6) && opt->eps <= 1e-2))
      return fail(DFMM_EUNSUPPORTED, fp64 ? "eps must be in [1e-8, 1e-2] for float64 plans"
                                          : "eps must be in [1e-6, 1e-2] (float64 plans: from 1e-8)");
    if (opt->opset) {
      for (auto& v : opt->opset->hf)
        for (auto& s : v)
          if (s.r < 1) return fail(DFMM_EINVAL, "operator set has unset skeletons");
      if (opt->opset->lf.r < 1) return fail(DFMM_EINVAL, "operator set has no LF skeleton");
    }
    const double lim = K / 2.0 * (1.0 + 1e-12);
    for (int64_t i = 0; i < N; ++i) {
      double x = points[3 * i], y = points[3 * i + 1], z = points[3 * i + 2];
      if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z))
        return fail(DFMM_EDOMAIN, "point " + std::to_string(i) + " is not finite");
      if (std::sqrt(x * x + y * y + z * z) > lim)
        return fail(DFMM_EDOMAIN, "point " + std::to_string(i) + " lies outside |p| <= K/2");
    }
    if (!(opt->leaf_width == 0.0 || opt->leaf_width == 0.5))
      return fail(DFMM_EUNSUPPORTED, "leaf_width must be 1/2 (0 = default): the first low-frequency level "
                                     "has width 1/2 (finer leaves come from leaf_max)");
    if (opt->leaf_max < 0 || opt->lf_levels < 0 || opt->lf_levels > kMaxLfLevels)
      return fail(DFMM_EINVAL, "leaf_max must be >= 0 and lf_levels in [0, " + std::to_string(kMaxLfLevels) + "]");
    if (!opt->opset && !(opt->tol_factor == 0.0 || (opt->tol_factor > 0.0 && opt->tol_factor <= 1.0)))
      return fail(DFMM_EINVAL, "tol_factor must be in (0, 1] (0 = default)");
    // HBM budget, checked before any device call: sorted points (hi + lo float4
    // pairs), the float64 copy of the input, permutation and leaf index per point
    if (opt->hbm_budget_bytes > 0 && uint64_t(N) * 64u > opt->hbm_budget_bytes)
      return fail(DFMM_ENOMEM, "the plan needs at least " + std::to_string(uint64_t(N) * 64u) +
                                   " device bytes; hbm_budget_bytes is " + std::to_string(opt->hbm_budget_bytes));
    const double tau_plan = opt->opset ? opt->opset->tau
                            : (opt->tol_factor > 0.0 ? opt->tol_factor * opt->eps
                                                     : (fp64 ? tau_for_eps64(opt->eps) : tau_for_eps(opt->eps)));
    // float32 plans below tau 3e-6 are "precise" (split operators, float64 partial
    // sums); float64 plans need neither
    const bool precise = !fp64 && tau_plan < 3e-6;
    if (opt->precision < DFMM_PREC_FP32 || opt->precision > DFMM_PREC_FP64)
      return fail(DFMM_EINVAL, "unknown precision");
    if ((opt->precision == DFMM_PREC_FP16X3 || opt->precision == DFMM_PREC_BF16X3) && precise)
      return fail(DFMM_EINVAL, "split precision is for eps >= 1e-5 plans");
    if (opt->leaf_max > 0 && (opt->precision != DFMM_PREC_FP32 || precise))
      return fail(DFMM_EUNSUPPORTED, "adaptive trees (leaf_max > 0) are for float32 plans with eps >= 1e-5");
    int dev = opt->device;
    if (dev < 0) DFMM_HIP(hipGetDevice(&dev));
    DeviceScope on(dev);
    std::unique_ptr<dfmm_plan_s> P(new dfmm_plan_s());
    P->device = dev;
    P->precise = precise;
    P->prec = opt->precision;
    if (const char* dir = opt->cache_dir ? opt->cache_dir : std::getenv("DFMM_CACHE_DIR")) P->tune_dir = dir;
    PlanCtx ctx{opt, nullptr, nullptr};
    P->leaf_max = opt->leaf_max;
    P->lf_levels = opt->leaf_max > 0 ? (opt->lf_levels > 0 ? opt->lf_levels : 3) : 0;
    build_plan(*P, points, N, K, &plan_ops, &plan_lf_deep, &ctx);
    if (opt->hbm_budget_bytes > 0 && uint64_t(P->info.device_bytes) > opt->hbm_budget_bytes)
      return fail(DFMM_ENOMEM, "the plan holds " + std::to_string(P->info.device_bytes) +
                                   " device bytes; hbm_budget_bytes is " + std::to_string(opt->hbm_budget_bytes));
    *out = P.release();
    return int(DFMM_OK);
  });
}

int dfmm_apply(dfmm_plan_t plan, const void* f, void* u, int nrhs, void* stream) {
  return guarded([&]() {
    if (!plan || !f || !u) return fail(DFMM_EINVAL, "null plan or vector");
    if (nrhs < 1 || nrhs > 4096) return fail(DFMM_EINVAL, "nrhs must be in [1, 4096]");
    const char* fb = static_cast<const char*>(f);
    const char* ub = static_cast<const char*>(u);
    size_t bytes = size_t(plan->prec == DFMM_PREC_FP64 ? 16 : 8) * size_t(plan->N) * size_t(nrhs);
    if (fb < ub + bytes && ub < fb + bytes) return fail(DFMM_EINVAL, "f and u overlap");
    ReqTable R{};
    R.f[0] = static_cast<const float2*>(f);
    R.u[0] = static_cast<float2*>(u);
    R.k0[0] = 0;
    R.n = 1;
    DeviceScope on(plan->device);
    run_apply(*plan, R, nrhs, static_cast<hipStream_t>(stream), nullptr, 0, false);
    return int(DFMM_OK);
  });
}

int dfmm_apply_batch(dfmm_plan_t plan, int nreq, const void* const* f, void* const* u, const int* nrhs,
                     void* stream) {
  return guarded([&]() {
    if (!plan || !f || !u || !nrhs) return fail(DFMM_EINVAL, "null plan or array");
    if (nreq < 1 || nreq > DFMM_MAX_BATCH) return fail(DFMM_EINVAL, "nreq must be in [1, DFMM_MAX_BATCH]");
    if (plan->prec == DFMM_PREC_FP64) return fail(DFMM_EUNSUPPORTED, "float64 plans take dfmm_apply or dfmm_apply_ws");
    ReqTable R{};
    int total = 0;
    const size_t col = size_t(8) * size_t(plan->N);
    for (int r = 0; r < nreq; ++r) {
      if (!f[r] || !u[r]) return fail(DFMM_EINVAL, "null request vector");
      if (nrhs[r] < 1) return fail(DFMM_EINVAL, "request nrhs must be >= 1");
      R.f[r] = static_cast<const float2*>(f[r]);
      R.u[r] = static_cast<float2*>(u[r]);
      R.k0[r] = total;
      total += nrhs[r];
      if (total > 4096) return fail(DFMM_EINVAL, "total nrhs must be <= 4096");
    }
    // no output may overlap an input or another output
    for (int r = 0; r < nreq; ++r) {
      const char* ur = static_cast<const char*>(u[r]);
      const size_t ub = col * size_t(nrhs[r]);
      for (int q = 0; q < nreq; ++q) {
        const char* fq = static_cast<const char*>(f[q]);
        const char* uq = static_cast<const char*>(u[q]);
        const size_t qb = col * size_t(nrhs[q]);
        if (fq < ur + ub && ur < fq + qb) return fail(DFMM_EINVAL, "an output overlaps an input");
        if (q != r && uq < ur + ub && ur < uq + qb) return fail(DFMM_EINVAL, "two outputs overlap");
      }
    }
    R.n = nreq;
    DeviceScope on(plan->device);
    run_apply(*plan, R, total, static_cast<hipStream_t>(stream), nullptr, 0, false);
    return int(DFMM_OK);
  });
}

int dfmm_apply_ws(dfmm_plan_t plan, const void* f, void* u, int nrhs, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&]() {
    if (!plan || !f || !u || !ws) return fail(DFMM_EINVAL, "null plan, vector or workspace");
    if (nrhs < 1 || nrhs > 4096) return fail(DFMM_EINVAL, "nrhs must be in [1, 4096]");
    if (reinterpret_cast<uintptr_t>(ws) % kWsAlign != 0) return fail(DFMM_EINVAL, "workspace not 256-byte aligned");
    const char* fb = static_cast<const char*>(f);
    const char* ub = static_cast<const char*>(u);
    const char* wb = static_cast<const char*>(ws);
    size_t bytes = size_t(plan->prec == DFMM_PREC_FP64 ? 16 : 8) * size_t(plan->N) * size_t(nrhs);
    if (fb < ub + bytes && ub < fb + bytes) return fail(DFMM_EINVAL, "f and u overlap");
    if ((wb < ub + bytes && ub < wb + ws_bytes) || (wb < fb + bytes && fb < wb + ws_bytes))
      return fail(DFMM_EINVAL, "the workspace overlaps f or u");
    ReqTable R{};
    R.f[0] = static_cast<const float2*>(f);
    R.u[0] = static_cast<float2*>(u);
    R.k0[0] = 0;
    R.n = 1;
    DeviceScope on(plan->device);
    run_apply(*plan, R, nrhs, static_cast<hipStream_t>(stream), ws, ws_bytes, false);
    return int(DFMM_OK);
  });
}

int dfmm_apply_noalloc(dfmm_plan_t plan, const void* f, void* u, int nrhs, void* stream) {
  return guarded([&]() {
    if (!plan || !f || !u) return fail(DFMM_EINVAL, "null plan or vector");
    if (plan->prec == DFMM_PREC_FP64) return fail(DFMM_EUNSUPPORTED, "float64 plans take dfmm_apply or dfmm_apply_ws");
    if (nrhs < 1 || nrhs > 4096) return fail(DFMM_EINVAL, "nrhs must be in [1, 4096]");
    const char* fb = static_cast<const char*>(f);
    const char* ub = static_cast<const char*>(u);
    size_t bytes = size_t(8) * size_t(plan->N) * size_t(nrhs);
    if (fb < ub + bytes && ub < fb + bytes) return fail(DFMM_EINVAL, "f and u overlap");
    ReqTable R{};
    R.f[0] = static_cast<const float2*>(f);
    R.u[0] = static_cast<float2*>(u);
    R.k0[0] = 0;
    R.n = 1;
    DeviceScope on(plan->device);
    run_apply_noalloc(*plan, R, nrhs, static_cast<hipStream_t>(stream));
    return int(DFMM_OK);
  });
}

int dfmm_workspace_bytes(dfmm_plan_t plan, int nrhs, size_t* bytes) {
  return guarded([&]() {
    if (!plan || !bytes) return fail(DFMM_EINVAL, "null plan or output");
    if (nrhs < 1 || nrhs > 4096) return fail(DFMM_EINVAL, "nrhs must be in [1, 4096]");
    *bytes = workspace_bytes(*plan, nrhs);
    return int(DFMM_OK);
  });
}

void dfmm_destroy(dfmm_plan_t plan) {
  if (!plan) return;
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != plan->device) (void)hipSetDevice(plan->device);
  destroy_apply_state(plan->ws);
  plan->ws = nullptr;
  delete plan->timer;
  plan->timer = nullptr;
  const int dev = plan->device;
  delete plan;
  if (cur != dev) (void)hipSetDevice(cur);
}

int dfmm_plan_info(dfmm_plan_t plan, dfmm_info* info) {
  if (!plan || !info) return fail(DFMM_EINVAL, "null argument");
  *info = plan->info;
  return DFMM_OK;
}

int dfmm_export(dfmm_plan_t plan, int what, int level, void* buf, size_t* bytes) {
  return guarded([&]() {
    if (!plan || !bytes) return fail(DFMM_EINVAL, "null argument");
    const std::vector<int64_t>* v = nullptr;
    auto lvl_ok = [&]() { return level >= 0 && level <= plan->D; };
    auto any_lvl = [&]() { return level >= 0 && level < int(plan->boxes.size()); };  // LF levels below D too
    switch (what) {
      case DFMM_EXPORT_PERM: v = &plan->perm; break;
      case DFMM_EXPORT_BOXES: if (any_lvl()) v = &plan->boxes[level]; break;
      case DFMM_EXPORT_PAIRS: if (any_lvl()) v = &plan->pairs[level]; break;
      case DFMM_EXPORT_NEAR: v = &plan->near; break;
      case DFMM_EXPORT_LEAVES: v = &plan->leaves; break;
      case DFMM_EXPORT_OUT_SLOTS: if (lvl_ok()) v = &plan->out_slots[level]; break;
      case DFMM_EXPORT_IN_SLOTS: if (lvl_ok()) v = &plan->in_slots[level]; break;
      default: break;
    }
    if (!v) return fail(DFMM_EINVAL, "bad export selector or level");
    size_t need = v->size() * sizeof(int64_t);
    if (!buf) {
      *bytes = need;
      return int(DFMM_OK);
    }
    if (*bytes < need) return fail(DFMM_EINVAL, "buffer too small");
    std::memcpy(buf, v->data(), need);
    *bytes = need;
    return int(DFMM_OK);
  });
}

int dfmm_set_timing(dfmm_plan_t plan, int applies) {
  return guarded([&]() {
    if (!plan) return fail(DFMM_EINVAL, "null plan");
    if (applies < 0 || applies > 100000) return fail(DFMM_EINVAL, "applies must be in [0, 100000]");
    DeviceScope on(plan->device);
    delete plan->timer;
    plan->timer = nullptr;
    if (applies > 0) plan->timer = new StageTimer(applies);
    return int(DFMM_OK);
  });
}

int dfmm_stage_times(dfmm_plan_t plan, double* ms, int64_t* launches, int cap, int* n) {
  return guarded([&]() {
    if (!plan || !n || !ms || !launches) return fail(DFMM_EINVAL, "null argument");
    if (!plan->timer) return fail(DFMM_EINVAL, "timing is not enabled on this plan");
    DeviceScope on(plan->device);
    double t[ST_COUNT];
    int64_t c[ST_COUNT];
    plan->timer->collect(t, c);
    int k = std::min(cap < 0 ? 0 : cap, int(ST_COUNT));
    for (int i = 0; i < k; ++i) {
      ms[i] = t[i];
      launches[i] = c[i];
    }
    *n = k;
    return int(DFMM_OK);
  });
}

}  // extern "C"
