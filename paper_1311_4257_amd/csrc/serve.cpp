// Serving loop of libdfmm (contract in include/dfmm.h): the request scheduler
// of batcher.hpp wired to dfmm_apply_batch, one stream per plan, with pass
// completion reported by a host function enqueued behind each pass.
#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "batcher.hpp"
#include "internal.hpp"

struct dfmm_server_s {
  std::vector<dfmm_plan_t> plans;
  std::vector<hipStream_t> streams;
  // workspace bytes of each plan at 0 .. 4096 right-hand sides, computed at
  // creation, so the scheduler never calls into a plan under its own lock
  std::vector<std::vector<size_t>> wsb;
  int device = 0;
  std::unique_ptr<dfmm::Batcher> B;
};

namespace {

int fail(int code, const char* msg) {
  dfmm::set_error(msg);
  return code;
}

struct PassDone {
  dfmm::Batcher* B;
  int64_t pass;
};

// Runs on the runtime's callback thread once the stream has reached the end of
// the pass: host bookkeeping only, no HIP call.
void pass_done(void* p) {
  auto* d = static_cast<PassDone*>(p);
  d->B->complete(d->pass, DFMM_OK);
  delete d;
}

void destroy_streams(dfmm_server_s* S) {
  for (hipStream_t s : S->streams) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  S->streams.clear();
}

}  // namespace

extern "C" {

int dfmm_server_create(const dfmm_plan_t* plans, int nplans, size_t hbm_budget_bytes, int max_batch_rhs,
                       int single, dfmm_server_t* out) {
  if (!out) return fail(DFMM_EINVAL, "null output");
  *out = nullptr;
  if (!plans || nplans < 1) return fail(DFMM_EINVAL, "need at least one plan");
  if (max_batch_rhs < 1 || max_batch_rhs > 4096) return fail(DFMM_EINVAL, "max_batch_rhs must be in [1, 4096]");
  const int dev = plans[0] ? plans[0]->device : 0;
  size_t resident = 0;
  for (int p = 0; p < nplans; ++p) {
    if (!plans[p]) return fail(DFMM_EINVAL, "null plan");
    if (plans[p]->device != dev) return fail(DFMM_EINVAL, "the plans of a server must share one device");
    if (plans[p]->prec == DFMM_PREC_FP64) return fail(DFMM_EUNSUPPORTED, "float64 plans do not take batched passes");
    for (int q = 0; q < p; ++q)
      if (plans[q] == plans[p]) return fail(DFMM_EINVAL, "a plan appears twice");
    resident += size_t(plans[p]->info.device_bytes);
  }
  auto S = std::make_unique<dfmm_server_s>();
  S->plans.assign(plans, plans + nplans);
  S->device = dev;
  S->wsb.resize(size_t(nplans));
  for (int p = 0; p < nplans; ++p) {
    S->wsb[size_t(p)].resize(4097, 0);
    for (int n = 1; n <= 4096; ++n) {
      const int st = dfmm_workspace_bytes(plans[p], n, &S->wsb[size_t(p)][size_t(n)]);
      if (st != DFMM_OK) return st;
    }
  }
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return fail(DFMM_EDEVICE, "hipGetDevice failed");
  if (cur != dev && hipSetDevice(dev) != hipSuccess) return fail(DFMM_EDEVICE, "hipSetDevice failed");
  for (int p = 0; p < nplans; ++p) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      destroy_streams(S.get());
      if (cur != dev) (void)hipSetDevice(cur);
      return fail(DFMM_EDEVICE, "hipStreamCreateWithFlags failed");
    }
    S->streams.push_back(s);
  }
  if (cur != dev) (void)hipSetDevice(cur);
  dfmm_server_s* raw = S.get();
  auto ws = [raw](int p, int n) {
    return n >= 0 && n <= 4096 ? raw->wsb[size_t(p)][size_t(n)] : (~size_t(0)) / 4;
  };
  auto launch = [raw](int p, const std::vector<const dfmm::ServeReq*>& rs, int, int64_t b) -> int {
    std::vector<const void*> f;
    std::vector<void*> u;
    std::vector<int> k;
    for (const dfmm::ServeReq* r : rs) {
      f.push_back(r->f);
      u.push_back(r->u);
      k.push_back(r->nrhs);
    }
    hipStream_t s = raw->streams[size_t(p)];
    const int st = dfmm_apply_batch(raw->plans[size_t(p)], int(rs.size()), f.data(), u.data(), k.data(), s);
    if (st != DFMM_OK) return st;
    auto* d = new PassDone{raw->B.get(), b};
    if (hipSetDevice(raw->device) != hipSuccess || hipLaunchHostFunc(s, pass_done, d) != hipSuccess) {
      delete d;
      (void)hipStreamSynchronize(s);
      return DFMM_EDEVICE;
    }
    return DFMM_OK;
  };
  S->B = std::make_unique<dfmm::Batcher>(nplans, resident, hbm_budget_bytes, max_batch_rhs, DFMM_MAX_BATCH,
                                         single != 0, ws, launch);
  *out = S.release();
  return DFMM_OK;
}

int dfmm_server_submit(dfmm_server_t s, int plan, const void* f, void* u, int nrhs, int64_t* ticket) {
  if (!s) return fail(DFMM_EINVAL, "null server");
  if (plan >= 0 && plan < int(s->plans.size()) && f && u && nrhs >= 1 && nrhs <= 4096) {
    const char* fb = static_cast<const char*>(f);
    const char* ub = static_cast<const char*>(u);
    const size_t bytes = size_t(8) * size_t(s->plans[size_t(plan)]->N) * size_t(nrhs);
    if (fb < ub + bytes && ub < fb + bytes) return fail(DFMM_EINVAL, "f and u overlap");
  }
  const int st = s->B->submit(plan, f, u, nrhs, ticket);
  if (st == DFMM_EINVAL) return fail(st, "bad plan index, vector, nrhs or ticket pointer");
  if (st == DFMM_ENOMEM) return fail(st, "the request does not fit the server's HBM budget");
  return st;
}

int dfmm_server_wait(dfmm_server_t s, int64_t ticket, double* t_submit, double* t_done) {
  if (!s) return fail(DFMM_EINVAL, "null server");
  return s->B->wait(ticket, t_submit, t_done);
}

int dfmm_server_drain(dfmm_server_t s) {
  if (!s) return fail(DFMM_EINVAL, "null server");
  s->B->drain();
  return DFMM_OK;
}

double dfmm_server_now(dfmm_server_t s) { return s ? s->B->now() : 0.0; }

int dfmm_server_passes(dfmm_server_t s, int64_t* n) {
  if (!s || !n) return fail(DFMM_EINVAL, "null argument");
  *n = s->B->passes();
  return DFMM_OK;
}

int dfmm_server_pass(dfmm_server_t s, int64_t pass, int* plan, int* nreq, int* nrhs) {
  if (!s || !plan || !nreq || !nrhs) return fail(DFMM_EINVAL, "null argument");
  dfmm::ServePass P;
  if (!s->B->pass(pass, &P)) return fail(DFMM_EINVAL, "no such pass");
  *plan = P.plan;
  *nreq = int(P.ids.size());
  *nrhs = P.nrhs;
  return DFMM_OK;
}

int dfmm_server_footprint(dfmm_server_t s, size_t* bytes) {
  if (!s || !bytes) return fail(DFMM_EINVAL, "null argument");
  *bytes = s->B->footprint_now();
  return DFMM_OK;
}

void dfmm_server_destroy(dfmm_server_t s) {
  if (!s) return;
  s->B.reset();  // waits for every submitted request, then stops the worker
  int cur = 0;
  const bool ok = hipGetDevice(&cur) == hipSuccess;
  if (ok && cur != s->device) (void)hipSetDevice(s->device);
  destroy_streams(s);
  if (ok && cur != s->device) (void)hipSetDevice(cur);
  delete s;
}

}  // extern "C"
