/*
 * dfmm.h -- C ABI of the directional fast multipole matvec for MI355X (gfx950).
 *
 * Computes u_i = sum_{j : p_j != p_i} G(p_i, p_j) f_j with
 * G(x, y) = exp(2 pi i |x - y|) / |x - y| (Eq. 1 of Benson, Poulson, Tran,
 * Engquist, Ying, "A parallel directional fast multipole method", Section 1),
 * approximately, by the evaluation pass of the sequential directional FMM
 * (Algorithm 1, Section 2.3) plus the near-field sum between adjacent leaves.
 *
 * Conventions shared by every call:
 *   - Lengths are in wavelengths; the points satisfy |p| <= K/2 (Eq. 1) and the
 *     root box is the cube [-K/2, K/2]^3; K is a power of two >= 1.
 *   - Every function returns an int status (DFMM_OK = 0 or a negative
 *     dfmm_status); no C++ exception crosses the ABI.  dfmm_last_error()
 *     returns a thread-local message describing the last failure.
 *   - Host pointers are read during the call only; the library copies what it
 *     keeps.  Device pointers must stay valid until the work enqueued on the
 *     stream has completed.
 *   - Calls that work on a plan make its device current for their duration
 *     and leave the caller's current device as they found it, also on failure.
 */
#ifndef DFMM_H
#define DFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DFMM_OK = 0,
  DFMM_EINVAL = -1,       /* bad argument: null pointer, N < 1, nrhs < 1, bad size */
  DFMM_EDOMAIN = -2,      /* a point is not finite or |p| > K/2 (1 + 1e-12) */
  DFMM_EUNSUPPORTED = -3, /* K not a power of two, eps out of range, tree wider than the operator set */
  DFMM_ENOMEM = -4,       /* host or device allocation failed */
  DFMM_EDEVICE = -5,      /* a HIP call failed */
  DFMM_EIO = -6           /* operator-set file could not be read or written */
} dfmm_status;

typedef struct dfmm_plan_s* dfmm_plan_t;
typedef struct dfmm_opset_s* dfmm_opset_t;

/* Human-readable name of a status code (static storage). */
const char* dfmm_status_string(int status);
/* Detail of the last failure on the calling thread (empty if none). */
const char* dfmm_last_error(void);

/* ------------------------------------------------------------------------
 * Operator sets: the directional skeletons of Eq. 2 (Section 2.1).
 *
 * For each high-frequency width w in {1, 2, 4, ..., w_hi} and each of the
 * 6 w^2 wedges (cube-face cells, Section 2.2), and once for the
 * low-frequency width 1/2, a skeleton holds r equivalent points b (inside the
 * box, box-centred frame), r check points a (in the far region) and the r x r
 * complex matrix D with G(x, y) ~= sum_q G(x, b_q) sum_p D_qp G(a_p, y) for y
 * in the box and x in the wedge.  Skeletons depend only on (tau, w, wedge),
 * not on the geometry (Section 2.2), so one set serves every plan whose top
 * interaction width is <= w_hi.
 *
 * Width argument: w = 0.5 selects the low-frequency skeleton (dir must be 0);
 * w = 1/4, 1/8, ..., 1/128 the deeper low-frequency widths of adaptive trees
 * (dir 0; dfmm_opset_set adds them to a set, dfmm_opset_build builds them
 * when an adaptive plan first needs them); w = 1, 2, 4, ... selects a
 * high-frequency width, dir in [0, 6 w^2).
 * Point arrays are r x 3 row-major float64; D is r x r row-major complex128
 * stored as interleaved (re, im) doubles.
 * ---------------------------------------------------------------------- */

/* Build a set with the library's own float64 precompute (column-pivoted QR,
 * Eq. 2): tau is the relative Frobenius truncation of each skeleton.  Uses
 * all host cores; results are cached in cache_dir when it is non-null. */
int dfmm_opset_build(double tau, int w_hi, const char* cache_dir, dfmm_opset_t* out);
/* An empty set to be filled with dfmm_opset_set (every skeleton must be set
 * before the set is used by a plan). */
int dfmm_opset_create(double tau, int w_hi, dfmm_opset_t* out);
/* Copy one skeleton into the set (r >= 1). */
int dfmm_opset_set(dfmm_opset_t set, double w, int dir, int r,
                   const double* a, const double* b, const double* D);
/* Query one skeleton: *r receives its rank; a, b, D (may be null) receive
 * copies of size r*3, r*3 and 2*r*r doubles. */
int dfmm_opset_get(dfmm_opset_t set, double w, int dir, int* r,
                   double* a, double* b, double* D);
/* tau and w_hi of a set. */
int dfmm_opset_info(dfmm_opset_t set, double* tau, int* w_hi);
/* Binary file round trip (little-endian; format documented in the source). */
int dfmm_opset_save(dfmm_opset_t set, const char* path);
int dfmm_opset_load(const char* path, dfmm_opset_t* out);
void dfmm_opset_destroy(dfmm_opset_t set);

/* ------------------------------------------------------------------------
 * Plans
 * ---------------------------------------------------------------------- */

typedef struct {
  double eps;             /* end-to-end relative L2 target; selects tau when opset is null */
  dfmm_opset_t opset;     /* skeletons to use (borrowed; must outlive the plan's creation
                             call only -- the plan copies what it needs); null = build */
  const char* cache_dir;  /* cache directory (may be null; DFMM_CACHE_DIR is used then): operator
                             sets, and the GEMM launch choices the first apply of each nrhs
                             measures (dfmm_tune_*.txt, keyed by launch shapes, nrhs, device) */
  int device;             /* HIP device ordinal; -1 = current device */
  int precision;          /* DFMM_PREC_*: arithmetic of the translation GEMMs (default FP32) */
  double leaf_width;      /* width of the first low-frequency level in wavelengths; 0 = the default
                             1/2, the only value accepted (DFMM_EUNSUPPORTED otherwise); finer
                             leaves come from leaf_max */
  double tol_factor;      /* skeleton truncation tau = tol_factor * eps (Eq. 2 holds to tau per
                             translation, Section 2.1; the end-to-end error is a small multiple of
                             it); 0 = the calibrated default (0.1 for eps >= 1e-5, else 0.03);
                             must lie in (0, 1]; ignored when opset is given */
  uint64_t hbm_budget_bytes; /* device bytes the plan may hold (0 = no limit): a plan that would
                             exceed it returns DFMM_ENOMEM -- checked on the host before any
                             device allocation against a lower bound of the plan's size (its
                             points and per-point tables), and again against the built plan */
  int leaf_max;           /* adaptive low-frequency tree (Section 2.2): a box of width <= 1/2 splits
                             while it holds more than leaf_max points, down to lf_levels levels below
                             width 1/2; each LF width has its own skeleton, LF-M2M / LF-L2L run
                             between the LF levels and leaves of different sizes that are adjacent
                             at the coarser one's level are summed directly in the near field.
                             0 = the uniform tree (all leaves of width 1/2).  Float32 plans with
                             eps >= 1e-5 only (DFMM_EUNSUPPORTED otherwise); an explicit operator set
                             must then hold the deeper LF skeletons (dfmm_opset_set with
                             w = 1/4, 1/8, ...) */
  int lf_levels;          /* levels below width 1/2 an adaptive tree may reach: 1..6, 0 = 3 */
  int reserved[2];
} dfmm_options;

/* Arithmetic of the translation GEMMs (M2M, M2L, L2L) of a plan.  FP32: float32
 * MFMA.  FP16X3 / BF16X3: every operator entry a and vector entry x is split into
 * a hi and a lo part of the 16-bit type (a = a_hi + a_lo to 22 resp. 16 bits)
 * and a x is formed as a_hi x_hi + a_hi x_lo + a_lo x_hi on the 16-bit MFMA with
 * float32 accumulation.  FP16X3 scales each operator (at plan time) and each
 * source vector (per GEMM column, at staging) by a power of two into the fp16
 * range and unscales the sums, and keeps float32-level accuracy; BF16X3 needs no
 * scaling and keeps about 16 bits.  The near field and the leaf passes stay in
 * float32 / float64.  Split precision is for fast plans only (eps >= 1e-5):
 * DFMM_EINVAL otherwise. */
#define DFMM_PREC_FP32 0
#define DFMM_PREC_FP16X3 1
#define DFMM_PREC_BF16X3 2
/* FP64: the whole pass in float64 (Table 1 of the paper goes to eps = 1e-8):
 * densities f and potentials u are complex128 (interleaved double re, im),
 * the leaf weights, check potentials and translation operators float64, the
 * GEMMs on v_mfma_f64_16x16x4f64 and the near-field sum with float64 sin/cos.
 * Accepts 1e-8 <= eps <= 1e-2; the skeleton tolerance is the float32 rule's
 * but not below 1e-9.  The middle factors D of Eq. 2 grow like 1/tau, so the
 * float64 rounding of the check potentials reaches u amplified by ~1/tau, and
 * the float64 precompute holds Eq. 2 on fresh samples to 3e-8 .. 1e-7 at
 * tau = 1e-9: an eps = 1e-8 plan gives a relative error of 6e-8 .. 2e-7
 * against the direct sum (K = 4 and 8 spheres), the floor of this
 * factorisation in float64.  dfmm_apply and dfmm_apply_ws serve these
 * plans (workspace from dfmm_workspace_bytes); dfmm_apply_batch and
 * dfmm_apply_noalloc return DFMM_EUNSUPPORTED for them. */
#define DFMM_PREC_FP64 3

/* Fill *opt with defaults: eps 1e-4, no opset, no cache, current device, FP32,
 * leaf width 1/2, the calibrated tau rule, no HBM budget. */
void dfmm_options_default(dfmm_options* opt);

/* Plan for N points (host pointer, N x 3 row-major float64, original order)
 * in a domain of width K with end-to-end target eps (1e-6 <= eps <= 1e-2; below
 * 1e-6 the float32 equivalent densities and check potentials set the floor).
 * Builds the Morton-sorted octree (leaf width 1/2), the interaction lists of
 * every level (Section 2.2), the wedge labels, the needed directions and the
 * translation tables, all resident on the device.  Synchronous.
 * The skeletons use tau = 0.1 eps (eps >= 1e-5) or 0.03 eps (or tol_factor eps,
 * see dfmm_options); they depend only on tau and the box width, not on the
 * geometry (Section 2.2), and are cached in the cache directory.  Plans with
 * eps < 1e-5 (or an operator set with tau < 3e-6) are "precise": the
 * near-field distances, 1/r and products are float64, the directional
 * operators are stored as float32 hi + lo parts, and every translation GEMM adds
 * its float32 sums into float64 partial sums every 32 products. */
int dfmm_plan(const double* points, int64_t N, double K, double eps, dfmm_plan_t* out);
int dfmm_plan_ex(const double* points, int64_t N, double K, const dfmm_options* opt,
                 dfmm_plan_t* out);

/* u = A f for nrhs right-hand sides.  f and u are DEVICE pointers to complex64
 * data (interleaved float re, im), layout [nrhs][N], in the caller's original
 * point order; u is overwritten; f and u must not overlap.  Work is enqueued
 * on `stream` (a hipStream_t; null = the null stream) and the call returns
 * without waiting.  The first apply with a new nrhs grows the plan's workspace
 * if nrhs is the largest so far (synchronous allocation) and fixes the GEMM
 * launch shapes for it: for a power of two from the tuning record in the cache
 * directory if one matches, else by timing the candidate shapes on `stream`
 * (waits for them; DFMM_AUTOTUNE=0 takes the default shapes instead), including
 * whether the M2L launches of all levels run fused into one (DFMM_FUSED=0 or 1
 * forces the separate or the fused form); for
 * other nrhs from the power of two below (see dfmm_apply_batch).  Later
 * applies with the same nrhs allocate nothing and do not wait.  The near-field sum runs on a second stream owned by the
 * plan (default priority), forked from and joined back into `stream` with
 * events, so the apply is complete when `stream` reaches its end.  Applies on
 * one plan must not run concurrently.  An apply may be captured into a HIP
 * graph (stream capture on `stream`) once an uncaptured apply with the same
 * nrhs has run on the plan; the captured apply reads f and writes u at the
 * addresses given at capture.  Capturing before that returns DFMM_EINVAL;
 * stage timing is off inside a capture.  A captured graph stays valid when a
 * later apply with more right-hand sides grows the workspace: once a plan has
 * been captured, the workspaces it replaces are kept until dfmm_destroy. */
int dfmm_apply(dfmm_plan_t plan, const void* f, void* u, int nrhs, void* stream);

/* Batched form of dfmm_apply for a request loop: nreq (1 .. DFMM_MAX_BATCH)
 * requests on one plan in one pass.  Request r has nrhs[r] >= 1 right-hand
 * sides at DEVICE pointer f[r] and its result goes to u[r] (both complex64,
 * [nrhs[r]][N], caller's point order; total nrhs <= 4096).  The pass sees one
 * apply with sum(nrhs) right-hand sides: the densities are gathered from the
 * requests' buffers by the first kernel and the potentials scattered to
 * theirs by the last, without staging copies; every result equals what
 * dfmm_apply gives for that request alone up to the float32 rounding of the
 * translations (the column order of a batch does not change a column's
 * arithmetic).  The host arrays are read before the call returns.  No output
 * may overlap an input or another output (DFMM_EINVAL).  The workspace grows to
 * the largest total nrhs seen and keeps the GEMM launch shapes of every total
 * nrhs seen.  Only powers of two are tuned; any other total takes the shapes
 * of the largest power of two below it (tuned first if needed) and builds
 * only its chunk tables, so a loop with many batch sizes allocates and tunes
 * a few times at its start.  Stream, capture and concurrency rules as for
 * dfmm_apply. */
#define DFMM_MAX_BATCH 32
int dfmm_apply_batch(dfmm_plan_t plan, int nreq, const void* const* f, void* const* u, const int* nrhs,
                     void* stream);

/* Device bytes of the apply workspace for nrhs right-hand sides (vectors, pair
 * scratch, sorted densities and near-field sums), for admission against an HBM
 * budget and for sizing the workspace of dfmm_apply_ws; the plan's own memory is
 * dfmm_info.device_bytes.  The plan-owned workspace of dfmm_apply is grow-only:
 * it holds the size of the largest nrhs applied so far. */
int dfmm_workspace_bytes(dfmm_plan_t plan, int nrhs, size_t* bytes);

/* dfmm_apply with a caller-owned workspace: `ws` is a DEVICE pointer to at least
 * dfmm_workspace_bytes(plan, nrhs) bytes (256-byte aligned; DFMM_EINVAL if null,
 * misaligned or too small), which the apply uses for every intermediate vector
 * and which must not be touched until the stream has reached the end of the
 * apply.  The repeated-call use is the matvec inside an iterative boundary
 * integral solver (Section 1): several such solves can share one plan, and
 * their applies may run concurrently, from several host threads and on
 * several streams, as long as each in-flight apply has its own workspace (the
 * plan itself is read-only in an apply; the first apply of a new nrhs on a plan
 * prepares its launch shapes under a lock and may allocate and time them, as
 * dfmm_apply does).  Everything, the near-field sum included, runs on `stream`.
 * f, u, nrhs, layout, stream and capture rules as for dfmm_apply; u is
 * overwritten. */
int dfmm_apply_ws(dfmm_plan_t plan, const void* f, void* u, int nrhs, void* ws, size_t ws_bytes, void* stream);

/* dfmm_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): it
 * calls no allocator.  Its workspace is a static device array of the library,
 * DFMM_NOALLOC_MAX_BYTES bytes on every GPU the library runs on, held until the
 * process ends; an apply whose workspace (dfmm_workspace_bytes) is larger
 * returns DFMM_EINVAL.  The launch shapes come from an earlier dfmm_apply (or
 * dfmm_apply_ws / dfmm_apply_batch) with the same nrhs on this plan; without one
 * the call returns DFMM_EINVAL.  Everything runs on `stream`.  Every call on one
 * GPU uses that GPU's array, which keeps the last call's contents (no apply
 * reads workspace memory it has not written): calls that overlap on one GPU --
 * on different streams, from different threads or plans -- race, so the caller
 * serializes them.  f, u, nrhs, layout and stream as for dfmm_apply. */
#define DFMM_NOALLOC_MAX_BYTES (64u << 20)
int dfmm_apply_noalloc(dfmm_plan_t plan, const void* f, void* u, int nrhs, void* stream);

void dfmm_destroy(dfmm_plan_t plan);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of matvec requests over resident plans.
 *
 * An iterative boundary-integral solver issues one matvec per iteration
 * (Section 1); a serving process keeps the plans of several geometries on one
 * device and takes such requests as they come.  A server owns one stream per
 * plan (default priority) and a worker thread.  The worker starts a plan's next
 * pass (one dfmm_apply_batch) as soon as the plan's previous pass has
 * finished, so passes of different plans run concurrently and requests that
 * arrive while a plan is busy join its next pass.  A pass takes the plan's
 * queued requests in submission order, up to max_batch_rhs right-hand sides
 * (a longer request runs alone) and DFMM_MAX_BATCH requests, while the HBM
 * footprint stays within hbm_budget_bytes.  The footprint counts the resident
 * plans (dfmm_info.device_bytes) plus each plan's workspace at the largest
 * pass it has run (dfmm_workspace_bytes; workspaces only grow).  Plans whose
 * oldest queued request is older start first.  With single != 0 a pass holds
 * one request and one pass runs at a time, in submission order: the plain
 * form, for comparison.  Completion is reported by a host function enqueued
 * behind each pass; nothing polls.
 *
 * The plans must share one device and must not be applied elsewhere while the
 * server lives; float64 plans are refused (DFMM_EUNSUPPORTED).  Each request
 * reads f and writes u (DEVICE pointers, complex64, [nrhs][N], caller's point
 * order, not overlapping): f must hold its values when dfmm_server_submit is
 * called (synchronize the stream that wrote them first), and neither may be
 * touched or freed until dfmm_server_wait has returned for it.  A request that
 * can never fit the budget fails with DFMM_ENOMEM, at submission when it does
 * not fit then, else in its dfmm_server_wait.  Times are seconds on the
 * server's monotonic clock (dfmm_server_now, 0 at creation): t_submit when the
 * request was taken, t_done when the host function after its pass ran. */
typedef struct dfmm_server_s* dfmm_server_t;
int dfmm_server_create(const dfmm_plan_t* plans, int nplans, size_t hbm_budget_bytes, int max_batch_rhs,
                       int single, dfmm_server_t* out);
/* Queues a request for plan index `plan` (into the array given at creation);
 * *ticket names it in dfmm_server_wait.  Thread-safe; does not wait. */
int dfmm_server_submit(dfmm_server_t s, int plan, const void* f, void* u, int nrhs, int64_t* ticket);
/* Blocks until the request has finished; returns its status (DFMM_OK, or the
 * error of its pass).  Either time pointer may be null. */
int dfmm_server_wait(dfmm_server_t s, int64_t ticket, double* t_submit, double* t_done);
/* Blocks until no request is queued or in flight. */
int dfmm_server_drain(dfmm_server_t s);
double dfmm_server_now(dfmm_server_t s);
/* Passes started so far, and pass i's plan index, request count and total nrhs. */
int dfmm_server_passes(dfmm_server_t s, int64_t* n);
int dfmm_server_pass(dfmm_server_t s, int64_t i, int* plan, int* nreq, int* nrhs);
/* The current HBM footprint under the admission rule. */
int dfmm_server_footprint(dfmm_server_t s, size_t* bytes);
/* Waits for every submitted request, then frees the server (not the plans). */
void dfmm_server_destroy(dfmm_server_t s);

/* ------------------------------------------------------------------------
 * Introspection (tests and benchmarks)
 * ---------------------------------------------------------------------- */

typedef struct {
  int64_t N;
  double K;
  int depth;              /* D: leaves are at level D, width 1/2 */
  int w_top;              /* largest width with a non-empty interaction list (0 if none) */
  int nlevels_hf;         /* number of HF levels from w_top down to 1 */
  int64_t boxes[32];      /* non-empty boxes per level 0..D */
  int64_t pairs[32];      /* interaction pairs per level 0..D (0 where no list) */
  int64_t offsets[32];    /* distinct offsets per level */
  int64_t out_slots[32];  /* needed outgoing (box, wedge) slots per HF level */
  int64_t in_slots[32];   /* needed incoming (box, wedge) slots per HF level */
  int rank[32];           /* skeleton size (padded) per level (HF levels and the leaf level) */
  int64_t near_pairs;     /* adjacent leaf pairs, self included */
  int64_t near_point_pairs; /* point pairs of the near-field sum (targets x sources) */
  double flops_m2l_hf;    /* 8 r_in r_out summed over HF pairs, per right-hand side */
  double flops_m2l_lf;    /* 8 r r summed over leaf-level pairs, per right-hand side */
  double plan_seconds;
  int64_t device_bytes;   /* device memory held by the plan (without the apply workspace) */
  double bytes_m2l_op;    /* M2L operators (complex64, unpadded r_in x r_out), once per offset group */
  double bytes_m2l_vec;   /* M2L vectors per right-hand side: every source slot read once (8 r_out) and
                             every target slot read and written once (16 r_in), complex64, unpadded */
  double flops_m2l_level[32]; /* flops_m2l_hf / flops_m2l_lf split by level 0..D */
  double tau;             /* skeleton tolerance of the plan's operator set */
  double flops_m2m;       /* HF-M2M: 8 r_parent r_child per (out-slot, child), per right-hand side */
  double flops_l2l;       /* HF-L2L (into the leaves too): 8 r_child r_parent per (in-slot, parent wedge),
                             per right-hand side */
  double bytes_l2l_op;    /* HF-L2L operators used (complex64, unpadded r_child x r_parent), once each */
  double bytes_l2l_vec;   /* HF-L2L vectors per right-hand side: every parent incoming slot read once */
  int64_t leaves;         /* leaves (= boxes[depth] in a uniform tree) */
  int depth_max;          /* deepest level with boxes (> depth in an adaptive tree) */
  int reserved_i;
} dfmm_info;

int dfmm_plan_info(dfmm_plan_t plan, dfmm_info* info);

/* Export a plan structure into a host buffer.  If buf is null, *bytes receives
 * the size needed.  `level` selects the level where relevant.
 *   DFMM_EXPORT_PERM        int64[N]: original index of each sorted point
 *   DFMM_EXPORT_BOXES       int64[nb][5]: (ix, iy, iz, first point, end point), Morton order
 *   DFMM_EXPORT_PAIRS       int64[np][5]: (B, A, dir_in, dir_out, 0), sorted by (B, A);
 *                           boxes are indices into that level's box table; dirs -1 at the leaves
 *   DFMM_EXPORT_NEAR        int64[np][2]: near-field leaf pairs (B, A), sorted (leaf indices:
 *                           level-D boxes in a uniform tree, DFMM_EXPORT_LEAVES rows in an
 *                           adaptive one)
 *   DFMM_EXPORT_LEAVES      int64[nleaf][4]: (level, box, first point, end point) of every leaf,
 *                           in point order (adaptive trees; boxes as in DFMM_EXPORT_BOXES)
 *   DFMM_EXPORT_OUT_SLOTS   int64[ns][2]: needed outgoing (box, dir), sorted
 *   DFMM_EXPORT_IN_SLOTS    int64[ns][2]: needed incoming (box, dir), sorted */
enum {
  DFMM_EXPORT_PERM = 1,
  DFMM_EXPORT_BOXES = 2,
  DFMM_EXPORT_PAIRS = 3,
  DFMM_EXPORT_NEAR = 4,
  DFMM_EXPORT_OUT_SLOTS = 5,
  DFMM_EXPORT_IN_SLOTS = 6,
  DFMM_EXPORT_LEAVES = 7
};
int dfmm_export(dfmm_plan_t plan, int what, int level, void* buf, size_t* bytes);

/* Stage timing with HIP events recorded on the apply stream after every
 * launch (no host synchronisation inside dfmm_apply).  dfmm_set_timing(plan, n)
 * enables recording for up to n following applies (n = 0 disables and frees
 * the events).  dfmm_stage_times waits for the recorded work, writes per stage
 * the summed milliseconds and the number of launches over all recorded
 * applies, and restarts the recording.  Stages, in order:
 *   0 permute-in, 1 S2M, 2 HF-M2M, 3 HF-M2L (grouped GEMM), 4 HF-M2L reduction,
 *   5 HF-L2L, 6 LF-M2L (grouped GEMM), 7 LF-M2L reduction,
 *   8 leaf evaluation (L2T, adds the near field, permute-out), 9 zero fill,
 *   10 near field (on the plan's second stream, concurrent with stages 1-7).
 * Stages 0-9 are intervals between launches on the apply stream (they add up
 * to the apply time); stage 10 overlaps them.
 * *n receives the number of stages written (<= cap). */
enum { DFMM_NUM_STAGES = 11 };
int dfmm_set_timing(dfmm_plan_t plan, int applies);
int dfmm_stage_times(dfmm_plan_t plan, double* ms, int64_t* launches, int cap, int* n);

#ifdef __cplusplus
}
#endif
#endif /* DFMM_H */
