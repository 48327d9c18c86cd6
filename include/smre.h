/*
 * smre.h -- C ABI of the MI355X (gfx950) SMRE projection library.
 *
 * What it computes (paper: "Parallel Statistical Multi-resolution Estimation",
 * arXiv 1503.03492):
 *   - the Euclidean projection of a residual image x0 onto
 *       { v : sum_{i in S} v_i^2 <= r2_S  for every square window S }
 *     (the feasible set tau_G of Sec. 2, Eqs. (tau_s), (tau_G); the projection
 *     P_G of Sec. 2.2), by Dykstra's cyclic projection algorithm (Sec. 2.3,
 *     Algorithm 2, single-set projection Eq. (dykstra:if)).  The family holds
 *     every s x s square lying fully inside the image, for each configured
 *     side s.  The paper writes the constraint as c_s * sum <= 1; here the
 *     bound r2_S = 1/c_s is passed directly.
 *   - the paper's incomplete Dykstra (ICD) of Sec. 3.2: squares of side 2^k
 *     (k <= K) on lattices shifted diagonally by 2^i, projected blockwise.
 *
 * Conventions.
 *   - Every function returns an int status (smre_status); no exception or
 *     abort crosses this boundary.  SMRE_NOT_CONVERGED is a warning: the
 *     result has been written.
 *   - Image buffers are row-major with a row stride `ld` (elements, ld >= W).
 *     `x` arguments of the projection calls are DEVICE pointers, updated in
 *     place; the caller owns them.  Bounds, sides and reports are HOST memory.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *     it in order.  The projection calls return after the result is complete
 *     (the convergence test needs the host), so `x` may be read right away.
 *   - A context (smre_ctx) is bound to one device; it caches workspaces and
 *     tuning results.  It is not thread-safe: use one per host thread.
 */
#ifndef SMRE_H
#define SMRE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SMRE_OK = 0,
  SMRE_NOT_CONVERGED = 1, /* warning: sweep cap reached, result written        */
  SMRE_PENDING = 2,       /* serving: ticket not finished yet                  */
  SMRE_EINVAL = -1,       /* invalid argument                                  */
  SMRE_ENONFINITE = -2,   /* NaN or Inf in the input image or the bounds       */
  SMRE_ENOMEM = -3,       /* device allocation failed / workspace too small    */
  SMRE_ETOOBIG = -4,      /* request can never fit the memory budget           */
  SMRE_EBUSY = -5,        /* queue full                                        */
  SMRE_EDEVICE = -6,      /* HIP runtime error                                 */
  SMRE_ECANCELLED = -7,   /* server shut down before the ticket finished       */
  SMRE_EUNKNOWN_TICKET = -8
} smre_status;

typedef enum { SMRE_F32 = 0, SMRE_F64 = 1 } smre_dtype;       /* dtype of x        */
typedef enum { SMRE_INC_SAME = 0, SMRE_INC_BF16 = 1 } smre_inc; /* increment storage */
typedef enum { SMRE_TOL_MAXABS = 0, SMRE_TOL_MEANABS = 1 } smre_tolmode;
/* Cyclic order of the full projection (see "Sweep order" below). */
typedef enum { SMRE_ORDER_REGION = 0, SMRE_ORDER_DESC = 1, SMRE_ORDER_ASC = 2 } smre_order;

typedef struct smre_ctx smre_ctx;

/* Parameters of the full projection.
 *   sides[n_sides]    distinct window sides, 1 <= s <= min(H, W), s <= 32
 *   radius2[n_sides]  bound r2_s of the sum of squares over a window of side s
 *                     (finite, > 0)
 *   tol               stop after the first checked sweep whose largest
 *                     pixel change max_i |x_i - x_prev_i| (FP64) is < tol;
 *                     tol <= 0 runs exactly max_sweeps sweeps
 *   max_sweeps        sweep cap (>= 1)
 *   check_every       test convergence every this many sweeps (>= 1)
 *   region            side R of the anchor regions of the sweep order
 *                     (0 = choose; else 8, 16 or 32 with R >= max side - 1)
 *   inc               increment storage (FP32 x only for SMRE_INC_BF16)
 *   kahan             FP32: compensated per-lane window sums (0/1)
 *   warm              0: start from zero increments.  1: start from the
 *                     increments the previous smre_dykstra_project call left
 *                     in this workspace (same dtype, H, W, sides, bounds,
 *                     region and increment storage; SMRE_EINVAL otherwise,
 *                     also after a call that failed): Dykstra from any
 *                     increments reaches the same limit (it minimises the
 *                     dual function block by block), so a slowly moving
 *                     input -- the eps-step of Algorithm 1 -- needs fewer
 *                     sweeps.  x holds the new input x0; the iterate starts at
 *                     x0 - sum_S I_S, with sum_S I_S = x0_prev - z_prev kept
 *                     from the previous call (Dykstra's invariant)
 *   guard_rel         FP32: windows with |n - r2| <= guard_rel * r2 are
 *                     re-summed in FP64 before the threshold test (0 = off)
 *
 * Sweep order.  Dykstra's limit does not depend on the cyclic order of the
 * sets (Sec. 2.3).  order = SMRE_ORDER_REGION (the default, and the fast one)
 * needs no ordering between overlapping sets inside a kernel: the anchor
 * (top-left) plane is cut into R x R regions coloured 2 (p mod 2) + (q mod 2);
 * colour by colour, each region (p, q) visits its windows side by side
 * (descending), then offset (a', b') in raster order, where offset (a', b')
 * selects the windows anchored at (p R + a' + s i, q R + b' + s j) --
 * disjoint, so projected together.  Regions of one colour touch disjoint
 * pixels.  SMRE_ORDER_DESC / SMRE_ORDER_ASC: the canonical orders -- sides
 * descending / ascending, for each side s its s^2 tilings (a, b) in raster
 * order, a tiling being the disjoint windows anchored at (a + s i, b + s j);
 * one launch per tiling (several times slower: every launch re-reads the
 * image), the iterates of the paper's own visiting order (Algorithm 2 with
 * the sets grouped by tiling).  region is ignored for those orders.
 */
typedef struct {
  int32_t n_sides;
  const int32_t* sides;
  const double* radius2;
  double tol;
  int32_t max_sweeps;
  int32_t check_every;
  int32_t region;
  int32_t inc;
  int32_t kahan;
  int32_t warm;
  double guard_rel;
  int32_t order;      /* smre_order */
  int32_t reserved1;  /* 0 */
} smre_params;

typedef struct {
  int32_t sweeps;              /* sweeps run (the converged sweep if converged) */
  int32_t converged;           /* 1 if the tolerance was met                   */
  int32_t region;              /* region side R used                           */
  int32_t inner_sweeps;        /* ICD: total inner sweeps over all blocks       */
  double last_delta;           /* last measured max |x - x_prev| (FP64)         */
  double max_violation;        /* max_S sum_S x^2 / r2_S - 1 at exit (FP64)     */
  double elapsed_ms;           /* wall time of the call, device-side events     */
  double kernel_ms;            /* sum of sweep-kernel durations (timing on)     */
  double bytes_moved;          /* algorithmic HBM bytes of the sweeps           */
  double window_projections;   /* single-window projections performed           */
  int64_t kernel_launches;     /* sweep-kernel launches timed                   */
  double pixel_updates;        /* (window, pixel) pairs updated: the sum of the
                                  pixel counts of the projections performed     */
} smre_report;

const char* smre_status_string(int status);

/* Context bound to `device` (a HIP device ordinal). */
int smre_ctx_create(int device, smre_ctx** out);
void smre_ctx_destroy(smre_ctx* ctx);
/* Record HIP events around the sweep kernels (reported in smre_report as
 * kernel_ms and kernel_launches): every = 0 off, 1 around every launch, k > 1
 * around every k-th launch of a call (each event pair costs a launch gap, so a
 * long solve can be timed on a sample; kernel_ms and kernel_launches then
 * cover the timed launches only).  SMRE_EINVAL for every < 0. */
int smre_ctx_set_timing(smre_ctx* ctx, int every);

/* Window bounds on the host: chi-square(s*s degrees of freedom) p-quantile
 * for each side, i.e. the bound that i.i.d. N(0,1) noise meets with
 * probability p on one window. */
int smre_chi2_bounds(const int32_t* sides, int32_t n, double p, double* radius2_out);
/* The paper's weights (Sec. 2.1): r2 = 1/c_s = (q_alpha sigma_s + mu_s)^4,
 * mu_s = (|s| - 1/2)^(1/4), sigma_s^2 = 1/(8 sqrt|s|), |s| = side^2. */
int smre_paper_bounds(const int32_t* sides, int32_t n, double q_alpha, double* radius2_out);

/* Bytes of device workspace smre_dykstra_project needs for this problem. */
int smre_workspace_size(smre_dtype dtype, int64_t H, int64_t W, const smre_params* p,
                        size_t* bytes);

/* Full Dykstra projection of x (device, H x W, stride ld), in place.
 * workspace: device memory of at least smre_workspace_size bytes, or NULL
 * (the context allocates and caches it).  report may be NULL.
 * Returns SMRE_OK, SMRE_NOT_CONVERGED, or an error. */
int smre_dykstra_project(smre_ctx* ctx, smre_dtype dtype, void* x, int64_t H, int64_t W,
                         int64_t ld, const smre_params* p, void* workspace, size_t ws_bytes,
                         void* stream, smre_report* report);

/* Incomplete Dykstra (Sec. 3.2), in place on x (device).
 *   K             block side 2^K (0 <= K <= 6; K = 6 runs on the nested-hierarchy
 *                 kernel, smre_dykstra_incomplete_nested); levels k = 0..K
 *   radius2[K+1]  bound of a square of side 2^k
 *   tol, tolmode  block stopping rule after each inner sweep:
 *                 MAXABS: max |dx| < tol; MEANABS: sum |dx| <= tol * block pixels
 *   max_inner     cap on inner sweeps per block (>= 1; one always runs)
 *   num_phases    phases i = 0..num_phases-1 (1..K+1; the paper's family: K+1)
 * Phase i: blocks on the lattice shifted by 2^i mod 2^K on both axes; a block
 * projects onto its squares of side 2^k, k = K down to i, with increments
 * zeroed at the start of the phase.
 * Returns SMRE_OK, SMRE_NOT_CONVERGED (the result is written, but at least one
 * block stopped at max_inner without meeting tol; report->converged = 0), or
 * an error; SMRE_ENONFINITE (NaN or Inf in x) leaves x as it came.  The call
 * blocks the host once, after its last kernel: the input check runs on the
 * stream ahead of the phases, which leave x alone when it fails.  report (may
 * be NULL): counters, and max_violation over every window of the levels'
 * sides (a pass over x that is skipped when report is NULL). */
int smre_dykstra_incomplete(smre_ctx* ctx, smre_dtype dtype, void* x, int64_t H, int64_t W,
                            int64_t ld, int32_t K, const double* radius2, double tol,
                            int32_t tolmode, int32_t max_inner, int32_t num_phases, void* stream,
                            smre_report* report);

/* smre_dykstra_incomplete for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): same arguments, same results and report (except kernel_ms and
 * kernel_launches, which are 0: no per-kernel timing), but no hipMalloc,
 * hipFree or other allocating call on any path.  Its device scratch (the work
 * counters of the blocks) is a fixed 32,768-byte static array per GPU, located
 * when the context is created;
 * it does not grow with the image, so the only size limit is K <= 5
 * (SMRE_EINVAL beyond, as for smre_dykstra_incomplete).  Every call on one
 * GPU uses that GPU's single copy and overwrites it: calls that overlap on one
 * GPU (other host threads, other streams) race and must be serialised by the
 * caller.  The context still holds the control block (input check, counter
 * sums, feasibility report) and the events, allocated by smre_ctx_create. */
int smre_dykstra_incomplete_noalloc(smre_ctx* ctx, smre_dtype dtype, void* x, int64_t H,
                                    int64_t W, int64_t ld, int32_t K, const double* radius2,
                                    double tol, int32_t tolmode, int32_t max_inner,
                                    int32_t num_phases, void* stream, smre_report* report);

/* The incomplete Dykstra on every frame of a movie (the paper preprocesses the
 * frames of a fluorescence time series with it, Sec. 4): frames of H x W (row
 * stride ld) stacked
 * H ld elements apart from x (device), each projected in place exactly as
 * smre_dykstra_incomplete would project it alone; every phase is one launch
 * over all frames.  frames * H <= 2^31 - 1.  report: inner_sweeps, window and
 * pixel counts summed over frames; max_violation over all frames (report may be
 * NULL: the feasibility pass behind max_violation is then skipped). */
int smre_dykstra_incomplete_frames(smre_ctx* ctx, smre_dtype dtype, void* x, int64_t H,
                                   int64_t W, int64_t ld, int64_t frames, int32_t K,
                                   const double* radius2, double tol, int32_t tolmode,
                                   int32_t max_inner, int32_t num_phases, void* stream,
                                   smre_report* report);

/* The incomplete Dykstra over a caller-given family of phases (the paper's
 * family is one of them; Sec. 3.2 leaves the choice of subsets open): phase p
 * uses blocks of side 2^K on the lattice shifted by (shift_y[p], shift_x[p])
 * (0 <= shift < 2^K; blocks cut by the image edge are clipped) and projects
 * each block onto its squares of side 2^k, k = K down to min_level[p]
 * (0 <= min_level <= K), by Dykstra with increments zeroed at the phase start,
 * until the block meets the stopping rule.  radius2[K+1] bounds a square of
 * side 2^k.  1 <= n_phases <= 64.  Frames as in
 * smre_dykstra_incomplete_frames (frames = 1 for one image).  The paper's
 * family: shift 2^i mod 2^K on both axes and min_level i, i = 0..K. */
int smre_dykstra_incomplete_family(smre_ctx* ctx, smre_dtype dtype, void* x, int64_t H,
                                   int64_t W, int64_t ld, int64_t frames, int32_t K,
                                   const double* radius2, int32_t n_phases,
                                   const int32_t* shift_y, const int32_t* shift_x,
                                   const int32_t* min_level, double tol, int32_t tolmode,
                                   int32_t max_inner, void* stream, smre_report* report);

/* The incomplete Dykstra over a nested hierarchy of squares of any sides
 * (Sec. 3.2 with the sides 2^k replaced by a divisor chain; Sec. 5 names the
 * partition of the image as the method's open choice): level j
 * (0 <= j < n_levels <= 7) has squares of side level_side[j] (host array,
 * ascending, each dividing the next, at most 96) bounded by radius2[j]; the
 * block side is B = level_side[n_levels - 1].  Phase p uses blocks of side B
 * on the lattice shifted by (shift_y[p], shift_x[p]) (0 <= shift < B; blocks
 * cut by the image edge are clipped) and projects each block onto its squares
 * of the levels n_levels - 1 down to min_level[p] that lie inside the image, by
 * Dykstra with increments zeroed at the phase start, until the block meets the
 * stopping rule (as smre_dykstra_incomplete).  One workgroup per block: the
 * chain needs a level whose squares hold at most 16 pixels, with B^2 / that
 * many <= 1024 (<= 512 for 9 pixels, <= 256 for 16); SMRE_EINVAL otherwise
 * (so 1, 2, ..., 64, and 1, 3, 6, 12, 24, 48 run; 1, 5, 10, 20, 40 does not).
 * The chain 1, 2, ..., 2^K with shifts 2^i mod 2^K and lowest level i is the
 * paper's ICD; smre_dykstra_incomplete with K = 6 runs here.  Frames, report
 * and return codes as smre_dykstra_incomplete_family (max_violation over every
 * window of the levels' sides). */
int smre_dykstra_incomplete_nested(smre_ctx* ctx, smre_dtype dtype, void* x, int64_t H,
                                   int64_t W, int64_t ld, int64_t frames, int32_t n_levels,
                                   const int32_t* level_side, const double* radius2,
                                   int32_t n_phases, const int32_t* shift_y,
                                   const int32_t* shift_x, const int32_t* min_level, double tol,
                                   int32_t tolmode, int32_t max_inner, void* stream,
                                   smre_report* report);

/* ---- Batches: images of different sizes in one persistent launch per colour ----
 * Each image carries its own sides, bounds, tolerance and sweep cap; the
 * batch shares dtype, increment storage, Kahan flag, check cadence and the
 * region side R (all images need R >= their max side - 1).  One sweep is four
 * persistent launches (one per region colour) walking device work lists of
 * (image, region) items, then a per-image FP64 convergence check; images that
 * converge (or reach their cap) are retired and their items skipped.  Sweeps
 * are captured once in a HIP graph and replayed.  Every image gets exactly
 * the arithmetic it gets alone with the same R, so batched and single results
 * are bitwise equal. */
typedef struct {
  void* x;               /* device image (dtype of the call), row stride ld, in place */
  int64_t H, W, ld;
  int32_t n_sides;
  const int32_t* sides;  /* host */
  const double* radius2; /* host */
  double tol;            /* <= 0: run exactly max_sweeps sweeps */
  int32_t max_sweeps;
  int32_t reserved;
} smre_batch_image;

typedef struct {
  int32_t region;        /* 0 = autotune (cached in the context), else 8, 16 or 32 */
  int32_t inc;           /* smre_inc */
  int32_t kahan;
  int32_t check_every;   /* >= 1 */
  double guard_rel;
  int32_t use_graph;     /* replay HIP-graph-captured sweeps (1) or launch directly (0) */
  int32_t grid;          /* persistent workgroups per launch, 0 = from occupancy */
} smre_batch_params;

/* Device workspace bytes for a batch (covers every region side the tuner tries). */
int smre_batch_workspace_size(smre_dtype dtype, int32_t n, const smre_batch_image* imgs,
                              const smre_batch_params* bp, size_t* bytes);

/* Full Dykstra on n images at once; reports[n] (host) receives one report
 * per image (may be NULL).  workspace as in smre_dykstra_project.  Returns
 * SMRE_OK if every image with tol > 0 converged, SMRE_NOT_CONVERGED if some
 * hit their cap (results written), or an error. */
int smre_dykstra_project_batch(smre_ctx* ctx, smre_dtype dtype, int32_t n,
                               const smre_batch_image* imgs, const smre_batch_params* bp,
                               void* workspace, size_t ws_bytes, void* stream,
                               smre_report* reports);

/* ---- Serving: continuous batching of projection requests ----
 * A server owns one device, a memory arena of hbm_budget_bytes and a
 * scheduler thread.  submit() copies the host image and returns a ticket at
 * once; requests are admitted first-in first-out while an active slot is free
 * and their device footprint (increments, region table, image, snapshot)
 * fits the arena, and join the running set at the next sweep.  Each active
 * request advances by one sweep per step (the batched kernels, region side
 * 16, FP32 images), is checked in FP64 on its own cadence and retires when
 * it converges or reaches its cap; its slot and memory are then reused.
 * A request gets the same arithmetic alone or in any mix.  submit(), poll()
 * and stats() are thread-safe. */
typedef struct smre_server smre_server;
typedef struct {
  int device;
  size_t hbm_budget_bytes;  /* arena size (0 = 80% of free device memory) */
  int32_t max_active;       /* requests on the device at once */
  int32_t queue_cap;        /* queued requests beyond which submit returns SMRE_EBUSY */
  int32_t inc;              /* smre_inc */
  int32_t kahan;
  int32_t check_every;
  int32_t reserved;
  double guard_rel;
} smre_serve_config;

typedef struct {
  int64_t submitted, completed, rejected, failed, active, queued, sweeps, bytes_in_use;
  int64_t peak_active;     /* most requests on the device at once */
  int64_t joined_running;  /* admissions while other requests were mid-solve */
} smre_serve_counters;

int smre_serve_create(const smre_serve_config* cfg, smre_server** out);
/* Stops the scheduler; unfinished tickets are cancelled. */
void smre_serve_destroy(smre_server* s);
/* x_host: H x W row-major FP32 (copied before return).  p: sides, radius2
 * (max side 17), tol, max_sweeps; other fields come from the server config.
 * Errors: SMRE_EINVAL, SMRE_ENONFINITE, SMRE_ETOOBIG (can never fit the
 * arena), SMRE_EBUSY (queue full), SMRE_EDEVICE (server failed). */
int smre_serve_submit(smre_server* s, const float* x_host, int32_t H, int32_t W,
                      const smre_params* p, uint64_t* ticket);
/* SMRE_PENDING while queued or running.  Otherwise the ticket is released:
 * SMRE_OK / SMRE_NOT_CONVERGED with out_host (>= H W floats) and rep filled,
 * or the request's error.  latency_s (may be NULL): completion - submission. */
int smre_serve_poll(smre_server* s, uint64_t ticket, float* out_host, size_t out_elems,
                    smre_report* rep, double* latency_s);
int smre_serve_stats(smre_server* s, smre_serve_counters* out);

/* FP64 feasibility of x (device): *out = max_S sum_S x^2 / r2_S - 1 over all
 * windows of the given sides (1 <= side <= min(H, W), side <= 96; <= 0 means
 * every constraint holds). */
int smre_max_violation(smre_ctx* ctx, smre_dtype dtype, const void* x, int64_t H, int64_t W,
                       int64_t ld, int32_t n_sides, const int32_t* sides, const double* radius2,
                       void* stream, double* out);

/* ---- Monte-Carlo weights (Sec. 2.1, selection of the weights) ----
 * The paper balances the window bounds with q_alpha, the alpha-quantile of
 *   Q = max over windows S of ((t_S)^(1/4) - mu_s) / sigma_s,  t_S = sum_S e^2,
 * where e is an H x W field of i.i.d. N(0,1) values, mu_s = (s^2 - 1/2)^(1/4)
 * and sigma_s^2 = 1/(8 s); the bounds are then r2_s = (q_alpha sigma_s + mu_s)^4
 * (smre_paper_bounds).  These calls estimate q_alpha by sampling fields; the
 * family is every s x s window inside the field, for each listed side
 * (1 <= s <= min(H, W), s <= 32, distinct, at most 32 sides).
 *
 * Drawn fields: pixel p = i W + j (row-major) of field f is normal number
 * (p mod 4) of the Philox4x64-10 block (Salmon, Moraes, Dror, Shaw, SC 2011)
 * with counter {p / 4, f, 0, 0} and key {seed, 0}; words (w0, w1) and (w2, w3)
 * give two normals each by Box-Muller: u = ((w >> 11) + 1/2) 2^-53,
 * z = sqrt(-2 ln u0) cos(2 pi u1), z' = sqrt(-2 ln u0) sin(2 pi u1).
 * Sums, transform and maximum are FP64.  H, W <= 2^20.  Results go to HOST
 * arrays; each call returns when they are written. */

/* Fields field0 .. field0 + n_fields - 1 to out (device, FP64): field k at
 * out + k H ld, row stride ld >= W. */
int smre_mc_fields(smre_ctx* ctx, int64_t H, int64_t W, uint64_t seed, int64_t field0,
                   int64_t n_fields, double* out, int64_t ld, void* stream);

/* Q of the drawn fields field0 .. field0 + n_fields - 1: q_out[n_fields]
 * (host).  tmax_out (host, may be NULL): [n_fields][n_sides], the largest
 * window sum of squares of each side, sides in the caller's order.  report
 * (may be NULL): elapsed_ms, kernel_ms / kernel_launches of the window kernels
 * (when timing is on), window_projections = windows evaluated. */
int smre_mc_statistic(smre_ctx* ctx, int64_t H, int64_t W, int32_t n_sides, const int32_t* sides,
                      uint64_t seed, int64_t field0, int64_t n_fields, double* q_out,
                      double* tmax_out, void* stream, smre_report* report);

/* As smre_mc_statistic, for caller-supplied fields (device, dtype FP32 or
 * FP64): field k at fields + k H ld elements, row stride ld >= W. */
int smre_mc_statistic_fields(smre_ctx* ctx, smre_dtype dtype, const void* fields, int64_t H,
                             int64_t W, int64_t ld, int64_t n_fields, int32_t n_sides,
                             const int32_t* sides, double* q_out, double* tmax_out, void* stream);

/* q_alpha from fields 0 .. n_fields - 1: the ceil(alpha n_fields)-th smallest
 * Q (0 < alpha <= 1).  report as in smre_mc_statistic. */
int smre_mc_quantile(smre_ctx* ctx, int64_t H, int64_t W, int32_t n_sides, const int32_t* sides,
                     uint64_t seed, int64_t n_fields, double alpha, double* q_alpha, void* stream,
                     smre_report* report);

/* ---- ADMM outer loop (Sec. 2.2, Algorithm 1, split form) ----
 * Minimises G(eps) + lam/2 ||z||^2 subject to I = A x + eps and z = x, where
 * A is a Gaussian PSF of width sigma px (zero outside the image; taps
 * k = -R..R with R = floor(4 sigma + 1/2) <= 32, weights exp(-k^2 / (2 sigma^2))
 * normalised to sum 1; sigma = 0 is the identity) and G the multi-resolution
 * constraint.  Starting from x = eps = z = Y1 = Y2 = 0, each iteration:
 *   x   <- x - (-A (rho1 (I - A x - eps) + Y1) + rho2 (x - z) + Y2) / (2 gamma)
 *   eps  = P_G(I - A x + Y1 / rho1)      (ICD or full Dykstra, below)
 *   z    = (rho2 x + Y2) / (lam + rho2)
 *   Y1  += alpha1 (I - A x - eps),  Y2 += alpha2 (x - z)
 * and it stops once ||x_new - x||_2 <= delta and ||I - A x - eps||_2 <= delta
 * (FP64 sums), or after max_iter iterations.  The defaults of the paper's
 * parameter file: rho1 6.192, rho2 1.8, alpha1 1.2, alpha2 0.12, lam 1. */
typedef enum { SMRE_ADMM_ICD = 0, SMRE_ADMM_FULL = 1 } smre_admm_method;

typedef struct {
  double sigma, lam, rho1, rho2, alpha1, alpha2;
  double gamma;          /* x-step stabilisation; <= 0: (rho1 + rho2) / 2 */
  double delta;          /* stopping threshold; < 0: run exactly max_iter */
  int32_t max_iter;      /* >= 1 */
  int32_t method;        /* smre_admm_method */
  /* ICD projection: K, radius2_icd[K+1], the inner rule (tolmode, tol, cap) */
  int32_t K;
  int32_t icd_tolmode;
  double icd_tol;
  int32_t icd_max_inner;
  int32_t warm;          /* full projection: 1 = every eps-step after the first
                            starts from the previous one's increments */
  const double* radius2_icd;
  /* full projection: sides, radius2, tol, max_sweeps, ... (smre_params) */
  const smre_params* full;
} smre_admm_params;

typedef struct {
  int32_t iterations;    /* iterations run */
  int32_t converged;     /* 1 if the delta rule stopped it */
  double last_dx;        /* ||x_new - x||_2 of the last iteration */
  double last_residual;  /* ||I - A x - eps||_2 of the last iteration */
  double elapsed_ms;     /* wall time of the call */
  double projection_ms;  /* of which in the projections (host clock) */
  int64_t projection_sweeps;  /* inner sweeps (ICD) or sweeps (full), summed */
} smre_admm_report;

/* I: device image (dtype, row stride ld), read only; x: device output (same
 * layout), the estimate.  eps_out (device, same layout, may be NULL): the
 * final eps.  H, W <= 65535.  Errors as for the projections; SMRE_ENOMEM if
 * the working set (10 images) cannot be allocated. */
int smre_admm(smre_ctx* ctx, smre_dtype dtype, const void* I, void* x, int64_t H, int64_t W,
              int64_t ld, const smre_admm_params* p, void* eps_out, void* stream,
              smre_admm_report* report);

#ifdef __cplusplus
}
#endif
#endif /* SMRE_H */
