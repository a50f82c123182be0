/*
 * hull.h - C ABI of the MI355X (gfx950) interior-point-discarding 2D convex
 * hull library.
 *
 * The method is G. Mei's preprocessing for planar convex hulls (arXiv:1405.3454,
 * "A Straightforward Preprocessing Approach for Accelerating Convex Hull
 * Computations on the GPU"): find extreme points of the point set along the
 * axes of the original and of three rotated copies (Sec. 2, Step 1), form
 * their convex polygon with Andrew's algorithm (Step 2), discard every point
 * strictly inside it (Step 3) and compute the hull of the remaining points
 * (Sec. 3, case (2)).  Every step runs in this library's own HIP kernels.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Points are structure-of-arrays float32 x[n], y[n] in DEVICE memory owned
 *    by the caller, each 4-byte aligned and both at the same address modulo
 *    16 (for example equal offsets into two 16-byte aligned arrays); reads
 *    may touch the up to three floats before x[0] and y[0] that share their
 *    16-byte block, never anything beyond x[n-1].  The exactness guarantees hold for
 *    coordinates that are multiples of 2^-24 in [0, 1) (HULL_VALIDATE checks
 *    this); on that grid every orientation test is exact in binary64.
 *  - Indices are uint32 positions into x/y, global even in the batched
 *    calls; HULL_NONE = 2^32 - 1 marks an empty slot, so n <= 2^32 - 2
 *    (larger n: HULL_ETOOBIG).
 *  - Every output array is caller-owned device memory; counts are written to
 *    device memory (int64).  Calls are asynchronous on `stream` (a hipStream_t
 *    passed as void*, NULL = the null stream) and never synchronise, except
 *    with HULL_VALIDATE, which synchronises to report domain errors.
 *  - The context owns a device workspace that grows on demand; growth is not
 *    possible while `stream` is being captured into a graph (HULL_ECAPTURE):
 *    call once outside capture with the largest sizes first.
 *  - Extreme slots: for rotation group g (angle t, constants c = cos t,
 *    s = sin t) the rotated coordinates are u = c*x - s*y and v = s*x + c*y,
 *    each product rounded to binary64 and then the sum (no fused multiply-add).
 *    slots[4g+0] = argmin u, [4g+1] = argmax u, [4g+2] = argmin v,
 *    [4g+3] = argmax v; ties go to the lowest index.  A set has
 *    hull_slot_count() slots: max(16, 4G) fixed positions for a preset of G
 *    groups (positions past 4G hold HULL_NONE), then, with HULL_LEARNED, the
 *    argmax of c*x + s*y along eight directions chosen per set by the learned
 *    proposal (only for presets of at most 16 fixed slots).
 *  - Polygon and hull vertex lists are counter-clockwise, start at the
 *    lexicographically smallest (x, y), exclude collinear points and name a
 *    repeated coordinate pair by its lowest index.
 *  - Survivors (points not strictly inside the polygon; boundary points
 *    survive; a polygon with fewer than 3 vertices discards nothing) are
 *    listed in ascending index order.
 *
 * Errors: every call returns HULL_OK or a negative code; hull_strerror() names
 * it and hull_last_hip_error() gives the underlying hipError_t for HULL_EHIP.
 */
#ifndef HULL_H
#define HULL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hull_ctx hull_ctx;

#define HULL_OK 0
#define HULL_EINVAL (-1)   /* null pointer, bad size, bad preset, misaligned */
#define HULL_ETOOBIG (-2)  /* n > 2^32 - 2 (index 2^32 - 1 is HULL_NONE) */
#define HULL_ENOMEM (-3)   /* workspace allocation failed */
#define HULL_EHIP (-4)     /* HIP runtime error, see hull_last_hip_error() */
#define HULL_EDOMAIN (-5)  /* HULL_VALIDATE: coordinate off the 2^-24 grid of [0,1) */
#define HULL_ECAPTURE (-6) /* workspace would have to grow during stream capture */
#define HULL_ENOMODEL (-7) /* HULL_LEARNED without loaded network weights */
#define HULL_ESCRATCH (-8) /* input larger than hull_extremes_noalloc's fixed scratch */
#define HULL_EOVERFLOW (-9) /* more survivors than the caller's output capacity */

/* direction presets (angles of the rotated copies, Sec. 2 Step 1) */
#define HULL_DIRS_PAPER 0      /* 0, 30, 45, 60 degrees (Figure 1, Sec. 5) */
#define HULL_DIRS_CUMULATIVE 1 /* 30, 45, 45 of Sec. 2 read cumulatively: 0, 30, 75, 120 */
/* Direction families beyond the paper's table: G = 1..6 rotation groups at
 * 90 j / G degrees (j = 0..G-1), i.e. 4G evenly spaced extreme directions.
 * G = 1 is the min/max x and y quadrilateral, the simplest preprocessing
 * filter the paper cites (Sec. 1, ref. [3]); G = 4 gives 16 evenly spaced
 * directions, as many as the paper's table. */
#define HULL_DIRS_EVEN(G) (1 + (G))
#define HULL_DIRS_QUAD HULL_DIRS_EVEN(1)
#define HULL_NUM_PRESETS 8

/* flags */
#define HULL_NOFILTER 1 /* hull of all points, no preprocessing (Sec. 3, case (1)) */
#define HULL_LEARNED 2  /* add eight learned directions to the sixteen fixed slots */
#define HULL_VALIDATE 4 /* check the input domain first (synchronises) */
#define HULL_NOREFINE 8 /* hull of the survivors by sort + chain alone, without the
                           QuickHull refinement rounds that shrink them first */

#define HULL_NCOUNTS 5  /* entries of hull_candidate_counts: the discard pass, then
                           each of the four refinement rounds */

#define HULL_NONE 0xFFFFFFFFu
#define HULL_FIXED_SLOTS 16
#define HULL_MAX_SLOTS 24

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device` (made current by each call). */
int hull_create(hull_ctx **ctx, int device);
/* Free the context, its workspace, graphs and network weights. */
int hull_destroy(hull_ctx *ctx);
/* Select the rotation angles of Step 1 (HULL_DIRS_*, 0 <= preset <
 * HULL_NUM_PRESETS); default PAPER.  HULL_EINVAL for an unknown preset. */
int hull_set_directions(hull_ctx *ctx, int preset);
/* Slots per set that hull_extremes(_batched) writes for this context's
 * preset with these flags (only HULL_LEARNED matters): 16 for the paper's
 * presets, max(16, 4G) for an even family, plus 8 with HULL_LEARNED.
 * HULL_EINVAL for a null ctx, or HULL_LEARNED with more than 16 fixed slots. */
int hull_slot_count(hull_ctx *ctx, int flags);
/* Host-only: copy a direction table into c[], s[] (capacity cap).
 * which = 0: the rotation groups of ctx's preset (PAPER if ctx is NULL);
 * which = 1: the 64 candidate directions 2*pi*d/64 of the learned proposal;
 * which = 16 + p: the rotation groups of preset p (ctx not needed).
 * Returns the number of entries or a negative code (HULL_EINVAL for a null
 * array, an unknown table or cap below the table's size). */
int hull_direction_table(hull_ctx *ctx, int which, double *c, double *s, int cap);
const char *hull_strerror(int code);
int hull_last_hip_error(hull_ctx *ctx);

/* ---- Step 1: extreme points (Sec. 2, Step 1) --------------------------- */
/* slots: device uint32[hull_slot_count(ctx, flags)]; vals: device
 * double[same] with the extreme values (NaN for HULL_NONE slots), or NULL.
 * n == 0 gives HULL_NONE.  HULL_EINVAL for HULL_LEARNED with a preset of
 * more than 16 fixed slots; HULL_ENOMODEL without network weights. */
int hull_extremes(hull_ctx *ctx, const float *x, const float *y, int64_t n,
                  uint32_t *slots, double *vals, int flags, void *stream);

/* Allocation-free form of hull_extremes, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments and results as
 * hull_extremes (plain slots only: flags must be 0), but its working memory
 * is a fixed array of HULL_NOALLOC_SCRATCH_BYTES in device memory that the
 * library holds on each device from hull_create until the process ends; the
 * call itself allocates and frees nothing and records no timing events.
 * Limits: n <= HULL_NOALLOC_MAX_POINTS, else HULL_ESCRATCH.  Every call on
 * one device shares that device's array, so calls that overlap on one
 * device (two streams, two threads, two contexts) race: serialise them. */
#define HULL_NOALLOC_MAX_POINTS (1LL << 27)
#define HULL_NOALLOC_SCRATCH_BYTES (40u << 20)
int hull_extremes_noalloc(hull_ctx *ctx, const float *x, const float *y, int64_t n,
                          uint32_t *slots, double *vals, int flags, void *stream);

/* ---- Step 2: convex polygon of the extremes (Sec. 2, Step 2) ----------- */
/* slots: device uint32[n_slots] (n_slots <= 24, HULL_NONE entries ignored).
 * verts: device uint32[n_slots]; m: device int32, the vertex count. */
int hull_polygon(hull_ctx *ctx, const float *x, const float *y, int64_t n,
                 const uint32_t *slots, int n_slots, uint32_t *verts, int32_t *m,
                 void *stream);

/* ---- Step 3: discard interior points (Sec. 2, Step 3) ------------------ */
/* Builds the polygon of `slots` and writes the survivors (ascending indices)
 * to surv (device uint32, capacity n) and their count to *n_surv (device). */
int hull_discard(hull_ctx *ctx, const float *x, const float *y, int64_t n,
                 const uint32_t *slots, int n_slots, uint32_t *surv,
                 int64_t *n_surv, void *stream);

/* ---- hull of a subset (the hull of the remaining points, Sec. 3) ------- */
/* idx: device uint32 list of point indices (e.g. survivors), its length in
 * device memory *k_dev, at most k_cap.  hull: device uint32 (capacity k_cap),
 * *h: device int64. */
int hull_of_subset(hull_ctx *ctx, const float *x, const float *y, int64_t n,
                   const uint32_t *idx, const int64_t *k_dev, int64_t k_cap,
                   uint32_t *hull, int64_t *h, void *stream);

/* ---- the whole method -------------------------------------------------- */
/* Steps 1-3 and the hull of the survivors (HULL_NOFILTER: hull of all
 * points).  hull: device uint32 (capacity n); *h: device int64. */
int hull_compute(hull_ctx *ctx, const float *x, const float *y, int64_t n,
                 uint32_t *hull, int64_t *h, int flags, void *stream);

/* ---- host-resident input (the paper's setting, Sec. 3) ----------------
 * The whole method for a set that lives in HOST memory (pageable or pinned),
 * as on the paper's 1 GB card: the points cross PCIe in chunks of
 * chunk_points (0: 2^24; rounded up to a multiple of 1024), copies
 * overlapped with the kernels on a second stream.  Pass 1 runs Step 1 on
 * each chunk and reduces the extremes across chunks (better value, then
 * lower index: the same slots as hull_extremes on the whole set); pass 2
 * builds the polygon of those extremes and runs Step 3 on each chunk,
 * appending its survivors.  Chunks beyond two streaming buffers stay on the
 * device after pass 1 while they fit in device_budget bytes (8 B per point;
 * a budget for the whole set means one crossing); the rest cross again.
 * The hull of the survivors runs on the device (sort + monotone chain; no
 * refinement rounds).
 *   slots: device uint32[hull_slot_count(ctx, 0)] or NULL;
 *   surv: device uint32[cap], survivors in ascending index order; *n_surv
 *         (device int64) their count;
 *   hull: device uint32[cap]; *h (device int64) its size.
 * Synchronises the stream (the staging buffers are reused, and the survivor
 * count sizes the hull stage).  flags must be 0.  Errors: HULL_EINVAL,
 * HULL_ETOOBIG, HULL_ENOMEM (chunk buffers, staging or workspace),
 * HULL_EHIP, HULL_EOVERFLOW when more than cap points survive (*n_surv then
 * holds the true count, only the first cap survivors are written and no
 * hull is computed). */
int hull_compute_host(hull_ctx *ctx, const float *x, const float *y, int64_t n,
                      int64_t chunk_points, int64_t device_budget, uint32_t *slots,
                      uint32_t *surv, int64_t *n_surv, int64_t cap, uint32_t *hull,
                      int64_t *h, int flags, void *stream);

/* ---- three dimensions (the extension the paper's Sec. 5 names) ---------
 * The method for one set of points x[n], y[n], z[n] (device float32 on the
 * 2^-24 grid of [0,1)^3, each array 16-byte aligned):
 *  Step 1: extremes along rotations about each axis: for each rotation group
 *    (c, s) of the context's preset (the paper's two four-group tables only;
 *    other presets: HULL_EINVAL) and each plane (a, b) = (x, y), (y, z),
 *    (z, x) -- rotations about z, x and y -- the extremes of u = c*a - s*b and
 *    v = s*a + c*b (products rounded to binary64, then the sum), and of the
 *    axis coordinate itself: six per rotation.  The 42 distinct slots:
 *    [0..5] argmin/argmax of x, y, z; then 6 + 4 (3 k + g - 1) +
 *    {argmin u, argmax u, argmin v, argmax v} for plane k = 0, 1, 2 and
 *    group g = 1..3; lowest index on ties.
 *  Step 2: the convex polyhedron of the slot points (exact predicates).
 *  Step 3: every point strictly inside it is discarded; boundary points
 *    survive; a polyhedron without interior discards nothing.
 *  Step 4: the extreme points of the survivors (vertices of their convex
 *    hull; points on an edge or a face that are not corners excluded; a
 *    repeated coordinate triple named by its lowest index).
 * slots: device uint32[42] or NULL; surv: device uint32[n] (survivors in
 * ascending order) or NULL; *n_surv: device int64 or NULL; hull: device
 * uint32[n], the extreme points in ascending index order; *h: device int64.
 * The hull stage runs in rounds: every face's farthest candidate is
 * proposed, and the proposals whose faces seen and horizon neighbours no
 * higher proposal claims are inserted together; with HULL3_SERIAL one block
 * inserts every face's farthest candidate in turn instead (the same result;
 * a slower form kept for checking and for proposals that see more than 512
 * faces, which the parallel rounds hand to it).
 * flags: 0, HULL_NOFILTER (hull of all points), HULL3_SERIAL.  Synchronises
 * (the hull stage sizes itself from the survivor count).
 * Errors: HULL_EINVAL (null output, misaligned input, bad flags or preset),
 * HULL_ETOOBIG, HULL_ENOMEM, HULL_EHIP. */
#define HULL3_SLOTS 42
#define HULL3_SERIAL 16 /* hull stage: one insertion at a time, one block */
int hull3_compute(hull_ctx *ctx, const float *x, const float *y, const float *z, int64_t n,
                  uint32_t *slots, uint32_t *surv, int64_t *n_surv, uint32_t *hull, int64_t *h,
                  int flags, void *stream);

/* ---- batched forms (many sets, CSR offsets) ----------------------------
 * S: 1 .. 65535 sets.
 * offsets: device int64[S+1], non-decreasing, offsets[0] = 0,
 * offsets[S] = n_total (checked with HULL_VALIDATE).  Set s is points
 * [offsets[s], offsets[s+1]).  Indices stay global. */
int hull_extremes_batched(hull_ctx *ctx, const float *x, const float *y,
                          const int64_t *offsets, int64_t S, int64_t n_total,
                          uint32_t *slots /* [S * hull_slot_count] */, int flags,
                          void *stream);
int hull_discard_batched(hull_ctx *ctx, const float *x, const float *y,
                         const int64_t *offsets, int64_t S, int64_t n_total,
                         const uint32_t *slots, int n_slots, uint32_t *surv,
                         int64_t *surv_offsets /* [S+1] */, void *stream);
int hull_compute_batched(hull_ctx *ctx, const float *x, const float *y,
                         const int64_t *offsets, int64_t S, int64_t n_total,
                         uint32_t *hull, int64_t *hull_offsets /* [S+1] */,
                         int flags, void *stream);

/* ---- graphs ------------------------------------------------------------
 * Record hull_compute_batched with these arguments into a hipGraph (the
 * workspace is sized first, outside capture) and replay it with
 * hull_graph_launch; the pointers are baked into the graph. */
int hull_graph_capture(hull_ctx *ctx, const float *x, const float *y,
                       const int64_t *offsets, int64_t S, int64_t n_total,
                       uint32_t *hull, int64_t *hull_offsets, int flags,
                       void *stream);
int hull_graph_launch(hull_ctx *ctx, void *stream);

/* ---- launch tuning ------------------------------------------------------
 * The two persistent filter kernels (0: the extremes pass, 1: the discard
 * pass) launch with a shape: threads per block (128, 256 or 512), blocks
 * per CU (1..16, capped at what stays resident for that kernel) and the
 * fewest tiles of 1024 points (16 per lane) a wave walks (1..1024; small
 * inputs get fewer waves).  Shapes are kept per size bucket: points below
 * 2^14, 2^17, 2^20, 2^23, 2^26 and above, each for one set (S = 1) and for
 * batches (S > 1); untuned buckets use the defaults (256, 3, 1) and
 * (256, 4, 1).  No shape changes any result.
 *
 * hull_autotune times every candidate shape of both kernels on these
 * inputs (the discard pass in the full method's mode) and keeps the
 * fastest for their bucket.  Synchronises; allocates only outside capture. */
int hull_autotune(hull_ctx *ctx, const float *x, const float *y,
                  const int64_t *offsets, int64_t S, int64_t n_total, void *stream);
/* Read (get != 0) or set the default blocks per CU of the two kernels.
 * Setting them also clears every tuned bucket. */
int hull_tuning(hull_ctx *ctx, int get, int *k1_blocks_per_cu, int *k3_blocks_per_cu);
/* Read (get != 0) or set the shape of kernel 0 or 1 for the bucket holding
 * n points in S sets.  Get returns 1 when the bucket is tuned, 0 when it
 * uses the default; set returns HULL_OK, or HULL_EINVAL for a shape outside
 * the ranges above. */
int hull_shape(hull_ctx *ctx, int get, int kernel, int64_t n, int64_t S, int *block_size,
               int *blocks_per_cu, int *tiles_per_wave);
/* The tuned buckets as rows of six int32 (kernel, size bucket 0..5,
 * batched 0/1, block size, blocks per CU, tiles per wave); copies up to cap
 * rows and returns how many are tuned. */
int hull_tuning_table(hull_ctx *ctx, int32_t *rows, int cap);

/* ---- learned direction proposal ----------------------------------------
 * This project's extension, not part of the paper's method.  A 32 x 32
 * occupancy histogram of each set (hull_histogram_batched) feeds an MLP
 * 1024 -> 512 -> 512 -> 64 (ReLU; bf16 weights and activations, fp32
 * accumulation on MFMA) that scores the 64 directions 2*pi*d/64; the eight
 * best become extra extreme slots.  Extra extremes only enlarge the filter
 * polygon inside the hull, so every hull stays exact whatever the weights.
 *
 * Parameters: one float32 array of hull_mlp_param_count() values in the
 * order W1[512][1024], b1[512], W2[512][512], b2[512], W3[64][512], b3[64]
 * (W[out][in]); host memory in the set/get calls. */
int64_t hull_mlp_param_count(void);
int hull_mlp_set_params(hull_ctx *ctx, const float *params_host, int64_t count);
int hull_mlp_get_params(hull_ctx *ctx, float *params_host, int64_t count);
/* Training state, for checkpoint and resume: count = 3 * hull_mlp_param_count()
 * float32 values in host memory -- the parameters, then Adam's first moments,
 * then its second moments, each in the parameter order above -- and the step
 * count (the bias corrections of the next step use step + 1).  After
 * hull_mlp_set_state the next hull_mlp_train_step continues exactly where the
 * saved run stopped (hull_mlp_set_params instead starts a new run: moments
 * zero, step 0).  Synchronous.  Errors: HULL_EINVAL (count, null pointers,
 * step < 0; get before any parameters were set). */
int hull_mlp_get_state(hull_ctx *ctx, float *state_host, int64_t count, int64_t *step);
int hull_mlp_set_state(hull_ctx *ctx, const float *state_host, int64_t count, int64_t step);
/* hist: device bf16 bits [S][1024]; hist_f32: device float [S][1024] or NULL.
 * offsets NULL means one set of n_total points (S must be 1).  The sample
 * is every point when n <= 16384, else 256 runs of 64 consecutive points,
 * run r starting at floor(r (n - 64) / 255); the bins cover a square window centred
 * on the sample's bounding box, its side the box's longer side (so the
 * set's aspect ratio is kept); value = count * 1024 / sample size. */
int hull_histogram_batched(hull_ctx *ctx, const float *x, const float *y,
                           const int64_t *offsets, int64_t S, int64_t n_total,
                           uint16_t *hist, float *hist_f32, void *stream);
/* scores: device float [B][64]. */
int hull_mlp_forward(hull_ctx *ctx, const uint16_t *hist, int64_t B, float *scores,
                     void *stream);
/* Gradient of sum(dscores * scores) w.r.t. every parameter (device float
 * [param_count]); dscores is rounded to bf16 first. */
int hull_mlp_backward(hull_ctx *ctx, const uint16_t *hist, const float *dscores, int64_t B,
                      float *grads, void *stream);
/* One Adam step (beta 0.9/0.999, eps 1e-8) on the mean squared error between
 * the scores and gain / max(gain) per set; *loss (device float) gets the loss
 * before the step. gain: device float [B][64]. */
int hull_mlp_train_step(hull_ctx *ctx, const uint16_t *hist, const float *gain, int64_t B,
                        float lr, float *loss, void *stream);
/* The eight chosen directions per set (device int32 [S][8]) for scores
 * [S][64]: highest first, lower index on ties, NaN as -inf; with a direction
 * gap g (hull_set_direction_gap) each pick also rules out the directions
 * within g steps of it on the circle of 64. */
int hull_top_directions(hull_ctx *ctx, const float *scores, int64_t S, int32_t *dirs,
                        void *stream);
/* Minimum spacing of the learned picks: gap g in [0, 3] (default 2) makes
 * any two of the eight chosen directions at least g + 1 of the 64 steps
 * apart, for hull_top_directions and for the HULL_LEARNED paths.
 * Errors: HULL_EINVAL for g outside [0, 3]. */
int hull_set_direction_gap(hull_ctx *ctx, int gap);
/* Training labels (device float [S][64]): for direction d, the fraction of the
 * set's points that the plain filter keeps but the polygon of the sixteen
 * fixed extremes plus the extreme along d discards. */
int hull_labels_batched(hull_ctx *ctx, const float *x, const float *y, const int64_t *offsets,
                        int64_t S, int64_t n_total, float *gain, void *stream);
/* Greedy joint training targets (device float [S][64]) and the greedy order
 * (device int32 [S][rounds], -1 after the sequence ends), 1 <= rounds <= 8.
 * Starting from the fixed filter's polygon, each round adds the candidate
 * direction whose extreme point makes the polygon strictly contain the most
 * of the fixed filter's survivors not yet contained (ties: lowest direction);
 * a round without gain ends the sequence.  The direction chosen in round r
 * gets 1 - r / (2 rounds); every other direction d gets 0.5 g_d / max g, g_d
 * its gain in the first round (0 if all are 0).  Targets peak at 1, so
 * hull_mlp_train_step's scaling by the per-set maximum leaves them as they
 * are.  Errors: HULL_EINVAL for rounds outside [1, 8]. */
int hull_label_targets_batched(hull_ctx *ctx, const float *x, const float *y,
                               const int64_t *offsets, int64_t S, int64_t n_total, int rounds,
                               float *target, int32_t *order, void *stream);

/* ---- per-kernel timing (hipEvents around every launch) ----------------- */
int hull_timing_enable(hull_ctx *ctx, int on);
/* Copy accumulated milliseconds and launch counts for up to cap kernel
 * kinds; names via hull_timing_name().  Synchronises.  Returns the count. */
int hull_timing_read(hull_ctx *ctx, double *ms, int64_t *launches, int cap);
const char *hull_timing_name(int kind);
int hull_timing_reset(hull_ctx *ctx);

/* ---- candidate counts (diagnostics) ------------------------------------ */
/* Copy up to cap (at most HULL_NCOUNTS) counts, summed over all sets, of the
 * context's last hull_compute / hull_compute_batched call (or graph replay):
 * [0] candidates handed to the hull stage's input, i.e. the discard pass's
 * survivors (every point with HULL_NOFILTER); [1 + r] candidates left after
 * QuickHull refinement round r (each round splits every polygon edge at its
 * farthest survivor), -1 when refinement did not run.  Synchronises the
 * device.  Returns the number of entries copied; HULL_EINVAL for a null
 * pointer or cap < 0. */
int hull_candidate_counts(hull_ctx *ctx, int64_t *counts, int cap);

#ifdef __cplusplus
}
#endif
#endif /* HULL_H */
