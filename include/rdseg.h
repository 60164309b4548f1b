/*
 * rdseg.h -- C ABI of the MI355X (gfx950) implementation of the restricted-domain
 * dual method for convexly relaxed two-phase segmentation
 * (Spencer, arXiv 1807.11534).
 *
 * The method minimises TV(u) + lambda <f, u> over u in [0, 1] (Sec. 2, eq. CR)
 * with the split energy of eq. DF (Sec. 2.1), alternating
 *   - Chambolle's semi-implicit fixed-point step for the dual field p (Sec. 3),
 *   - the u-step        u = v - theta div p               (Sec. 2.1 / Sec. 3),
 *   - the v-step        v = min(max(u - theta lambda f, 0), 1),
 * and runs the three steps only on the restricted domain RD = {|f| < delta}
 * (Sec. 3, where delta is called q-hat); elsewhere u = v = H(-f), p = 0, with
 * u0 = H(-f) (Sec. 1) and H(0) = 0.  The discrete gradient is the forward
 * difference with a zero component on the last column / row; the divergence
 * is its negative adjoint (Chambolle 2004, cited at the end of Sec. 2.1).
 * Frozen neighbours enter the dual step through w = -H(-f)/theta.
 *
 * Conventions shared by every entry point
 *   - Images are row-major FP32 planes [H][ld], x contiguous, ld >= W elements.
 *     The dual field p is two planes [2][H][ld]: p (x component) then
 *     p + H*ld (y component).
 *   - Pointers marked "device" are HIP device pointers; "host" are host memory.
 *   - The caller allocates and owns every buffer, including the workspace
 *     `ws` (device) and the tape.  Nothing is allocated on the device by
 *     rdseg_active_set, rdseg_solve, rdseg_backward or the fit-term calls;
 *     rdseg_solve_batched allocates only inside its plan (see there).
 *   - All work is enqueued asynchronously on `stream` (a hipStream_t; NULL =
 *     the default stream).  Device-side counts are device scalars: synchronise
 *     the stream before reading them.
 *   - Every call validates its arguments on the host before enqueuing work and
 *     returns an rdseg_status; no C++ exception crosses the ABI.  On failure
 *     rdseg_last_error() returns a thread-local message.
 *   - Calls that overlap on one stream are ordered; calls on different streams
 *     that share a workspace race.
 */
#ifndef RDSEG_H
#define RDSEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RDSEG_OK = 0,
    RDSEG_ERR_ARG = 1,        /* invalid scalar or NULL / aliased pointer */
    RDSEG_ERR_SHAPE = 2,      /* H or W < 1, ld < W, or H*ld >= 2^31 */
    RDSEG_ERR_WORKSPACE = 3,  /* ws NULL or ws_bytes below the required size */
    RDSEG_ERR_HIP = 4,        /* a HIP runtime call or kernel launch failed */
    RDSEG_ERR_TAPE = 5,       /* tape missing or inconsistent with the parameters */
    RDSEG_ERR_TIMEOUT = 6     /* a bounded on-chip wait expired (see rdseg_solve_status) */
} rdseg_status;

typedef struct {
    int32_t H, W;   /* grid size, >= 1 */
    int64_t ld;     /* row pitch in elements, >= W */
} rdseg_shape;

/* Solver parameters.  lambda >= 0, theta > 0, tau > 0 finite; delta not NaN
 * (+INFINITY = full domain, the paper's q = 1; delta <= min|f| = pure
 * thresholding, q = 0).  iters >= 0 outer iterations, each `inner` dual steps
 * (Chambolle's fixed point for p with v held, Sec. 3), one u-step and one
 * v-step; inner = 0 or 1 means one dual step, at most 16 (between the dual
 * steps of one outer iteration w = div p - v/theta is refreshed with the same
 * v).  iters_per_launch, tile_w, tile_h: the temporally blocked kernel runs
 * iters_per_launch dual steps per launch (its halo depth, so
 * iters_per_launch / inner outer iterations; it must be >= inner) on
 * tile_w x tile_h blocks (multiples of 8); 0 = chosen by the library
 * (autotuned, see rdseg_autotune; choosing synchronises the stream once).
 * ckpt_every > 0 asks rdseg_solve to write a checkpoint of (v, p) every
 * ckpt_every iterations into `tape` for rdseg_backward (inner = 1 only).
 * components: whether a single-image solve (not under the stopping rule) runs
 * the RD components of at most 256 pixels whole in the component kernel (see
 * rdseg_set_components): 1 = on, 2 = off, 0 = the autotuner's choice for
 * this problem class when the library chooses the tiles, else on.
 * rdseg_backward uses the component path unless components is 2.  Results
 * are bitwise equal either way.
 * resident: the barrier between blocks of iterations of a single-image solve
 * without tape or stopping rule: 1 = on-chip exchange between the tiles of
 * one cooperative launch where the queued tiles all fit on the chip (see
 * rdseg_set_resident), else kernel boundaries; 2 = kernel boundaries
 * (separate launches); 0 = the autotuner's choice for this problem class when
 * the library chooses the tiles, else 1.  Results are bitwise equal either
 * way. */
typedef struct {
    double lambda, theta, tau, delta;
    int32_t iters;
    int32_t iters_per_launch;
    int32_t tile_w, tile_h;
    int32_t ckpt_every;
    int32_t inner;
    int32_t components;
    int32_t resident;
} rdseg_params;

/* Fitting term of Sec. 1: f = (z - c1)^2 - (z - c2)^2 + gamma P   (eq. CV when
 * P is NULL, eq. DS otherwise).  z, P: device planes with the solve's shape. */
typedef struct {
    const float* z;
    const float* P;   /* nullable */
    double c1, c2, gamma;
} rdseg_fit;

/* One image of a batch (all device pointers, layout as above). */
typedef struct {
    const float* f;
    float* u;
    float* v;
    float* p;         /* [2][H][ld] */
    rdseg_shape s;
    double lambda, delta;
} rdseg_image;

/* ---------------------------------------------------------------------- */
/* Sizes                                                                   */
/* ---------------------------------------------------------------------- */

/* Workspace bytes needed by rdseg_solve (prm may be NULL: the maximum over
 * all tile configurations) and by rdseg_active_set.  0 if the shape is invalid. */
size_t rdseg_workspace_size(const rdseg_shape* s, const rdseg_params* prm);

/* Tape bytes needed by rdseg_solve / rdseg_backward for prm->iters and
 * prm->ckpt_every: ceil(iters / ckpt_every) checkpoints of (v, px, py), each
 * 3 * H * ld floats.  0 if ckpt_every <= 0 or the arguments are invalid. */
size_t rdseg_tape_size(const rdseg_shape* s, const rdseg_params* prm);

/* Workspace bytes needed by rdseg_backward (includes a segment tape of
 * ckpt_every states and the adjoint state). */
size_t rdseg_backward_workspace_size(const rdseg_shape* s, const rdseg_params* prm);

/* ---------------------------------------------------------------------- */
/* Restricted domain (Sec. 3: Fg = {f <= -delta}, Bg = {f >= delta},       */
/* RD = the rest)                                                           */
/* ---------------------------------------------------------------------- */

/* Compacts RD = {x : |f(x)| < delta} (strict, compared in FP64; NaN is never
 * in RD) into 8x8 tiles.  Tile t = ty * ceil(W/8) + tx; its 64-bit mask has
 * bit (y mod 8) * 8 + (x mod 8) set for pixels of RD.
 * Outputs (device):
 *   tile_ids [ceil(H/8)*ceil(W/8)]  ascending ids of tiles with a non-empty mask
 *   tile_masks [same]               their masks
 *   slot_map [ceil(H/8)*ceil(W/8)]  position of tile t in tile_ids, or -1
 *   n_tiles (device int32)          number of listed tiles
 *   pixel_idx [H*W] (nullable)      ascending y*W + x of RD pixels
 *   n_pixels (device int64, nullable with pixel_idx)
 * Errors: RDSEG_ERR_ARG for NULL required pointers or NaN delta. */
rdseg_status rdseg_active_set(const float* f, rdseg_shape s, double delta,
                              int32_t* tile_ids, uint64_t* tile_masks, int32_t* slot_map,
                              int32_t* n_tiles, int32_t* pixel_idx, int64_t* n_pixels,
                              void* ws, size_t ws_bytes, void* stream);

/* Band threshold from a target fraction (Sec. 3: q-hat starts at 0 and grows
 * until the share of nodes in RD = {|f| < q-hat} reaches q).  Writes to
 * *delta_out (device double) the smallest double q-hat with
 * #{x : |f(x)| < q-hat} >= ceil(q * H * W), the ceiling taken exactly:
 * 0 for q = 0, otherwise the double just above the ceil(q H W)-th smallest |f|,
 * or +INFINITY when that value is +inf or NaN (fewer finite |f| than needed;
 * RD is then every finite node).  Ties can make the share exceed q.  The result
 * passed as prm->delta (or rdseg_image.delta) gives the restricted domain of
 * fraction q; it is exact (integer counting on the bit patterns of |f|), so it
 * equals a sort-based reference bit for bit.
 * q in [0, 1]; ws (device) of at least rdseg_band_workspace_size() bytes.
 * Errors: RDSEG_ERR_ARG for NULL f / delta_out or q outside [0, 1] or NaN. */
size_t rdseg_band_workspace_size(void);
rdseg_status rdseg_band_threshold(const float* f, rdseg_shape s, double q, double* delta_out,
                                  void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Solve (Sec. 2.1 iteration restricted as in Sec. 3)                      */
/* ---------------------------------------------------------------------- */

/* Runs prm->iters iterations from u0 (nullable: H(-f)) and p0 (nullable: 0;
 * [2][H][ld]); v0 = clamp(u0 - theta lambda f, 0, 1).  A start u0 / p0 is used
 * on RD only, and p0's x component on the last column and y component on the
 * last row are taken as 0.  Writes u, v, p (device, full grids; frozen pixels
 * hold u = v = H(-f), p = 0).  u0 == u and p0 == p are allowed (warm start in
 * place); u, v, p must not overlap f or each other.  iters == 0 returns the
 * initial state.  tape (device, nullable) receives the checkpoints when
 * prm->ckpt_every > 0 (size rdseg_tape_size; defined on RD pixels only).  A
 * solve with the component path on reads the tile-queue length once
 * (synchronises the stream, except under graph capture) to skip the tile path
 * when the components hold every RD pixel: always with a tape, and without
 * one unless the iterations run in the resident form (which ends at once on
 * an empty queue).  Results are bitwise identical
 * for every tile configuration and iters_per_launch, and a solve of K1
 * iterations resumed for K2 more (u0 = u, p0 = p) equals one of K1 + K2. */
rdseg_status rdseg_solve(const float* f, rdseg_shape s, const rdseg_params* prm,
                         const float* u0, const float* p0,
                         float* u, float* v, float* p, float* tape,
                         void* ws, size_t ws_bytes, void* stream);

/* Status of the last rdseg_solve / rdseg_solve_until that used the workspace
 * ws (device, the same shape s): synchronises `stream` (the stream that solve
 * was enqueued on) and reads the solve's status word, which every solve
 * clears when it starts.  RDSEG_ERR_TIMEOUT when the solve ran in the
 * resident form (see rdseg_set_resident) and a tile's bounded wait for a
 * neighbouring tile's frame expired: that tile, and every tile that would
 * have read its later frames, stopped and wrote NaN into u, v and p (the other
 * tiles hold their exact result); RDSEG_OK otherwise.  In normal operation the
 * waits do not expire, because a cooperative launch keeps every tile
 * resident; a preempted or time-sliced dispatch is the case this reports.
 * Errors: RDSEG_ERR_ARG / _SHAPE / _WORKSPACE for a NULL or invalid shape or
 * a workspace smaller than rdseg_workspace_size(s); RDSEG_ERR_HIP if the
 * read fails. */
rdseg_status rdseg_solve_status(const rdseg_shape* s, const void* ws, size_t ws_bytes,
                                void* stream);

/* Allocation-free rdseg_solve, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, outputs and results (bitwise) as
 * rdseg_solve without tape and workspace: prm->ckpt_every must be 0.  The
 * workspace is a file-scope device array of RDSEG_NOALLOC_SCRATCH_BYTES
 * (64 MiB) that each GPU holds from the library's load until the process
 * ends; its device address is looked up once per device, on the first call
 * with that device current.  The call allocates nothing (no hipMalloc /
 * hipFree, no stream or event creation, no pinned host memory, no timing
 * records) and runs every kernel on `stream`: the closed-tile and component
 * kernels run before the tiles instead of beside them on a side stream, and
 * the tiles use separate launches (not the resident form, so there is no
 * status word to read afterwards).  Letting the library choose the tile
 * configuration (tile_w = tile_h = iters_per_launch = 0) synchronises the
 * stream once, as in rdseg_solve.  Every call on one GPU shares that GPU's
 * array, which keeps the last call's contents (each call initialises what it
 * reads): calls that overlap on one GPU, on any streams, race.
 * Errors: as rdseg_solve; RDSEG_ERR_WORKSPACE when the image needs more than
 * RDSEG_NOALLOC_SCRATCH_BYTES of workspace (rdseg_workspace_size(s, NULL);
 * about 44 bytes a pixel: a 1024 x 1024 image needs 46.7 MB); RDSEG_ERR_ARG
 * when ckpt_every != 0; RDSEG_ERR_HIP when the array's address cannot be
 * obtained. */
#define RDSEG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
rdseg_status rdseg_solve_noalloc(const float* f, rdseg_shape s, const rdseg_params* prm,
                                 const float* u0, const float* p0, float* u, float* v, float* p,
                                 void* stream);

/* Convergence-driven solve with the stopping rule of Sec. 4: stop at the
 * first iteration l, among the multiples of check_every, where
 *     max( max|u^l - u^(l-1)|, max|v^l - v^(l-1)| ) <= tol
 * (the maximum norm over all nodes; frozen nodes never change), or after
 * prm->iters iterations.  Same arguments and outputs as rdseg_solve (no tape:
 * prm->ckpt_every must be 0), plus
 *   tol          stopping tolerance (the paper's delta: 1e-2 for its results,
 *                1e-10 for its ground truth); < 0 never stops; not NaN;
 *   check_every  >= 1 spacing of the checks;
 *   poll         0: every launch up to prm->iters is enqueued and the call
 *                never synchronises; launches after the stopping check exit
 *                at once (each still costs a launch).  1: the checks are read
 *                back to the host in chunks of doubling length (2, 4, ...,
 *                1024 checks), the next chunk running while the host looks at
 *                the last one, and enqueuing ends one chunk after the stop; the
 *                call waits for the checks it read and uses a small pinned host
 *                buffer that the library allocates once;
 *   iters_done   (device int32) iterations run, a multiple of check_every
 *                unless the solve ran to prm->iters;
 *   diffs        (device float[prm->iters / check_every], may be NULL only
 *                when that count is 0) the measured change at each check, in
 *                order; entries after the stopping check stay 0.
 * u, v, p hold iterate iters_done, bitwise equal to rdseg_solve with
 * prm->iters = iters_done (the change is measured in FP32).  The decision is
 * taken on the device: launches after the stopping check return at once, so
 * with poll = 0 the call never synchronises.  Tile configuration as in
 * rdseg_solve. */
rdseg_status rdseg_solve_until(const float* f, rdseg_shape s, const rdseg_params* prm,
                               double tol, int32_t check_every, int32_t poll,
                               const float* u0, const float* p0,
                               float* u, float* v, float* p,
                               int32_t* iters_done, float* diffs,
                               void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* The restriction on another solver (Sec. 5): primal-dual for eq. CR      */
/* ---------------------------------------------------------------------- */

/* Parameters of the primal-dual (Chambolle-Pock) iteration: lambda >= 0,
 * tau > 0, sigma > 0 finite (convergence needs tau * sigma <= 1/8), delta not
 * NaN as for rdseg_params; iters >= 0; tile_w, tile_h, iters_per_launch all 0
 * (chosen by the library) or a compiled configuration (8x8/16, 16x16/8,
 * 32x32/4, 64x64/8). */
typedef struct {
    double lambda, tau, sigma, delta;
    int32_t iters;
    int32_t iters_per_launch;
    int32_t tile_w, tile_h;
} rdseg_pd_params;

/* Workspace bytes for rdseg_solve_pd (0 if the shape is invalid). */
size_t rdseg_pd_workspace_size(const rdseg_shape* s);

/* Solves eq. CR itself, min over u in [0,1] of TV(u) + lambda <f, u>, with the
 * restriction of Sec. 3 carried over as Sec. 5 proposes: on RD = {|f| < delta}
 *     p    <- (p + sigma grad ubar) / max(1, |p + sigma grad ubar|)
 *     u'   =  clamp(u + tau div p - tau lambda f, 0, 1),  ubar = 2 u' - u
 * and u = ubar = H(-f), p = 0 elsewhere; start u0 (nullable: H(-f)),
 * ubar0 = u0, p0 (nullable: 0; [2][H][ld]).  Same operators, layout and
 * ownership as rdseg_solve; writes u and p (full grids). */
rdseg_status rdseg_solve_pd(const float* f, rdseg_shape s, const rdseg_pd_params* prm,
                            const float* u0, const float* p0, float* u, float* p,
                            void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Volumes (Sec. 5 names 3-D problems as the extension of interest)        */
/* ---------------------------------------------------------------------- */

/* A volume [D][H][W]: voxel (z, y, x) at z * lds + y * ld + x (elements);
 * ld >= W, lds >= H * ld, D * lds < 2^31. */
typedef struct {
    int32_t D, H, W;
    int64_t ld, lds;
} rdseg_shape3;

/* Workspace bytes for rdseg_solve3d (0 if the shape is invalid). */
size_t rdseg_workspace_size3(const rdseg_shape3* s);

/* The restricted iteration of rdseg_solve on a volume: forward-difference
 * gradient along x, y and z (zero component on the last plane of each axis),
 * divergence its negative adjoint, p a 3-vector with |g| its Euclidean norm;
 * RD = {|f| < delta}, frozen voxels u = v = H(-f), p = 0.  prm as for
 * rdseg_solve except that tile_w, tile_h, iters_per_launch and ckpt_every must
 * be 0 (one dual step per launch on 32 x 8 x 8 blocks; no tape).  Note that
 * Chambolle's step bound is tau <= 1/12 in three dimensions.
 * u0 (nullable), u, v: [D][lds] planes; p0 (nullable), p: [3][D][lds] (x, y, z
 * components).  u, v, p must not overlap f or each other.  A volume of
 * identical slices returns, slice by slice, the bits of rdseg_solve. */
rdseg_status rdseg_solve3d(const float* f, rdseg_shape3 s, const rdseg_params* prm,
                           const float* u0, const float* p0, float* u, float* v, float* p,
                           void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Evaluation measures (Sec. 4)                                             */
/* ---------------------------------------------------------------------- */

/* Measures of a result u against a reference u_ref (both device planes of
 * shape s): with the thresholded labels Omega = {u > eps} and
 * GT = {u_ref > eps} (values compared in FP64; the paper uses eps = 0.5),
 * writes to out (device double[3]) the node counts N(GT and Omega) and
 * N(GT or Omega) and E2 = sum over nodes of (u - u_ref)^2 (a unit cell per
 * node).  E1 = out[0] / out[1] (taken as 1 when both label sets are empty).
 * Counts are exact; E2 is an FP64 sum in a fixed order (the same bits on every
 * call with the same shape).  ws (device) of at least
 * rdseg_metrics_workspace_size() bytes.
 * Errors: RDSEG_ERR_ARG for NULL pointers or NaN eps. */
size_t rdseg_metrics_workspace_size(void);
rdseg_status rdseg_metrics(const float* u, const float* u_ref, rdseg_shape s, double eps,
                           double* out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Batched solve                                                            */
/* ---------------------------------------------------------------------- */

/* Solves n independent images (imgs: host array; per-image lambda and delta,
 * shared theta, tau, iters) over one global queue of (image, tile) work items,
 * each launch covering every image.  With graph_plan non-NULL, the first call
 * (*graph_plan == NULL) builds a plan (device descriptors, its own workspace,
 * a captured hipGraph of the whole sequence) and stores it in *graph_plan;
 * later calls with the same plan replay the graph (the image set, shapes,
 * pointers and scalars must then be unchanged; only the contents of f may
 * change).  The plan allocates its device memory once, at creation, and
 * frees it in rdseg_plan_destroy.  With graph_plan NULL, the call runs eagerly
 * using `ws` (size rdseg_batched_workspace_size; with tile_w = tile_h = 0 it is
 * the size for any configuration).  tile_w / tile_h / iters_per_launch all 0:
 * the library chooses the configuration and the form of the iterations (see
 * rdseg_set_batched_form) from the tuning cache's entry for the batch's class
 * (the size class of its total pixel count and the bucket of its active
 * fraction; entries written by rdseg_autotune_batched), else 16x16 tiles and
 * 8 iterations per launch below half active, 64x64 and 8 above, in the
 * process-wide form; choosing reads the batch's active-pixel count back
 * (synchronises the stream; a plan chooses once, when it is built).  Results
 * are bitwise identical to rdseg_solve on each image with the same tile
 * configuration, in either form. */
size_t rdseg_batched_workspace_size(const rdseg_image* imgs, int32_t n, int32_t tile_w,
                                    int32_t tile_h);
rdseg_status rdseg_solve_batched(const rdseg_image* imgs, int32_t n, double theta, double tau,
                                 int32_t iters, int32_t iters_per_launch, int32_t tile_w,
                                 int32_t tile_h, void** graph_plan, void* ws, size_t ws_bytes,
                                 void* stream);
rdseg_status rdseg_plan_destroy(void* plan);

/* Times the batched solve of these images (`probe_iters` iterations, captured
 * in a graph as a plan runs it; two rounds of three timed replays after a
 * warm-up per candidate) for every
 * compiled (tile_w, tile_h, iters_per_launch) configuration and both forms of
 * the iterations (1: one persistent launch, 2: one launch per block) and
 * returns the fastest.  A nonzero fix_tile_w, fix_tile_h,
 * fix_iters_per_launch or fix_form restricts the search to matching
 * candidates (RDSEG_ERR_ARG if no configuration matches); an unrestricted
 * search also stores the result in the tuning cache under the batch's class,
 * which rdseg_solve_batched reads when it chooses.  ws: at least
 * rdseg_batched_workspace_size(imgs, n, 0, 0) bytes; the images' u, v, p are
 * overwritten.  Synchronous. */
rdseg_status rdseg_autotune_batched(const rdseg_image* imgs, int32_t n, double theta, double tau,
                                    int32_t probe_iters, int32_t fix_tile_w, int32_t fix_tile_h,
                                    int32_t fix_iters_per_launch, int32_t fix_form, void* ws,
                                    size_t ws_bytes, void* stream, int32_t* tile_w,
                                    int32_t* tile_h, int32_t* iters_per_launch, int32_t* form);

/* The configuration and form rdseg_solve_batched chooses (all of tile_w,
 * tile_h, iters_per_launch 0) for these images when their active fraction is
 * q in [0, 1]: the tuning cache's entry (*cached = 1) or the fixed choice
 * (*cached = 0).  Host only.  Any output pointer may be NULL. */
rdseg_status rdseg_batched_lookup(const rdseg_image* imgs, int32_t n, double q, int32_t* tile_w,
                                  int32_t* tile_h, int32_t* iters_per_launch, int32_t* form,
                                  int32_t* cached);

/* ---------------------------------------------------------------------- */
/* Adjoint of the unrolled solve                                            */
/* ---------------------------------------------------------------------- */

/* Reverse-mode derivative of the solve that wrote `tape` (same f, shape and
 * prm, default start u0 = H(-f), p0 = 0; prm->ckpt_every > 0).  The domain RD
 * and u0 depend on f through comparisons only and are held fixed; the clamp
 * has derivative 1 strictly inside (0, 1); d|g|/dg = g/|g| (0 at g = 0).
 * Inputs: grad_u (device [H][ld]) = dL/du of the final u; grad_v (nullable).
 * Outputs: grad_f (device [H][ld], 0 off RD), grad_lambda (device double).
 * With fit non-NULL (the f of the solve came from rdseg_fit_forward with the
 * same fit), also grad_c1, grad_c2 and grad_gamma (device doubles) through
 * eq. CV / eq. DS.  Scalar reductions are FP64 in a fixed order
 * (deterministic).  With the component path on (prm->components != 2 and
 * rdseg_set_components), the RD components of at most 256 pixels run their
 * whole reverse sweep in one launch and the call synchronises the stream once
 * (to learn whether any tile is left to the per-step path); the results are
 * bitwise those of the per-step path.  RDSEG_ERR_TAPE if tape is NULL or
 * ckpt_every <= 0. */
rdseg_status rdseg_backward(const float* f, rdseg_shape s, const rdseg_params* prm,
                            const float* tape, const float* grad_u, const float* grad_v,
                            float* grad_f, double* grad_lambda, const rdseg_fit* fit,
                            double* grad_c1, double* grad_c2, double* grad_gamma,
                            void* ws, size_t ws_bytes, void* stream);

/* Fitting term of Sec. 1 (eq. CV / eq. DS), evaluated in FP64 and rounded to
 * FP32: f = (z - c1)^2 - (z - c2)^2 + gamma P.  f: device [H][ld]. */
rdseg_status rdseg_fit_forward(const rdseg_fit* fit, rdseg_shape s, float* f, void* stream);

/* dL/d(c1, c2, gamma) from grad_f = dL/df (device doubles out; FP64 fixed-order
 * reductions).  ws: at least rdseg_reduce_workspace_size(s) bytes. */
size_t rdseg_reduce_workspace_size(const rdseg_shape* s);
rdseg_status rdseg_fit_backward(const rdseg_fit* fit, rdseg_shape s, const float* grad_f,
                                double* grad_c1, double* grad_c2, double* grad_gamma,
                                void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Autotuning, timing, diagnostics                                          */
/* ---------------------------------------------------------------------- */

/* Times every compiled (tile_w, tile_h, iters_per_launch) configuration, with
 * the small-component path on and off and, where the configuration's queued
 * tiles can all fit on the chip, with both barrier kinds (on-chip exchange and
 * kernel boundaries), on this problem for `probe_iters` iterations
 * (synchronous) and returns the fastest (components: 1 on, 2 off; resident:
 * 1 on-chip exchange, 2 separate launches).  A nonzero prm->tile_w, tile_h,
 * iters_per_launch, components or resident fixes that parameter (only
 * matching candidates are timed; RDSEG_ERR_ARG if no configuration is
 * compiled); with all five zero the result is also stored in the
 * process-wide cache under (shape class, active-fraction bucket) that solves
 * with tile_w = tile_h = iters_per_launch = components = resident = 0 read.
 * u, v, p, ws as for rdseg_solve (their contents are overwritten); any output
 * pointer may be NULL. */
rdseg_status rdseg_autotune(const float* f, rdseg_shape s, const rdseg_params* prm,
                            int32_t probe_iters, float* u, float* v, float* p,
                            void* ws, size_t ws_bytes, void* stream,
                            int32_t* tile_w, int32_t* tile_h, int32_t* iters_per_launch,
                            int32_t* components, int32_t* resident);

/* Single-image solves without checkpoints or stopping rule whose queued
 * macro tiles all fit on the chip at once (one workgroup each; e.g. a 1024^2
 * image in 64x64 tiles) run as one cooperative launch in which every tile
 * stays on chip and exchanges only its halo frame with its neighbours after
 * each block of iterations (results bitwise equal to separate launches).
 * on = 0 forces separate launches, on != 0 (the default) allows the resident
 * form.  Process-wide. */
rdseg_status rdseg_set_resident(int32_t on);

/* Bound of each wait of the resident form in ticks of the GPU's 100 MHz
 * wall clock: ticks > 0 sets it, 0 restores the default (10^8, one second),
 * ticks < 0 makes every wait that is not already satisfied give up at once
 * (the expiry path forced from the host, for tests of rdseg_solve_status and
 * of the persistent batched form).  Process-wide; read when a resident solve
 * or a persistent batched launch is enqueued. */
rdseg_status rdseg_set_resident_wait(int64_t ticks);

/* The form of the iterations of rdseg_solve_batched when the caller fixes the
 * configuration (or the tuning cache holds none for the batch): form 1 runs
 * every block of iterations_per_launch iterations over the global (image,
 * macro tile) queue in one persistent cooperative launch, with a grid-wide
 * barrier between blocks (an empty queue ends it at once); form 2 (the
 * default) enqueues one launch per block.  Results are bitwise equal either
 * way.  Form 1's barrier waits are bounded like the resident form's
 * (rdseg_set_resident_wait); a workgroup whose wait expires writes NaN into
 * u, v and p of its macro tiles, so an incomplete batch never reads as a
 * solution.  A plan keeps the form it was built with.  Process-wide.
 * RDSEG_ERR_ARG for any other value. */
rdseg_status rdseg_set_batched_form(int32_t form);

/* In single-image solves without the stopping rule, the RD pixels whose
 * 4-connected RD component has at most 256 pixels run every iteration in one
 * launch, one pixel per lane (an RD pixel interacts only with its own
 * component, Sec. 3; up to 64 pixels in one wave, larger ones in a
 * workgroup); the tile path covers the larger components.  In a resident
 * solve the resident kernel's workgroups that hold no tile run the one-wave
 * ones;
 * with a tape they also write their checkpoints; rdseg_backward runs their
 * whole reverse sweep in one launch.  Skipped on the device when more than
 * 55 % of the pixels are RD.  Results are bitwise equal either way.  on = 0
 * forces the tile path for every pixel, on != 0 (the default) allows the
 * component path.  Process-wide. */
rdseg_status rdseg_set_components(int32_t on);

/* The reverse sweep of rdseg_backward's tile path (the RD pixels outside
 * the component path) runs `steps` reverse iterations per launch on tile x
 * tile macro tiles with a halo of 3 * steps pixels (the adjoint state stays
 * on chip between the steps; each step reads its stored forward state).
 * Forms: (32, 1), (16, 2), (16, 4), (32, 2), (32, 4); 0 selects the default
 * (32 and 2).  Results are bitwise equal across forms.  RDSEG_ERR_ARG for a
 * form that has no kernel.  Process-wide. */
rdseg_status rdseg_set_adjoint_form(int32_t tile, int32_t steps);

/* The autotuner's cache (the choices of rdseg_autotune, keyed by size class
 * and active-fraction bucket, read by solves that let the library choose) as
 * JSON text, so that a tuning run can be kept and reloaded in a later process:
 *   {"version": 1, "entries": [{"size_class": c, "q_bucket": b, "tile_w": w,
 *    "tile_h": h, "iters_per_launch": i, "components": m, "resident": r},
 *    ...]}
 * size_class c: the number of times H * W can be divided by 4 while it stays
 * above 4096 (at most 12); q_bucket b: 0 for an active fraction q < 0.01,
 * 1 for q < 0.05, 2 for q < 0.2, 3 for q < 0.5, 4 above; components m: 1 on,
 * 2 off; resident r: 1 on-chip exchange, 2 separate launches.  Host memory
 * only; no GPU call.
 * rdseg_tune_cache_export writes the text and its NUL into buf (host, cap
 * bytes; buf may be NULL when cap is 0) and the bytes needed, NUL included,
 * into *len; RDSEG_ERR_ARG (buf untouched) if cap is smaller than that.
 * rdseg_tune_cache_import merges the entries of such a text (host,
 * NUL-terminated) into the cache, replacing entries with the same key; a text
 * that does not parse, a key out of range or a configuration that is not
 * compiled is RDSEG_ERR_ARG and nothing is merged.
 * rdseg_tune_cache_clear empties the cache. */
rdseg_status rdseg_tune_cache_export(char* buf, size_t cap, size_t* len);
/* The configuration that a solve leaving the choice to the library uses for
 * an image of shape s whose RD holds the fraction q in [0, 1] of its pixels:
 * the cache entry of (size class, q bucket) when there is one (*cached = 1),
 * else the fixed choice by band width (*cached = 0; components and resident
 * then 0, i.e. the library's defaults).  Host only: reads the cache and, for
 * the fixed choice, whether the resident form's tiles fit on the current
 * device.  Any output pointer may be NULL.  RDSEG_ERR_ARG for q outside
 * [0, 1] or NaN. */
rdseg_status rdseg_tune_lookup(const rdseg_shape* s, double q, int32_t* tile_w, int32_t* tile_h,
                               int32_t* iters_per_launch, int32_t* components,
                               int32_t* resident, int32_t* cached);
rdseg_status rdseg_tune_cache_import(const char* json);
rdseg_status rdseg_tune_cache_clear(void);

/* Number of compiled configurations and their parameters (i < count). */
int32_t rdseg_config_count(void);
rdseg_status rdseg_config_get(int32_t i, int32_t* tile_w, int32_t* tile_h,
                              int32_t* iters_per_launch, int32_t* threads);

/* When enabled, every run of back-to-back launches of the iteration kernel
 * (a whole solve, or one checkpoint segment) is bracketed by a pair of HIP
 * events on its stream.  rdseg_timing_read synchronises on the recorded events
 * of configuration `config` (an index of rdseg_config_get; -1 = all) and
 * returns their summed kernel milliseconds, the launch count, the summed
 * algorithmic bytes (28 bytes per active pixel-iteration: read f, v, p_x, p_y,
 * write v, p_x, p_y) and pixel-updates.  Records accumulate until
 * rdseg_timing_reset.  Not recorded inside batched graph plans. */
rdseg_status rdseg_timing_enable(int32_t on);
rdseg_status rdseg_timing_read(int32_t config, double* kernel_ms, int64_t* launches,
                               double* alg_bytes, int64_t* pixel_updates);
/* As rdseg_timing_read, restricted to one form of launch: form 0 = separate
 * launches of the blocked kernel, 1 = resident launches (one per solve), -1 =
 * both.  RDSEG_ERR_ARG for any other form. */
rdseg_status rdseg_timing_read_form(int32_t config, int32_t form, double* kernel_ms,
                                    int64_t* launches, double* alg_bytes,
                                    int64_t* pixel_updates);
rdseg_status rdseg_timing_reset(void);

/* Releases what the library keeps for the process on the host and in the
 * HIP runtime: the per-device side streams (after their work completes), the
 * timing events and the pinned host buffers of timing, polling and the small
 * read-backs a solve waits for (queue lengths, class counts).  Device
 * memory of batched plans is not touched (rdseg_plan_destroy).  Call it
 * before the HIP runtime shuts down (the Python binding does at interpreter
 * exit); the library creates them again on later use.  Not concurrent with
 * other calls of the library. */
rdseg_status rdseg_release(void);

const char* rdseg_status_string(rdseg_status st);
const char* rdseg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RDSEG_H */
