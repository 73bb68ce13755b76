/*
 * g4d.h -- C ABI of the MI355X (gfx950) 4D Gaussian renderer.
 *
 * The operation is the rendering routine of "Real-time Photorealistic Dynamic
 * Scene Representation and Rendering with 4D Gaussian Splatting" (Yang et al.,
 * ICLR 2024), Sec. 3.2: a pixel (u, v) of view I at time t is
 *
 *     I(u,v,t) = sum_i p_i(t) p_i(u,v|t) alpha_i c_i(d,t)
 *                      prod_{j<i} (1 - p_j(t) p_j(u,v|t) alpha_j)      (Eq. 6)
 *
 * where each primitive is a 4D Gaussian with covariance R S S^T R^T,
 * R = L(q_l) R(q_r) (Sec. 3.2, "Representation of 4D Gaussian"), sliced at t
 * into a conditional 3D Gaussian weighted by its temporal marginal p_i(t),
 * projected by EWA splatting (Eqs. 3-4) and coloured by 4D spherindrical
 * harmonics (Sec. 3.2, "4D spherindrical harmonics"). render_backward returns
 * the gradient of a scalar loss with respect to every primitive parameter,
 * given dL/d(image).
 *
 * Conventions where the paper is silent (shared as specification, not code,
 * with the test oracle): unnormalised p(t) with the Sec. 4.2 filter p(t) >= t_cull;
 * near plane; 0.3 px^2 EWA low-pass; Jacobian evaluated at x/z clamped to 1.3x
 * the half field of view; footprint radius ceil(3 sqrt(lambda_max)) px; 16x16
 * tiles, a primitive covers the tiles overlapping [u-r, u+r] x [v-r, v+r];
 * front-to-back order by camera-space z, ties by primitive index; fragments with
 * alpha < 1/255 are skipped; alpha is clamped to 0.99; blending stops before a
 * fragment that would bring the transmittance below 1e-4; pixel centres at +0.5;
 * colour = max(0, 0.5 + 4DSH sum); real SH orthonormal with the Condon-Shortley
 * phase, index l*l + l + m; Fourier terms cos(2 pi n (t - mu_t) / T), n = 0..t_order.
 *
 * Memory: every tensor pointer is a DEVICE pointer to contiguous float32 data
 * with 16-byte alignment unless noted. All work is enqueued on the context's
 * HIP stream. The caller owns every tensor; the context owns only its scratch.
 *
 * Errors: every entry point returns a g4d_status. Argument validation happens
 * before any HIP call. G4D_EHIP is sticky for the context (destroy it).
 * On error the outputs are undefined. g4d_last_error() gives a message.
 *
 * Threading: a context is not thread-safe; use one context per host thread.
 */
#ifndef G4D_H
#define G4D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t g4d_status;
enum {
  G4D_OK = 0,
  G4D_EINVAL = -1,     /* bad argument */
  G4D_ENOMEM = -2,     /* device allocation failed */
  G4D_EHIP = -3,       /* a HIP call failed (sticky) */
  G4D_ESTATE = -4,     /* call out of order, e.g. backward without a render */
  G4D_ECAPACITY = -5   /* a size exceeds a fixed limit of the library */
};

typedef struct g4d_ctx g4d_ctx;

/* Rendering options, fixed for the life of a context. */
typedef struct {
  int32_t sh_degree;   /* spatial SH degree L, 0..3 */
  int32_t t_order;     /* Fourier order N_t, 0..2 (terms n = 0..N_t) */
  float t_period;      /* Fourier period T (> 0); 1 = normalised duration */
  float t_cull;        /* temporal filter: keep iff exp(-(t-mu_t)^2/(2 Sigma_44)) >= t_cull (Sec. 4.2: 0.05) */
  float near_plane;    /* keep iff camera-space z > near_plane (0.2) */
  float bg[3];         /* background colour composited with the final transmittance */
} g4d_options;

/* Pinhole camera, OpenCV axes (x right, y down, z forward). Host struct. */
typedef struct {
  int32_t width, height;     /* pixels, 1..16384 */
  float fx, fy, cx, cy;      /* intrinsics K (Eq. 3), pixels */
  float world_to_cam[12];    /* extrinsic E, row-major 3x4 [R | t]: x_cam = R x_world + t */
  float center[3];           /* camera position in world frame (for the view direction d) */
} g4d_camera;

/* Counters of the last render. */
typedef struct {
  int64_t n_views;
  int64_t active_total;   /* (view, primitive) pairs that passed every cull */
  int64_t instances;      /* (tile, primitive) pairs sorted for rasterisation */
  int64_t tiles;          /* 16x16 tiles over all views */
  int64_t max_tile_list;  /* longest per-tile list */
  int64_t fragments;      /* list entries visited per pixel up to its last contributor, summed */
  int64_t rounds;         /* view groups the render was binned and rasterised in */
  int64_t culled_nonfinite; /* (view, primitive) pairs left out because a parameter is not finite:
                             * every view of a primitive with a NaN or infinite mean, log scale,
                             * quaternion component or opacity logit; the views in which a
                             * primitive with a non-finite 4DSH coefficient passes every other
                             * cull (it is rendered fully transparent). Such primitives receive
                             * zero gradients. */
} g4d_stats;

/* Fills the defaults: L=3, N_t=2, T=1, t_cull=0.05, near=0.2, black background. */
void g4d_default_options(g4d_options* out);

/* Creates a context bound to `hip_stream` (a hipStream_t; NULL = default stream)
 * on the current HIP device. */
g4d_status g4d_create(const g4d_options* opts, void* hip_stream, g4d_ctx** out);
g4d_status g4d_destroy(g4d_ctx* ctx);
/* Rebinds the context to another stream (e.g. torch's current stream). */
g4d_status g4d_set_stream(g4d_ctx* ctx, void* hip_stream);

/* Borrows the primitive parameters (Sec. 3.2). The pointers must stay valid
 * and unchanged until the render_backward of every render that used them
 * has returned. n may be 0.
 *   means4        [n][4]  (mu_x, mu_y, mu_z, mu_t)
 *   log_scales4   [n][4]  s = exp(log_scales4), S = diag(s)
 *   q_left        [n][4]  (a, b, c, d), normalised inside
 *   q_right       [n][4]  (p, q, r, s), normalised inside
 *   opacity_logit [n]     alpha = sigmoid(logit)   (4-byte alignment suffices)
 *   coeffs        [n][K][3], K = (t_order+1)(sh_degree+1)^2, k = n_f*(L+1)^2 + l*l+l+m
 *                 (4-byte alignment suffices)
 * Invalidates the state kept for render_backward. */
g4d_status g4d_set_primitives(g4d_ctx* ctx, int64_t n, const float* means4, const float* log_scales4,
                              const float* q_left, const float* q_right, const float* opacity_logit,
                              const float* coeffs);

/* Renders n_views (camera, time) pairs in one batch.
 *   cams   host array [n_views]
 *   times  host array [n_views]
 *   out_rgb    device [sum_v 3*H_v*W_v], per view planar [3][H][W], views concatenated
 *   out_depth  device [sum_v H_v*W_v] or NULL: sum_i a_i T_i z_i (not normalised)
 *   out_alpha  device [sum_v H_v*W_v] or NULL: 1 - final transmittance
 * Keeps per-pixel final transmittance and last-contributor count for backward.
 * Views are processed in rounds of consecutive views: a round holds at most
 * G4D_TUNE_ROUND_PAIRS (view, primitive) pairs (but at least one view), at
 * most G4D_TUNE_ROUND_INSTANCES tile instances and at most 2^16 16x16 tiles
 * (unless one view alone has more); the first round takes at most
 * 16 views, later ones are sized from the instances per view seen so far, and
 * a round over the instance cap is shrunk and binned again. Each view's
 * result does not depend on the grouping. Synchronises the stream once per binning attempt, to size the
 * tile-instance arena (see G4D_TUNE_SYNC_FREE for the mode that does not).
 * G4D_ECAPACITY if one view alone exceeds the cap. Views reach the device as
 * kernel arguments: cams and times may be reused as soon as this returns. */
g4d_status g4d_render(g4d_ctx* ctx, int32_t n_views, const g4d_camera* cams, const float* times,
                      float* out_rgb, float* out_depth, float* out_alpha);

/* g4d_render for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc. Same
 * arguments, outputs and kernels as g4d_render (images are identical), but it
 * calls no hipMalloc, hipFree or other allocating routine: every scratch
 * buffer of the render lives in one fixed array per GPU (about 164 MiB,
 * allocated with the library's code when it is loaded on that GPU and held
 * until the process ends). Limits: at most 2^19 primitives (one view's
 * (view, primitive) pairs per round), 2^22 tile instances per round, 2^21
 * pixels per call (e.g. one 1920x1080 view) and 2^16 16x16 tiles per view;
 * beyond them the call returns G4D_ECAPACITY before enqueuing anything (the
 * instance limit: when one view alone needs more). It keeps no state for
 * render_backward (and invalidates a previous render's), and g4d_get_stats
 * does not describe it. Every call on one GPU, from any context, shares that
 * GPU's array: calls whose work overlaps on one GPU (other streams, other
 * threads) race; serialise them. Stage timing is off during the call. */
g4d_status g4d_render_noalloc(g4d_ctx* ctx, int32_t n_views, const g4d_camera* cams, const float* times,
                              float* out_rgb, float* out_depth, float* out_alpha);

/* Rendered optical flow (Sec. 4.4, "Ablation and analysis"): for each view, the alpha blend of Eq. (6)
 * (the render's weights, zero background) of every primitive's image-plane
 * displacement between t and t + frame_dt of its conditional mean
 * mu_xyz|t: f_i = pi(mu_c(t + frame_dt)) - pi(mu_c(t)) with pi the view's
 * pinhole projection, or 0 when mu_c(t + frame_dt) is not in front of the near
 * plane. Primitives, footprints and order are exactly those of g4d_render.
 *   out_flow  device [sum_v 2*H_v*W_v], per view planar [2][H][W] (du, dv, px)
 * There is no gradient of the flow: the call invalidates the state kept for
 * render_backward. */
g4d_status g4d_render_flow(g4d_ctx* ctx, int32_t n_views, const g4d_camera* cams, const float* times,
                           float frame_dt, float* out_flow);

/* Gradient of the last render. dL_drgb is required; dL_ddepth and dL_dalpha may
 * be NULL (treated as zero). Layouts match render's outputs. The gradient
 * buffers (layouts as set_primitives) receive the sum over the views of the
 * last render: overwritten (primitives active in no view get zeros), or added
 * to their contents when flags has G4D_GRAD_ACCUMULATE. When the render took
 * more than one round, every round except the last is binned again (the
 * same bins as in the render) before its backward passes.
 * Returns G4D_ESTATE if no render happened since the last set_primitives. */
enum { G4D_GRAD_ACCUMULATE = 1 };
g4d_status g4d_render_backward(g4d_ctx* ctx, const float* dL_drgb, const float* dL_ddepth,
                               const float* dL_dalpha, float* g_means4, float* g_log_scales4,
                               float* g_q_left, float* g_q_right, float* g_opacity_logit, float* g_coeffs,
                               int32_t flags);

/* The image loss and the gradient of the last render in one call: the same
 * as g4d_image_loss(kind, 3 * (render's pixels), img, target, scale,
 * loss_out, grad) followed by g4d_render_backward(grad, dL_ddepth, dL_dalpha,
 * ...), without the gradient image: the backward rasteriser reads img (the
 * render's rgb output, same layout) and target per pixel and forms dL/drgb
 * itself, identically. The loss is summed per tile, then per round in a fixed
 * order, and ADDED to the device float loss_out (clear it first); it can
 * differ from g4d_image_loss's in the last bits (another summation order).
 * Gradients, flags and errors as g4d_render_backward; kind, scale as
 * g4d_image_loss. */
g4d_status g4d_render_backward_loss(g4d_ctx* ctx, int32_t kind, const float* img, const float* target,
                                    float scale, float* loss_out, const float* dL_ddepth, const float* dL_dalpha,
                                    float* g_means4, float* g_log_scales4, float* g_q_left, float* g_q_right,
                                    float* g_opacity_logit, float* g_coeffs, int32_t flags);

/* Densification statistics (Sec. 3.3, "Densification in spacetime"): every
 * later render_backward adds, for each primitive and each view of the render
 * in which it blended at least one pixel (a fragment with alpha >= 1/255
 * before the stop):
 *   uv_grad_norm_sum[i] += |(dL/du_i, dL/dv_i)|   (that view's share, pixels)
 *   t_grad_abs_sum[i]   += |dL/dmu_t,i|           (that view's share)
 *   blend_count[i]      += 1
 * so that sum / count are the average gradient magnitudes the paper uses as
 * density-control indicators. Device arrays [n] of the current primitives,
 * borrowed, never cleared by the library (zero them to start an interval).
 * All three NULL switches the statistics off; set_primitives also does. */
g4d_status g4d_set_densify_stats(g4d_ctx* ctx, float* uv_grad_norm_sum, float* t_grad_abs_sum,
                                 int32_t* blend_count);

/* One Adam step over the six parameter groups, in one launch (Sec. 4.2: the
 * optimiser settings of 3D Gaussian Splatting, i.e. Adam with a learning rate
 * per group):
 *   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 *   p -= lr_g (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 *   params      host [6] of device pointers, updated in place: means4,
 *               log_scales4, q_left, q_right, opacity_logit, coeffs of n
 *               primitives (layouts of set_primitives; K from the options)
 *   grads       host [6] of device pointers, same layouts (render_backward's)
 *   exp_avg, exp_avg_sq  device [n (17 + 3K)] each: the groups' moments one
 *               group after the other in that order; zero them before step 1
 *   step        1, 2, ... (bias correction) */
typedef struct {
  float lr[6];
  float beta1, beta2, eps;
} g4d_adam_options;
g4d_status g4d_adam_step(g4d_ctx* ctx, int64_t n, const g4d_adam_options* opts, int64_t step,
                         float* const* params, const float* const* grads, float* exp_avg, float* exp_avg_sq);

/* New 4D positions for splitting primitives (Sec. 3.3 "Densification in
 * spacetime", Sec. 4.4: samples of the primitive's complete 4D Gaussian):
 *   out_means4[k] = mu_i + R_i S_i z[k],  i = idx[k]
 * over the primitives of set_primitives (R = L(q_l) R(q_r), S = exp(log
 * scales)); z [count][4] are the caller's standard-normal draws. Device
 * arrays: idx [count] int32, z and out_means4 [count][4] (16-byte aligned).
 * An idx outside [0, n) reads nothing and gives a NaN row. */
g4d_status g4d_split_sample(g4d_ctx* ctx, int64_t count, const int32_t* idx, const float* z, float* out_means4);

/* Image loss and its gradient dL/dI (Sec. 3.3: optimisation is supervised by
 * a rendering loss only), on the context's stream: over n values,
 *   G4D_LOSS_L1: loss += scale * sum |img - target|,  grad = scale * sign(img - target)
 *   G4D_LOSS_L2: loss += scale * sum (img - target)^2, grad = 2 scale (img - target)
 * loss_out is one device float that is ADDED to (clear it first); grad_out
 * (device, n values) is overwritten and may alias neither input. */
enum { G4D_LOSS_L1 = 1, G4D_LOSS_L2 = 2 };
g4d_status g4d_image_loss(g4d_ctx* ctx, int32_t kind, int64_t n, const float* img, const float* target,
                          float scale, float* loss_out, float* grad_out);

/* Counters of the last render, summed over its rounds; active_per_view
 * (host [n_views]) may be NULL. Synchronises the stream. Returns
 * G4D_ECAPACITY (after filling `out`) when a sync-free render since the last
 * call overflowed the instance arena. */
g4d_status g4d_get_stats(g4d_ctx* ctx, g4d_stats* out, int64_t* active_per_view);

/* Tuning knobs (key, value); unknown keys give G4D_EINVAL.
 *   G4D_TUNE_SORT_BLOCKS   max workgroups of each radix-sort pass (>= 1;
 *                          default 1280; a round of more than 2^26 tile
 *                          instances takes at most 768 for its tile sort)
 *   G4D_TUNE_STAGE_TIMING  1: bracket every stage with HIP events on the
 *                          context's stream (resets the totals); 0: off
 *   G4D_TUNE_ROUND_PAIRS     max (view, primitive) pairs per round (>= 1;
 *                            default 2^28, about 37 GB of per-pair scratch)
 *   G4D_TUNE_ROUND_INSTANCES max tile instances per round (>= 1; default
 *                            2^30, 16 GB of key/value arena)
 *   G4D_TUNE_SYNC_FREE     1: render and render_backward read no device
 *                          count on the host and never synchronise, so a
 *                          caller may capture them (with image_loss) into a
 *                          HIP graph. Rounds are planned from the views
 *                          alone (G4D_TUNE_ROUND_PAIRS pairs and 2^16 tiles
 *                          at most; the instance cap does not apply) and the
 *                          tile-instance arena keeps the capacity that
 *                          earlier synchronous renders or
 *                          G4D_TUNE_ARENA_INSTANCES gave it. A round that
 *                          needs more raises a sticky device flag and
 *                          outputs background only; get_stats reports it as
 *                          G4D_ECAPACITY and clears it.
 *                          Scratch that must grow grows (synchronising) when
 *                          the stream is not capturing; during capture that
 *                          is G4D_ECAPACITY, so make one uncaptured call of
 *                          the same shape first. 0 (default): off.
 *   G4D_TUNE_ARENA_INSTANCES  grow the tile-instance arena now to hold at
 *                          least this many instances (>= 0)
 *   G4D_TUNE_TILE_ORDER    1 (default): the rasterisers take tiles in order
 *                          of decreasing list length; 0: in tile-id order.
 *                          Results are identical; changing it invalidates
 *                          the state kept for render_backward.
 *   G4D_TUNE_ELLIPSE_CULL  1 (default): a record is binned only into the
 *                          tiles of its rectangle that its 1/255-alpha
 *                          ellipse reaches, and each 8x8-pixel quarter of a
 *                          tile walks only the entries whose ellipse meets
 *                          it; 0: whole rectangles, every entry walked
 *                          (slower, same images; for checking that the
 *                          ellipse tests are conservative). Changing it
 *                          invalidates the state kept for render_backward.
 *   G4D_TUNE_PERSISTENT_BLOCKS  0 (default): one rasteriser workgroup per
 *                          tile, dispatched in the tile order; -1: as many
 *                          workgroups as stay resident on the device, each
 *                          taking the next tile (in the tile order) from a
 *                          device counter until none is left; N > 0: N such
 *                          workgroups. Results are identical.
 *   G4D_TUNE_LDS_BATCH     list entries the forward rasteriser stages in
 *                          LDS at a time: 64, 128 or 256 (default). Results
 *                          are identical.
 *   G4D_TUNE_AUTOTUNE      1: the next render that is not being captured
 *                          first times its batch (once, then twice with HIP
 *                          events per candidate) under, in turn,
 *                          G4D_TUNE_SORT_BLOCKS in {512, 1024, 1280, 2048},
 *                          G4D_TUNE_TILE_ORDER x G4D_TUNE_PERSISTENT_BLOCKS
 *                          in {0, 1} x {0, -1}, and G4D_TUNE_LDS_BATCH in
 *                          {64, 128, 256}, keeping the fastest of each group
 *                          before the next, then renders normally. One-shot.
 *
 * The rasteriser knobs of a (lds_batch, split_threshold, persistent_blocks)
 * tuning call map to these keys: lds_batch -> G4D_TUNE_LDS_BATCH (the
 * forward's batch; the backward stages 12 entries at a time, fixed by its
 * LDS budget of five workgroups per CU and its 12-primitive x 16-column
 * second phase); persistent_blocks -> G4D_TUNE_PERSISTENT_BLOCKS;
 * split_threshold has no key: heavy tiles are not split. A wave owns an 8x8
 * quarter of its tile, so a split would not shorten its longest walk, and
 * with the tiles taken heaviest first the launch does not end on one heavy
 * tile (the heaviest carries at most an eighth of a resident workgroup's
 * share of the work on the workloads measured).                          */
enum {
  G4D_TUNE_SORT_BLOCKS = 1, G4D_TUNE_STAGE_TIMING = 2, G4D_TUNE_ROUND_PAIRS = 3, G4D_TUNE_ROUND_INSTANCES = 4,
  G4D_TUNE_SYNC_FREE = 5, G4D_TUNE_ARENA_INSTANCES = 6, G4D_TUNE_TILE_ORDER = 7, G4D_TUNE_AUTOTUNE = 8,
  G4D_TUNE_ELLIPSE_CULL = 9, G4D_TUNE_PERSISTENT_BLOCKS = 10, G4D_TUNE_LDS_BATCH = 11
};
g4d_status g4d_set_tuning(g4d_ctx* ctx, int32_t key, int32_t value);
/* Current value of a tuning key (G4D_TUNE_ARENA_INSTANCES: the arena's
 * capacity; counts above 2^31 - 1 read as 2^31 - 1). */
g4d_status g4d_get_tuning(g4d_ctx* ctx, int32_t key, int32_t* value);

/* Per-stage GPU time accumulated since stage timing was switched on
 * (synchronises the stream). ms_out and launches_out: host [G4D_NUM_STAGES]. */
enum {
  G4D_STAGE_PREPROCESS = 0,   /* slice, project, cull (geometry) */
  G4D_STAGE_BINNING = 1,      /* compaction, depth sort, emission, tile sort, ranges; the
                               * 4DSH colour of the active records runs on a second stream
                               * alongside, and the forward rasteriser waits for it */
  G4D_STAGE_RASTER_FWD = 2,   /* the forward rasteriser alone */
  G4D_STAGE_RASTER_BWD = 3,   /* the backward rasteriser alone */
  G4D_STAGE_PREPROCESS_BWD = 4, /* zeroing the gradient lines, then the per-record and
                                 * per-primitive backward (two timed windows per round) */
  G4D_STAGE_LOSS = 5,          /* g4d_image_loss; in g4d_render_backward_loss the per-tile
                                 * loss sums (the per-pixel terms run in the backward rasteriser) */
  G4D_STAGE_COLOUR = 6,       /* the 4DSH colour pass, timed on its own (second) stream */
  G4D_NUM_STAGES = 7
};
g4d_status g4d_stage_times(g4d_ctx* ctx, double* ms_out, int64_t* launches_out);

/* Message of the last error on this context (owned by the context). */
const char* g4d_last_error(const g4d_ctx* ctx);

/* Copies an intermediate of the last render to host memory, for inspection
 * by tests. Synchronises the stream. `bytes` must equal the size reported by
 * g4d_debug_size for the same `what`. Per-pair, per-instance and per-tile
 * items belong to the round binned last (tile ids and view indices relative
 * to it); per-pixel items cover all views.
 *   G4D_DBG_RECORDS   per active pair in depth order, 12 x float32:
 *                     u, v, z, opacity*p(t), conic00, conic01, conic11, rect x (x0 | x1<<16 as bits),
 *                     r, g, b, rect y (y0 | y1<<16 as bits)
 *   G4D_DBG_IDS       per active pair in depth order, uint32 view*n + primitive
 *   G4D_DBG_TILE_KEYS sorted instances, uint32 global tile id, as delimited by
 *                     the ranges (the sort's last pass writes ranges, not
 *                     keys; a position no range covers reads 0xFFFFFFFF)
 *   G4D_DBG_TILE_VALS sorted instances, uint32 depth-order record index
 *   G4D_DBG_RANGES    per global tile, uint32 [start, end)
 *   G4D_DBG_PIX_T     per pixel (views concatenated), float32 final transmittance
 *   G4D_DBG_PIX_LAST  per pixel, uint32 list entries up to the last contributor
 *   G4D_DBG_GRAD2D    after a backward: per active pair, 16 x float64
 *                     dL/du, dL/dv, dL/dconic00, 01, 11, dL/d(opacity*p), dL/dr, g, b, dL/dz, 0 x 5,
 *                     blended flag (1 when densification statistics are on and the pair blended)
 *   G4D_DBG_TILE_ORDER per global tile, uint32 tile id in the order the
 *                     rasterisers' workgroups take them (heavy-first: by
 *                     decreasing list-length bin); G4D_ESTATE when that order
 *                     is off (G4D_TUNE_TILE_ORDER = 0) */
enum {
  G4D_DBG_RECORDS = 1, G4D_DBG_IDS = 2, G4D_DBG_TILE_KEYS = 3, G4D_DBG_TILE_VALS = 4,
  G4D_DBG_RANGES = 5, G4D_DBG_PIX_T = 6, G4D_DBG_PIX_LAST = 7, G4D_DBG_GRAD2D = 8, G4D_DBG_TILE_ORDER = 9
};
g4d_status g4d_debug_size(g4d_ctx* ctx, int32_t what, int64_t* bytes);
g4d_status g4d_debug_copy(g4d_ctx* ctx, int32_t what, void* host_dst, int64_t bytes);

#ifdef __cplusplus
}
#endif

#endif /* G4D_H */
