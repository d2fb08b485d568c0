/*
 * gsr.h — C ABI of libgsr.so, a differentiable tile-based rasterizer of 3D
 * Gaussians into colour, depth and alpha for AMD Instinct MI355X (gfx950).
 *
 * It implements the rendering hot path of Gaussian-SLAM (Yugay et al., arXiv
 * 2312.10070): projection of Gaussians (Sec. 3.1, Eq. 1) with the EWA 2D
 * covariance (Eq. 2), front-to-back alpha compositing of colour (Eq. 3, 4)
 * and depth (Eq. 6), their explicit gradients (Sec. 3.3, Eq. 7-8 and the
 * colour/opacity/covariance analogues), the mapping losses (Eq. 9, Eq. 10
 * with its L1 and SSIM terms, the Eq. 11 scale regulariser of Eq. 12) and the
 * masked tracking loss (Eq. 15) with the pose gradient the tracking
 * optimisation (Eq. 14) needs; around them, the map upkeep of Sec. 3.2 and
 * the supplement: seeding candidates and their neighbour queries, and opacity
 * pruning.
 *
 * Conventions shared by every call
 *  - All array arguments are DEVICE pointers to contiguous float32 (unless
 *    stated), owned by the caller, 4-byte aligned (quats: 16-byte aligned),
 *    never aliased with an output of the same call.
 *  - Gaussians: means [n,3], scales [n,3] (the positive per-axis standard
 *    deviations s of Sigma = R diag(s)^2 R^T), quats [n,4] (w,x,y,z, any
 *    non-zero norm; normalised inside), opacities [n] (in (0,1]), colors [n,3]
 *    (RGB, no spherical harmonics, as the paper optimises RGB directly).
 *  - pose7 (device, 7 floats): (qw,qx,qy,qz,tx,ty,tz) of the world-to-camera
 *    transform x_cam = R(q/|q|) mu + t. Camera axes: +x right, +y down, +z
 *    forward; pixel (px,py) is sampled at the continuous point (px,py).
 *  - Images are planar: color [3,H,W], depth [H,W], alpha [H,W].
 *  - Every call enqueues work on the context's HIP stream and returns without
 *    waiting, except where noted ("synchronises"). Inputs must stay alive and
 *    unmodified until the stream has passed the call; the backward re-reads
 *    the forward's Gaussian and pose inputs.
 *  - Errors: every call returns GSR_OK (0) or a negative code; no exception
 *    crosses the ABI. gsr_last_error() gives a message for the last failure
 *    on that context (with NULL: of the calling thread's last failed
 *    context-free call). A degenerate Gaussian (non-finite parameters, zero
 *    quaternion, depth <= near_z, singular 2D covariance, opacity below
 *    alpha_min, support box off the image) is not an error: it is culled and
 *    receives zero gradient.
 */
#ifndef GSR_H_
#define GSR_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GSR_OK = 0,
  GSR_EINVAL = -1,    /* bad argument: NULL required pointer, n < 0, W/H <= 0,
                         non-finite intrinsics, unsupported tile shape */
  GSR_ENOMEM = -2,    /* device allocation failed */
  GSR_EHIP = -3,      /* a HIP runtime call failed (text in gsr_last_error) */
  GSR_EOVERFLOW = -4  /* a fixed-capacity (graph) buffer was too small */
};

typedef struct gsr_ctx gsr_ctx;     /* opaque: stream, workspaces, graphs */
typedef struct gsr_state gsr_state; /* opaque: what one forward leaves for its backward */

/* Pinhole camera (host struct, passed by pointer and copied). */
typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float near_z; /* Gaussians with camera depth <= near_z are culled */
  float bg[3];  /* background colour composited behind the last Gaussian */
} gsr_camera;

/* Rasterizer constants (host struct). Defaults: lowpass 0.3 px^2, alpha_min
 * 1/255, alpha_max 0.99, T_min 1e-4, guard 1.3, tile 16x16, deterministic 0. */
typedef struct {
  float lowpass;   /* h added to both diagonal entries of Sigma' */
  float alpha_min; /* pairs with alpha < alpha_min are skipped */
  float alpha_max; /* alpha = min(alpha_max, o exp(-sigma)) */
  float T_min;     /* a pixel stops before the Gaussian that would take T below it */
  float guard;     /* lateral clamp of x/z, y/z inside J: guard * max(c, size-c) / f */
  int32_t tile_w, tile_h; /* 16x16, 8x32 or 32x8 */
  /* 0: the backward adds per-tile partial sums with float atomics (fastest;
   *    the order of those additions, and so the last bits of the gradients,
   *    varies between runs).
   * 1: the backward stores every (Gaussian, tile, 8x8 pixel block) partial
   *    sum (4x4 quadrant when only the pose gradient is wanted) and adds them
   *    per Gaussian in a fixed order (tiles in row-major order of its tile
   *    rectangle, blocks in order), so
   *    gradients are bitwise reproducible; it needs 648 bytes per tile
   *    overlap and 4 per Gaussian and view more device memory, allocated by
   *    the first such backward of a state (synchronises), and is slower.
   *    Not supported by the tracking graph (GSR_EINVAL). */
  int32_t deterministic;
} gsr_opts;

typedef struct {
  int64_t n;
  const float *means, *scales, *quats, *opacities, *colors;
} gsr_gaussians;

/* Gradient outputs of the backward (device). NULL = not wanted. Overwritten. */
typedef struct {
  float *means, *scales, *quats, *opacities, *colors;
} gsr_grads;

/* Library / context ---------------------------------------------------- */

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the default stream). */
int gsr_ctx_create(gsr_ctx **out, int device, void *hip_stream);
int gsr_ctx_destroy(gsr_ctx *ctx);
/* Change the stream later calls enqueue on. */
int gsr_set_stream(gsr_ctx *ctx, void *hip_stream);
const char *gsr_strerror(int code);
const char *gsr_last_error(gsr_ctx *ctx);
void gsr_default_opts(gsr_opts *out);

/* Forward render (Eq. 1-4, 6) ------------------------------------------ */

/* Render colour (+ background), depth (sum z alpha T, background depth 0) and
 * accumulated alpha 1 - T_final. Projection, tile binning, the per-tile depth
 * sort and compositing all run on the device. The call waits once for the
 * tile-overlap count K (to size its buffers); when the state's tile-list
 * workspace from an earlier call is large enough, the rest of the forward is
 * already queued by then, so the device does not wait for the host.
 * *state receives a handle the backward needs; release it with
 * gsr_state_release (it owns the sorted tile lists and per-pixel state). */
int gsr_render_fwd(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cam, const gsr_opts *opts,
                   const float *pose7, float *color, float *depth, float *alpha, gsr_state **state);

/* Batched forward over n_views keyframes of one sub-map (the active sub-map
 * is optimised against all its keyframes, Sec. 3.2). poses7: device [V,7];
 * outputs color [V,3,H,W], depth [V,H,W], alpha [V,H,W]. All views' (tile,
 * depth) keys are sorted together and every (view, tile) item is composited
 * by ONE launch: with blocks_per_cu > 0 a persistent grid of blocks_per_cu x
 * (compute units) workgroups takes items from a work counter, longest tile
 * list first; with 0, one workgroup per item. gsr_render_fwd is the V = 1,
 * blocks_per_cu = 0 case. Synchronises once (overlap count). */
int gsr_render_fwd_batch(gsr_ctx *ctx, const gsr_gaussians *g, int32_t n_views, const gsr_camera *cam,
                         const gsr_opts *opts, int32_t blocks_per_cu, const float *poses7, float *color,
                         float *depth, float *alpha, gsr_state **state);

/* Backward of gsr_render_fwd for upstream gradients dL/dcolor [3,H,W],
 * dL/ddepth [H,W] and dL/dalpha [H,W] (NULL = zero). Writes the gradients
 * w.r.t. the activated parameters (Sec. 3.3; Eq. 8 for the depth-alpha term,
 * plus the direct depth term dD/dz_j = alpha_j T_j), and, if non-NULL,
 * dL/dpose7 (7 floats: quaternion through its normalisation, translation)
 * and dL/dtwist6 (6 floats: (rho, phi) of the left perturbation
 * T <- exp(xi^) T). Transmittance is recomputed back to front, not stored. */
int gsr_render_bwd(gsr_ctx *ctx, gsr_state *state, const float *dL_dcolor, const float *dL_ddepth,
                   const float *dL_dalpha, const gsr_grads *grads, float *dL_dpose7, float *dL_dtwist6);
/* For a batched state the same call takes [V,3,H,W] / [V,H,W] upstream
 * gradients, sums the parameter gradients over the views, writes per-view pose
 * gradients dL_dpose7 [V,7] / dL_dtwist6 [V,6], and runs the compositing
 * backward with the forward's launch shape. */

/* Adam state of the five Gaussian parameter tensors, in the order means,
 * scales, quats, opacities, colors (device pointers; exp_avg / exp_avg_sq of
 * the same shapes as the parameters), with per-tensor step sizes lr. step >= 1
 * is the 1-based step count. */
typedef struct {
  float *params[5], *exp_avg[5], *exp_avg_sq[5];
  float lr[5];
  int64_t step;
  float beta1, beta2, eps;
  float scale_reg; /* lambda_reg of Eq. 12: the gradient of lambda_reg * L_reg (Eq. 11, as
                      gsr_loss_reg defines it) joins the scale gradient before the step; 0 = none */
} gsr_adam5;

/* A mapping optimiser step fused into the backward: the result equals
 * gsr_render_bwd (parameter gradients, no pose) followed by gsr_adam_groups
 * on the five parameter tensors, but each Gaussian's gradient is applied by
 * Adam in the kernel that completes it and is never stored. adam->params must
 * be the tensors the forward read (checked; GSR_EINVAL otherwise); they and
 * the moments are updated in place, so the state must not be used for
 * another backward afterwards. For a batched state the gradient is the sum
 * over the views. */
int gsr_render_bwd_adam(gsr_ctx *ctx, gsr_state *state, const float *dL_dcolor, const float *dL_ddepth,
                        const float *dL_dalpha, const gsr_adam5 *adam);

/* Tile-shape autotuner for the batched path: times forward + backward (reps
 * runs after one warm-up, HIP events) for every tile shape in {16x16, 8x32,
 * 32x8} and blocks_per_cu in {0, 1, 2, 4, 8} with the given upstream
 * gradients, writes the fastest shape into opts->tile_w / tile_h (the other
 * fields are inputs) and the fastest blocks_per_cu into *best_blocks_per_cu.
 * The backward timed is the mapping one (gradients of all five parameter
 * groups). ms_table (may be NULL) receives the 15 mean times, shape-major.
 * Allocates scratch images and gradients; synchronises. */
int gsr_autotune_batch(gsr_ctx *ctx, const gsr_gaussians *g, int32_t n_views, const gsr_camera *cam, gsr_opts *opts,
                       const float *poses7, const float *dL_dcolor, const float *dL_ddepth, int32_t reps,
                       int32_t *best_blocks_per_cu, float *ms_table);

int gsr_state_release(gsr_ctx *ctx, gsr_state *state);

/* Introspection of a forward's tile lists (O(K) copy; synchronises).
 * *K = number of (tile, Gaussian) overlaps; ranges (device int32 [n_tiles,2],
 * [start,end) into ids) and ids (device int32 [K]) may be NULL. Tiles are
 * numbered row-major with ceil(W/tile_w) tiles per row. */
int gsr_tile_lists(gsr_ctx *ctx, const gsr_state *state, int64_t *K, int32_t *ranges, int32_t *ids);

/* Losses (device outputs) ----------------------------------------------- */

/* Mapping L1 (Eq. 9 and the L1 part of Eq. 10):
 * L = w_color mean_{3P}|C - C*| + w_depth mean_P|D - D*|, sign(0) = 0.
 * loss: device float[1] (overwritten); gradients [3,P] and [P]. */
int gsr_loss_l1(gsr_ctx *ctx, const float *color, const float *depth, const float *tgt_color,
                const float *tgt_depth, int64_t n_pixels, float w_color, float w_depth, float *loss,
                float *dL_dcolor, float *dL_ddepth);

/* Candidate points of the seeding step (Sec. 3.2; alpha_n from the
 * supplement): Bernoulli thinning of a keyframe's pixels with caller-supplied
 * uniform random numbers u [H,W]. A pixel with positive depth is chosen
 *   - alpha == NULL (a sub-map's first keyframe): iff u < p_uniform, or
 *     u < p_uniform + p_grad where the grey image's gradient is an edge:
 *     grey = ((r + g) + b) / 3, gx / gy = central differences (none on the
 *     border), gx^2 + gy^2 > grad_thre^2;
 *   - else (later keyframes; alpha = the rendered alpha [H,W]): iff
 *     alpha < alpha_n and u < p_uniform.
 * These decisions are taken in FP32 without contraction. Chosen pixel (x, y)
 * with depth d back-projects to X_c = ((x - cx) d / fx, (y - cy) d / fy, d)
 * and X_w = R^T (X_c - t) for the world-to-camera pose7 (device, q normalised
 * inside). points and colors (device float [W H, 3] capacity) receive the
 * chosen ones in row-major pixel order; *n_out (host) their count. color
 * [3,H,W], depth [H,W]; camera by pointer as for rendering. Allocates
 * temporary device memory and synchronises the context's stream. */
int gsr_seed_candidates(gsr_ctx *ctx, const gsr_camera *cam, const float *pose7, const float *color,
                        const float *depth, const float *alpha, const float *u, float p_uniform, float p_grad,
                        float grad_thre, float alpha_n, float *points, float *colors, int64_t *n_out);

/* Stable compaction by a mask: as gsr_prune, but Gaussian i is kept iff
 * keep[i] != 0 (device int32 [n]); with gsr_seed_query's keep output it is the
 * supplement's merge of a sub-map into the global map (a Gaussian joins if the
 * map so far has none within rho). Synchronises. */
int gsr_compact(gsr_ctx *ctx, int64_t n, const int32_t *keep, const float *const *in, float *const *out,
                int64_t *n_kept);

/* Sub-map offload and restore (Sec. 3.2: only the active sub-map is kept in
 * GPU memory; a finished one is stored away until the global map is built).
 * Offload copies the n Gaussians' five parameter arrays in[0..4] (device:
 * means, scales, quats, opacities, colors) into one host buffer laid out
 * [means 3n | scales 3n | quats 4n | opacities n | colors 3n] (14 n floats);
 * restore copies such a buffer into the device arrays out[0..4]. Both
 * enqueue copies on the context's stream and return without waiting: the
 * host buffer must stay alive (and, for restore, unchanged) until the stream
 * has passed the call. With pinned host memory (hipHostMalloc) the copies
 * are asynchronous DMA; with pageable memory HIP may stage them. n >= 0
 * (n = 0 copies nothing). GSR_EINVAL for NULL arrays or host buffer. */
int gsr_submap_offload(gsr_ctx *ctx, int64_t n, const float *const *in, float *host);
int gsr_submap_restore(gsr_ctx *ctx, int64_t n, const float *host, float *const *out);

/* Sub-map creation rule (Sec. 3.2): a new sub-map starts when the current
 * frame's camera centre is more than d_thre from that of the active sub-map's
 * first frame, or the rotation between the two frames exceeds theta_thre
 * (radians; the angle of the relative rotation); the paper uses 0.5 m and 50
 * degrees. pose_first7, pose_cur7: HOST float[7] world-to-camera poses (q
 * normalised inside). *start_new = 1 or 0. Pure host computation (FP64);
 * returns GSR_EINVAL for a zero quaternion or non-finite thresholds. */
int gsr_submap_trigger(const float *pose_first7, const float *pose_cur7, float d_thre, float theta_thre,
                       int32_t *start_new);

/* Neighbour queries of the seeding step (Sec. 3.2: a sampled point becomes a
 * new Gaussian only if the active sub-map has no Gaussian within the search
 * radius rho; the supplement sets a new Gaussian's scale from its
 * nearest-neighbour distance in the sub-map). For each query point q_j:
 *   nn_d2[j] = min(r_max^2, min_i d2(q_j, p_i)),  keep[j] = (nn_d2[j] >= rho^2),
 * with d2 = (dx^2 + dy^2) + dz^2 in FP32 without contraction, r_max^2 and rho^2
 * rounded to FP32, and p_i the n sub-map means. The nearest-neighbour distance
 * is searched up to r_max (distances beyond it read as r_max^2).
 * means [n,3], points [m,3]: device float; nn_d2 [m] float and keep [m] int32
 * (device; either may be NULL). 0 < rho <= r_max, both finite;
 * 0 <= n <= 2^27, 0 <= m <= 2^31; coordinates within +-8000 r_max of the
 * origin (beyond that FP32 cell indices lose the precision the exact search
 * relies on). Builds a spatial hash grid in temporary device memory and
 * synchronises the context's stream. */
int gsr_seed_query(gsr_ctx *ctx, const float *means, int64_t n, const float *points, int64_t m, float rho,
                   float r_max, float *nn_d2, int32_t *keep);

/* New Gaussians from the seeding step (Sec. 3.2: the sampled points with no
 * sub-map Gaussian within rho become new Gaussians; supplement: their
 * opacity starts at 0.5 and their scale at the nearest-neighbour distance in
 * the active sub-map). For every j with keep[j] != 0, in order, row r of the
 * outputs receives mean = points[j], colour = colors[j], scale =
 * sqrt(nn_d2[j]) (correctly rounded FP32) on all three axes, quaternion
 * (1, 0, 0, 0) and opacity 0.5 (activated values, as everywhere in this
 * API). points, colors [m,3], nn_d2 [m] float and keep [m] int32 are device
 * arrays, as gsr_seed_candidates and gsr_seed_query produce them (a kept
 * point has nn_d2 >= rho^2 > 0); out[0..4] = means [.,3], scales [.,3], quats
 * [.,4] (16-byte aligned), opacities [.], colors [.,3]: device buffers with
 * room for m rows, not aliased with the inputs (append new Gaussians by
 * passing pointers just past a sub-map's last row). *n_new (host) receives the
 * count. 0 <= m < 2^31 (m = 0: *n_new = 0, the arrays are not read).
 * Allocates temporary device memory and synchronises the context's stream.
 * GSR_EINVAL for NULL arrays (m > 0) or a misaligned quaternion output. */
int gsr_seed_gaussians(gsr_ctx *ctx, int64_t m, const float *points, const float *colors, const float *nn_d2,
                       const int32_t *keep, float *const *out, int64_t *n_new);

/* Opacity pruning (supplement, mapping: at the middle and the end of a new
 * keyframe's iterations, Gaussians with opacity below o_thre are removed;
 * o_thre = 0.1 on Replica-like data, 0.5 otherwise). Stable compaction:
 * Gaussian i is kept iff opacities[i] >= o_thre (NaN is removed) and the kept
 * ones are written, in their order, to rows 0..n_kept-1 of the outputs.
 * in[0..4] = means [n,3], scales [n,3], quats [n,4], opacities [n], colors [n,3];
 * in[5..9] and in[10..14] = the matching Adam exp_avg / exp_avg_sq tensors,
 * each entry NULL if absent (out[t] must be NULL exactly where in[t] is).
 * Outputs are device buffers of the inputs' shapes (n rows), not aliased with
 * any input. *n_kept (host) receives the count. Allocates temporary device
 * memory and synchronises the context's stream. 0 <= n < 2^31. */
int gsr_prune(gsr_ctx *ctx, int64_t n, float o_thre, const float *const *in, float *const *out, int64_t *n_kept);

/* Isotropic scale regulariser (Eq. 11): L_reg = (1/N) sum_k |s_k - sbar_k|_1
 * with sbar_k = (s_k,x + s_k,y + s_k,z) / 3, the mean of Gaussian k's own
 * scales (activated scales; sign(0) = 0 in the gradient).
 * ACCUMULATES: *loss += weight L_reg and, if dL_dscales != NULL,
 * dL_dscales += weight dL_reg/dscales, so it runs after gsr_render_bwd (which
 * overwrites the parameter gradients). scales, dL_dscales: device float [n,3];
 * loss: device float[1]; n >= 0 (n = 0 adds nothing); weight finite. */
int gsr_loss_reg(gsr_ctx *ctx, const float *scales, int64_t n, float weight, float *loss, float *dL_dscales);

/* SSIM term of the mapping colour loss (Eq. 10: L_color = (1 - lambda) L1 +
 * lambda (1 - SSIM)), with SSIM as Wang et al. 2004 define it and the paper
 * cites: per channel, an 11x11 Gaussian window (sigma 1.5, weights summing to
 * one), zero padding at the image border, C1 = 1e-4 and C2 = 9e-4 for values
 * in [0, 1], averaged over the 3 channels and all pixels.
 * ACCUMULATES: *loss += weight (1 - SSIM(color, tgt_color)) and
 * dL_dcolor += weight d(1 - SSIM)/d color, so it runs after gsr_loss_l1 (which
 * overwrites both) with w_color = 1 - lambda and weight = lambda.
 * color, tgt_color, dL_dcolor: device float [3, height, width]; loss: device
 * float[1]. 0 <= width, height <= 65535 (GSR_EINVAL otherwise); an empty image
 * adds nothing. The gradient is with respect to color only. */
int gsr_loss_ssim(gsr_ctx *ctx, const float *color, const float *tgt_color, int32_t width, int32_t height,
                  float weight, float *loss, float *dL_dcolor);

/* Tracking loss (Eq. 15 with the supplement's masks): valid = observed depth
 * > 0; e = |D - D*|; m = lower median of e over valid pixels (exact, radix
 * select on the device); inlier = valid and e <= inlier_mult * m; weight =
 * inlier * alpha^3 (treated as constant, so dL/dalpha = 0);
 * L = sum_p weight (lambda_c sum_ch |C - C*| + (1 - lambda_c) |D - D*|).
 * loss, median: device float[1]; median may be NULL. */
int gsr_loss_track(gsr_ctx *ctx, const float *color, const float *depth, const float *alpha,
                   const float *tgt_color, const float *tgt_depth, int64_t n_pixels, float lambda_c,
                   float inlier_mult, float *loss, float *dL_dcolor, float *dL_ddepth, float *median);

/* gsr_loss_track without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): no context is needed, and the call makes no
 * hipMalloc, hipFree or other allocating call. Same arguments, result and
 * layout as gsr_loss_track; work is enqueued on hip_stream (NULL = the null
 * stream) of the CURRENT device and not waited for.
 * Scratch: the median's histograms and the loss reduction use a 32 KiB
 * static device array of the library (one per device, held until the
 * process ends), cleared by a fill kernel at the start of every call. Every
 * call on one device shares it: calls that overlap on one device (other
 * streams or threads without ordering between them) race and give wrong
 * results. n_pixels <= GSR_NOALLOC_MAX_PIXELS (the histogram counts are
 * 32-bit); larger is GSR_EINVAL. Errors: GSR_EINVAL (NULL required pointer,
 * n_pixels out of range), GSR_EHIP (device lookup or launch failed); the
 * message is gsr_last_error(NULL) on the calling thread. */
#define GSR_NOALLOC_MAX_PIXELS 4294967295LL
int gsr_loss_track_noalloc(void *hip_stream, const float *color, const float *depth, const float *alpha,
                           const float *tgt_color, const float *tgt_depth, int64_t n_pixels, float lambda_c,
                           float inlier_mult, float *loss, float *dL_dcolor, float *dL_ddepth, float *median);

/* Optimiser --------------------------------------------------------------- */

/* One bias-corrected Adam step (Kingma & Ba) on n device floats, in place;
 * step >= 1 is the 1-based step count. */
int gsr_adam(gsr_ctx *ctx, float *param, float *exp_avg, float *exp_avg_sq, const float *grad, int64_t n,
             int64_t step, float lr, float beta1, float beta2, float eps);

/* The same step on up to 8 parameter tensors in one launch (e.g. the five
 * Gaussian parameter groups of a mapping iteration), each with its own step
 * size: params[i], exp_avg[i], exp_avg_sq[i], grads[i] hold counts[i] device
 * floats; the pointer arrays, counts and lrs are host arrays. */
int gsr_adam_groups(gsr_ctx *ctx, int32_t n_groups, float *const *params, float *const *exp_avg,
                    float *const *exp_avg_sq, const float *const *grads, const int64_t *counts, const float *lrs,
                    int64_t step, float beta1, float beta2, float eps);

/* Tracking (Sec. 3.4) ------------------------------------------------------ */

/* Constant-speed pose initialisation (Eq. 13) on the quaternion and the
 * translation: t = 2 t1 - t0, q = normalise(2 q1 - q0) after flipping q0 into
 * q1's hemisphere. All three are device pose7 buffers. */
int gsr_pose_const_velocity(gsr_ctx *ctx, const float *pose_prev2, const float *pose_prev1, float *pose_out);

/* One Adam step on a pose7 (quaternion step size lr_q, translation lr_t) with
 * the step count kept on the device: state is a device float[20] buffer,
 * zero before the first step (m[0..7), v[8..15), step count at [16]). */
int gsr_pose_adam(gsr_ctx *ctx, float *pose7, float *state, const float *grad7, float lr_q, float lr_t, float beta1,
                  float beta2, float eps);

/* Left perturbation of a pose by a twist (rho, phi): R' = Exp(phi) R,
 * t' = Exp(phi) t + rho (device pose7 in, twist6, pose7 out; the output
 * quaternion is unit). This is how a proposed correction is applied. */
int gsr_pose_apply_twist(gsr_ctx *ctx, const float *pose7, const float *twist6, float *pose_out);

typedef struct gsr_track_graph gsr_track_graph; /* opaque: a captured tracking loop */

typedef struct {
  float lambda_c;     /* colour weight of Eq. 15 (depth weight 1 - lambda_c) */
  float inlier_mult;  /* inlier threshold multiple of the median depth error (50) */
  float lr_q, lr_t;   /* Adam step sizes of the quaternion and the translation */
  float beta1, beta2, eps;
  int32_t n_iters;    /* optimisation iterations per frame */
} gsr_track_opts;

/* Capture n_iters tracking iterations (Eq. 14): render the frozen Gaussians at
 * the current pose, masked tracking loss (Eq. 15) against the observed frame,
 * backward to the pose only, Adam on (q, t) -- as ONE hipGraph with fixed
 * capacities (K_cap tile overlaps per iteration; every K-dependent kernel
 * reads the actual K from device memory). The Gaussian pointers are captured
 * (their contents may change between runs, their count may not); the observed
 * colour [3,H,W] and depth [H,W] are copied into graph-owned buffers now and by
 * gsr_track_graph_set_frame. */
int gsr_track_graph_create(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cam, const gsr_opts *opts,
                           const gsr_track_opts *topts, const float *obs_color, const float *obs_depth,
                           int64_t K_cap, gsr_track_graph **out);
int gsr_track_graph_set_frame(gsr_ctx *ctx, gsr_track_graph *tg, const float *obs_color, const float *obs_depth);
/* Run one frame: pose7 (device, in/out) holds the initial pose and receives the
 * optimised one; losses (device float[n_iters], may be NULL) receive the loss
 * of every iteration. One graph launch; synchronises once to read the
 * capacity flag and returns GSR_EOVERFLOW if an iteration had more than K_cap
 * overlaps (the pose is then not valid: re-create with a larger K_cap). */
int gsr_track_graph_run(gsr_ctx *ctx, gsr_track_graph *tg, float *pose7, float *losses);
int gsr_track_graph_destroy(gsr_ctx *ctx, gsr_track_graph *tg);

/* Learned tracking initialisation ------------------------------------------
 * A small CNN that proposes a pose correction from the render at the current
 * pose and the observed frame. Input: 8 channels at 160 x 120 (rendered RGB
 * and depth x depth_scale, then 4 x the observed-minus-rendered RGB and depth
 * x depth_scale, f x f average-pooled from the full frames). Four 3x3
 * stride-2 convolutions with 64 channels and ReLU (implicit GEMMs on the BF16
 * matrix cores, FP32 accumulation, BF16 activations), moment pooling of the
 * last 10 x 8 map (per channel the mean and the means weighted by the pixel
 * centre's x and y mapped to (-1, 1): 192 values), linear head to 6 outputs
 * (the twist (rho, phi) of a left perturbation). The paper suggests
 * learned components in its limitations (Sec. 5) and uses a loss-judged
 * alternative initialiser in its supplement; this network is such an
 * initialiser, judged against constant-speed init by the tracking loss. */
typedef struct gsr_initnet gsr_initnet;

int gsr_initnet_create(gsr_ctx *ctx, int32_t max_batch, gsr_initnet **out);
int gsr_initnet_destroy(gsr_ctx *ctx, gsr_initnet *net);
/* Parameters: a flat FP32 vector of n_params floats, in order: per layer
 * l = 0..3: W_l [64][KP_l] (K ordered (3 ky + kx, channel); KP_0 = 96 with
 * 24 zero pad columns, KP_1..3 = 576), b_l [64]; then the head W_fc [6][192]
 * (columns: moment k = 0, 1, 2 of channel c at 64 k + c) and b_fc [6]. Zero after create. set_params copies a device vector in (and
 * resets Adam); get_params copies parameters and/or the last gradients out
 * (either pointer may be NULL). */
int gsr_initnet_count(gsr_ctx *ctx, gsr_initnet *net, int64_t *n_params);
int gsr_initnet_set_params(gsr_ctx *ctx, gsr_initnet *net, const float *src);
int gsr_initnet_get_params(gsr_ctx *ctx, gsr_initnet *net, float *params, float *grads);
/* Inputs are BF16 NHWC [B,120,160,8] (device, BF16 bit patterns). */
int gsr_initnet_set_input(gsr_ctx *ctx, gsr_initnet *net, int32_t batch, const uint16_t *src);
/* Copy out layer l's activation (l = 0: input; 1..4: post-ReLU [B,H_l,W_l,64])
 * and/or the gradient w.r.t. its pre-activation (after a backward). */
int gsr_initnet_get_activation(gsr_ctx *ctx, gsr_initnet *net, int32_t layer, int32_t batch, uint16_t *act,
                               uint16_t *dact);
/* Pack one input sample from full-resolution frames (W = 160 f, H = 120 f):
 * f x f average pooling into dst (BF16 [120,160,8]) of the rendered colour
 * and depth (x depth_scale) in channels 0-3 and of the observed-minus-rendered
 * colour and depth (x depth_scale), times 4, in channels 4-7 (the residual is
 * formed in FP32 before rounding to BF16). */
int gsr_pack_rgbd_pair(gsr_ctx *ctx, const float *rend_color, const float *rend_depth, const float *obs_color,
                       const float *obs_depth, int32_t H, int32_t W, float depth_scale, uint16_t *dst);
/* Forward of the first `batch` input samples; out: device [B,6] or NULL. */
int gsr_initnet_forward(gsr_ctx *ctx, gsr_initnet *net, int32_t batch, float *out);
/* Backward of the last forward: with dL_dout == NULL the loss is
 * L = 1/(2B) sum_b sum_j ((out - label) / scale_j)^2 (labels [B,6], scale [6],
 * device; L written to *loss if non-NULL), else dL_dout [B,6] is used.
 * Overwrites the gradient buffer. */
int gsr_initnet_backward(gsr_ctx *ctx, gsr_initnet *net, int32_t batch, const float *labels, const float *scale,
                         const float *dL_dout, float *loss);
/* Adam step on all parameters (bias-corrected, internal step count). */
int gsr_initnet_adam(gsr_ctx *ctx, gsr_initnet *net, float lr, float beta1, float beta2, float eps);

/* Measurement ------------------------------------------------------------ */

/* Stage timing for benchmarks: while enabled, every stage a call enqueues
 * (project, bin_count, tile_bins, render_fwd, fill, render_bwd, project_bwd,
 * project_bwd_adam, loss_l1, loss_reg, loss_ssim, loss_track, prune, compact, seed_candidates, seed_query, adam, pose_adam, track_graph,
 * initnet_fwd, initnet_bwd) is bracketed by a pair of HIP events on the context's stream.
 * The events carry no system-scope fence, so they do not write back or
 * invalidate caches, but each still costs a few microseconds of stream time. */
int gsr_profile_enable(gsr_ctx *ctx, int on);
/* Restricts stage timing to the stage named `stage` (NULL or "" = every
 * stage), so a timed loop can measure one kernel's duration with one event
 * pair per launch. The name is copied; GSR_EINVAL if it is 32 bytes or
 * longer. */
int gsr_profile_only(gsr_ctx *ctx, const char *stage);
/* Synchronises, then reports per stage name (NUL-terminated, 32 bytes each in
 * `names`) the summed milliseconds and the number of launches since the last
 * read, and clears the record. *n_stages receives the number of names, which
 * may exceed max_stages (only the first max_stages are written). */
int gsr_profile_read(gsr_ctx *ctx, int max_stages, char *names, double *total_ms, int64_t *counts, int *n_stages);
/* Work counters of a forward (synchronises; re-runs the compositing pass in
 * a counting mode that writes no image): out[0] K = (tile, Gaussian)
 * overlaps, out[1] visible Gaussians, out[2] (pixel, Gaussian) pairs with the
 * pixel inside the Gaussian's support box before the pixel stops (what the
 * forward must evaluate), out[3] pairs composited, out[4] support-box pairs
 * before each pixel's last composited Gaussian (what the backward must
 * evaluate), out[5] tiles. */
int gsr_state_stats(gsr_ctx *ctx, gsr_state *state, int64_t out[6]);

#ifdef __cplusplus
}
#endif

#endif /* GSR_H_ */
