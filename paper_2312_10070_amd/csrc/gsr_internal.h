// Internal declarations of libgsr: launch-constant structs, device helpers
// shared by the forward and backward kernels, and the host-side launchers.
// gfx950 (CDNA4) only: wave64, 256-thread workgroups for the tile kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsr.h"

namespace gsr {

constexpr float kLog2e = 1.4426950408889634f;
constexpr int kTileThreads = 256;  // one pixel per lane, 4 waves per tile
constexpr int kWave = 64;
constexpr int kRec = 4;  // float4s per projected record
// The support box is taken at level (1 + kBoxSlack) ln(o / alpha_min) + kBoxSlack
// of sigma instead of ln(o / alpha_min).
constexpr float kBoxSlack = 1e-3f;


// Launch constants of one render (by value into every kernel).
struct Raster {
  int W, H;
  int tw, th;         // tile shape (tw * th == 256)
  int tw_log2;        // log2(tw)
  int ntx, nty;       // tiles per row / column
  int n_tiles;        // ntx * nty (per view)
  float fx, fy, cx, cy, near_z;
  float lowpass, amin, amax, tmin;
  float log2_amin;    // log2(amin)
  float limx, limy;   // guard band on x/z and y/z inside the Jacobian
  float bg0, bg1, bg2;
};

// Per-Gaussian record written by the projection kernel. The quadratic form of
// Eq. 4 is stored pre-scaled so that one pair costs three FMAs:
//   p = pa dx^2 + pb dx dy + pc dy^2 = -sigma * log2(e),   alpha = o * 2^p.
//   rec_uvab = (u, v, pa, pb), rec_cob = (pc, o, bx, by), rec_rgbz = (r, g, b, z_cam)
// The three float4s of a record are interleaved in one 64-byte slot (kRec
// float4s, the fourth unused): a record gathered by its index touches one
// cache line instead of three. rec_uvab[kRec i], rec_cob[kRec i], ... address
// record i.
// where bx / by carry the pixel support box as bit patterns px0 | px1 << 16 and
// py0 | py1 << 16 (a wave skips records whose box misses its pixels).
struct PairEval {
  float alpha;   // min(alpha_max, o 2^p)
  float e;       // 2^p = exp(-sigma)
  bool use;      // alpha >= alpha_min
  bool clamped;  // o 2^p > alpha_max (alpha does not depend on o, sigma)
};

// The single definition of every per-pair discrete decision. The forward and
// the backward both call it, so skip / clamp decisions agree bit for bit. FP
// contraction is pinned: only the explicit fmaf calls fuse.
__device__ __forceinline__ PairEval eval_pair(float dx, float dy, float pa, float pb, float pc, float o,
                                              float amin, float amax) {
#pragma clang fp contract(off)
  const float t = pc * dy;
  const float p = fmaf(pa * dx, dx, fmaf(pb * dx, dy, t * dy));
  PairEval r;
  r.e = __builtin_amdgcn_exp2f(p);
  const float raw = o * r.e;
  r.clamped = raw > amax;
  r.alpha = fminf(raw, amax);  // = clamped ? amax : raw (raw is finite: p is)
  r.use = r.alpha >= amin;
  return r;
}

// Tile index of a workgroup. Workgroups are dealt round-robin to the 8 XCDs
// (each with its own L2); this gives each XCD a contiguous run of row-major
// tiles so neighbouring tiles, which share most Gaussians, hit the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// Wave-wide sums of ten per-lane values: returns the sum the lane ends with
// and sets *f to its field, or -1 (ten lanes end with one field each).
// Field-splitting butterfly: at each of four exchange steps a
// lane keeps half of its remaining fields and hands the other half to its
// partner (v_permlane32_swap across the 32-lane halves, v_permlane16_swap
// across rows, then DPP row_mirror / row_half_mirror inside rows), so the ten
// sums cost ~27 VALU operations instead of ten full 64-lane reductions. After
// the last quad reduction lane L holds field 8 b2 + 4 b3 + 2 b4 + b5 of its
// lane bits b_i.
__device__ __forceinline__ float perm_add32(float a, float b) {
  auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
__device__ __forceinline__ float perm_add16(float a, float b) {
  auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float wave_reduce10(const float v[10], int lane, int* f) {
  // step 1 (lane bit 5): pairs of fields (2k, 2k+1)
  const float r10 = perm_add32(v[0], v[1]);
  const float r11 = perm_add32(v[2], v[3]);
  const float r12 = perm_add32(v[4], v[5]);
  const float r13 = perm_add32(v[6], v[7]);
  const float r14 = perm_add32(v[8], v[9]);
  // step 2 (lane bit 4)
  const float r20 = perm_add16(r10, r11);
  const float r21 = perm_add16(r12, r13);
  const float r22 = perm_add16(r14, 0.f);
  // step 3 (lane bit 3): partner = 15 - i inside the row
  const bool b3 = (lane >> 3) & 1;
  const float a0 = b3 ? r21 : r20, c0 = b3 ? r20 : r21;
  const float r30 = a0 + dpp_f<0x140>(c0);                 // row_mirror
  const float a1 = b3 ? 0.f : r22, c1 = b3 ? r22 : 0.f;
  const float r31 = a1 + dpp_f<0x140>(c1);
  // step 4 (lane bit 2): partner = 7 - i inside the half row
  const bool b2 = (lane >> 2) & 1;
  const float a2 = b2 ? r31 : r30, c2 = b2 ? r30 : r31;
  float r4 = a2 + dpp_f<0x141>(c2);                        // row_half_mirror
  // steps 5-6: sum the quad
  r4 += dpp_f<0xb1>(r4);                                   // quad_perm [1,0,3,2]
  r4 += dpp_f<0x4e>(r4);                                   // quad_perm [2,3,0,1]
  const int fld = 8 * ((lane >> 2) & 1) + 4 * ((lane >> 3) & 1) + 2 * ((lane >> 4) & 1) + ((lane >> 5) & 1);
  *f = ((lane & 3) == 0 && fld < 10) ? fld : -1;
  return r4;
}

__device__ __forceinline__ int wave_max_int(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ float wave_sum_all(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Rotation matrix of a unit quaternion (w, x, y, z), row-major.
__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float R[9]) {
  const float xx = x * x, yy = y * y, zz = z * z;
  const float xy = x * y, xz = x * z, yz = y * z, wx = w * x, wy = w * y, wz = w * z;
  R[0] = 1.f - 2.f * (yy + zz);
  R[1] = 2.f * (xy - wz);
  R[2] = 2.f * (xz + wy);
  R[3] = 2.f * (xy + wz);
  R[4] = 1.f - 2.f * (xx + zz);
  R[5] = 2.f * (yz - wx);
  R[6] = 2.f * (xz - wy);
  R[7] = 2.f * (yz + wx);
  R[8] = 1.f - 2.f * (xx + yy);
}

// Gradient of <G, R(q)> w.r.t. a unit quaternion, then through q / |q|.
__device__ __forceinline__ void quat_rot_vjp(const float qh[4], float inv_norm, const float G[9], float gq[4]) {
  const float w = qh[0], x = qh[1], y = qh[2], z = qh[3];
  float gw = 2.f * (x * (G[7] - G[5]) + y * (G[2] - G[6]) + z * (G[3] - G[1]));
  float gx = 2.f * (y * (G[1] + G[3]) + z * (G[2] + G[6]) + w * (G[7] - G[5])) - 4.f * x * (G[4] + G[8]);
  float gy = 2.f * (x * (G[1] + G[3]) + w * (G[2] - G[6]) + z * (G[5] + G[7])) - 4.f * y * (G[0] + G[8]);
  float gz = 2.f * (w * (G[3] - G[1]) + x * (G[2] + G[6]) + y * (G[5] + G[7])) - 4.f * z * (G[0] + G[4]);
  const float d = w * gw + x * gx + y * gy + z * gz;
  gq[0] = (gw - w * d) * inv_norm;
  gq[1] = (gx - x * d) * inv_norm;
  gq[2] = (gy - y * d) * inv_norm;
  gq[3] = (gz - z * d) * inv_norm;
}

// ---------------------------------------------------------------------------
// Host-side launchers (defined in the .hip files, called by gsr_api.cpp).
// ---------------------------------------------------------------------------

struct ProjectArgs {
  int64_t n;
  const float *means, *scales, *quats, *opacities, *colors;
  const float* pose7;  // device
  float4* rec_uvab;
  float4* rec_cob;
  float4* rec_rgbz;
  int4* rect;          // (tx0 | tx1 << 16, ty0 | ty1 << 16, depth bits, tiles); see BinArgs
  uint32_t* counts;    // tiles per Gaussian (0 = culled)
  int n_views;         // outputs are [n_views * n]; view v uses pose7 + 7 v
};
void launch_project(const Raster& R, const ProjectArgs& a, hipStream_t s);

// Exclusive scan of n uint32 values; writes the total to *total (device) and,
// if total_host is not NULL, to that device-visible pinned host word.
// temp must hold scan_temp_words(n) uint32.
int64_t scan_temp_words(int64_t n);
void launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* temp,
                           hipStream_t s, uint32_t* total_host = nullptr);

// Seeding candidates (k_seed.hip): chosen pixels back-projected to world
// points [m,3] with their colours [m,3], in pixel order; the count goes to
// count_host (pinned, device-visible). temp: seed_sample_temp_words(W H) uint32.
struct SeedSample {
  const float *color, *depth, *alpha, *u, *pose7;  // alpha NULL: a sub-map's first keyframe
  int W, H;
  float fx, fy, cx, cy;
  float p_uniform, p_grad, g2thre, alpha_n;
};
int64_t seed_sample_temp_words(int64_t P);
void launch_seed_sample(const SeedSample& a, float* points, float* colors, uint32_t* temp, uint32_t* count_host,
                        hipStream_t s);

// New Gaussians from the kept seeding points (k_seed.hip): rows 0..n_new-1 of
// the outputs, in point order; count_host (pinned, device-visible) receives
// n_new. temp: seed_init_temp_words(m) uint32.
struct SeedInit {
  int64_t m;
  const float* points;   // [m,3]
  const float* pcolors;  // [m,3]
  const float* nn_d2;    // [m]
  const int32_t* keep;   // [m]
  float *means, *scales, *quats, *opacities, *colors;
};
int64_t seed_init_temp_words(int64_t m);
void launch_seed_init(const SeedInit& a, uint32_t* temp, uint32_t* count_host, hipStream_t s);
// Seeding neighbour queries (k_seed.hip): nn_d2[j] = min(r_max^2, min_i |q_j - p_i|^2),
// keep[j] = nn_d2[j] >= rho^2 (either output may be NULL); rho <= r_max.
// temp: seed_temp_words(n) uint32, 16-byte aligned; launch_seed_grid fills it
// with the hash grid of the means, launch_seed_query then answers the queries.
uint32_t seed_buckets(int64_t n);
int64_t seed_temp_words(int64_t n);
void launch_seed_grid(const float* means, int64_t n, float r_max, uint32_t* temp, hipStream_t s);
void launch_seed_query(int64_t n, const float* points, int64_t m, float rho, float r_max, float* nn_d2,
                       int32_t* keep, const uint32_t* temp, hipStream_t s);

// Opacity pruning / compaction: in[0..4] = means, scales, quats, opacities,
// colors (widths 3, 3, 4, 1, 3), in[5..9] / in[10..14] their Adam moments
// (NULL = absent; out[t] NULL exactly where in[t] is). Keeps the Gaussians
// with mask[i] != 0 (mask given) or opacity >= thre (mask NULL), in their
// order, at the front of out; the count goes to kept_host (pinned,
// device-visible). temp: prune_temp_words(n) uint32.
struct PruneArgs {
  const float* in[15];
  float* out[15];
};
int64_t prune_temp_words(int64_t n);
void launch_prune(const PruneArgs& a, int64_t n, float thre, const int32_t* mask, uint32_t* temp, uint32_t* kept_host,
                  hipStream_t s);

// Tile binning (see k_sort.hip). Workgroup w of view v handles the Gaussians
// [w c, (w + 1) c) with c = ceil(n / n_wg); M[item][w] is the offset of its
// pairs inside the range of the (view, tile) item, R[item] that range.
// rect[o] = (tx0 | tx1 << 16, ty0 | ty1 << 16, float bits of the camera
// depth, number of tiles; 0 = not binned): everything binning reads, 16 bytes.
struct BinArgs {
  int64_t n;
  int n_views;
  int n_wg;                // workgroups per view
  const int4* rect;
  uint32_t* M;             // [n_items][n_wg]
  uint32_t* T;             // [n_items] pair totals; zero between launches
  int2* R;                 // [n_items] unclipped ranges
  uint32_t* ticket;        // zero between launches
  uint32_t* K;             // overlap count
  uint32_t* K_host;        // NULL or a device-visible host word that also receives K
  int64_t cap;             // positions >= cap are dropped and flagged
  uint64_t* keys;          // [cap] (depth bits << 32 | record index)
  int* overflow;
  int2* ranges;            // [n_items] written by the placement pass (NULL while counting)
};
int bin_workgroups(int64_t n);
// M, R and K from the tile rectangles (LDS histograms, one reservation atomic
// per (tile, workgroup), the last workgroup scans the tile totals).
void launch_bin_count(const Raster& R, const BinArgs& a, hipStream_t s);
// ranges from R, slot placement (LDS counters seeded from R and M), then one
// LDS sort per tile writing ids[cap] (record indices in depth order).
// scratch: [cap] keys, used by ranges longer than LDS holds.
void launch_tile_bins(const Raster& R, const BinArgs& a, int64_t n_items, int2* ranges, uint64_t* scratch,
                      uint32_t* ids, hipStream_t s);

struct FwdArgs {
  const int2* ranges;
  const uint32_t* ids;
  const float4* rec_uvab;
  const float4* rec_cob;
  const float4* rec_rgbz;
  float *color, *depth, *alpha, *Tfin;  // [V,3,H,W] / [V,H,W]
  int* last;
  unsigned long long* stats;  // non-NULL: count work only, write no outputs
  int n_items;                // views * tiles; item = view * n_tiles + tile
  int* queue;                 // persistent launch: work counter (zeroed first)
  const int* order;           // persistent launch: item order (NULL = identity)
  int blocks;                 // persistent launch: workgroups (0 = one per item)
};
void launch_render_fwd(const Raster& R, const FwdArgs& a, hipStream_t s);

struct BwdArgs {
  const int2* ranges;
  const uint32_t* ids;
  const float4* rec_uvab;
  const float4* rec_cob;
  const float4* rec_rgbz;
  const float* Tfin;
  const int* last;
  const float *gC, *gD, *gA;
  float* g2d;  // [V*n, 10]: sums of q (dx, dy, dx^2, dx dy, dy^2), q = dL/dp / ln 2; o, r, g, b, z
  bool geom_only;  // only fields 0-4 and 9 are needed (no opacity or colour gradient wanted)
  int n_items;
  int* queue;
  const int* order;
  int blocks;
  // deterministic backward (both NULL otherwise): per (list position,
  // quadrant of the tile) sums [K, 16, 10 or 6] and per list position the
  // 16-bit mask of the quadrants that stored one (zero before the launch)
  float* part;
  uint32_t* mask;
};
void launch_render_bwd(const Raster& R, const BwdArgs& a, hipStream_t s);
// Deterministic backward: list positions of each record's tiles (before the
// compositing pass), and the fixed-order sums into g2d (after it).
void launch_det_rev(const Raster& R, const int2* ranges, const uint32_t* ids, const int4* rect, const uint32_t* goff,
                    uint32_t* rev, int n_items, hipStream_t s);
void launch_det_reduce(const int4* rect, const uint32_t* goff, const uint32_t* rev, const uint32_t* mask,
                       const float* part, int64_t n_rec, bool geom_only, float* g2d, hipStream_t s);

// Adam applied by the projection backward to each Gaussian's gradient as soon
// as it is complete (groups: means, scales, quats, opacities, colors); p[i]
// are the parameters the forward read, updated in place.
struct AdamFused {
  float *p[5], *m[5], *v[5];
  float lr[5];
  float b1, b2, eps, bc1, bc2;
  float reg_w;  // Eq. 11 weight lambda_reg / N added to the scale gradient before the step; 0 = none
  bool on;
};

// Isotropic scale regulariser (Eq. 11) of one Gaussian: returns
// sum_i |s_i - sbar| with sbar = (s0 + s1 + s2) / 3, and writes
// d[j] = w (sign(r_j) - mean_i sign(r_i)), r = s - sbar, sign(0) = 0.
// Contraction is pinned so every kernel that applies it rounds alike.
__device__ __forceinline__ float reg_term(float s0, float s1, float s2, float w, float d[3]) {
#pragma clang fp contract(off)
  const float sbar = (s0 + s1 + s2) / 3.f;
  const float r0 = s0 - sbar, r1 = s1 - sbar, r2 = s2 - sbar;
  const float g0 = (float)((r0 > 0.f) - (r0 < 0.f)), g1 = (float)((r1 > 0.f) - (r1 < 0.f)),
              g2 = (float)((r2 > 0.f) - (r2 < 0.f));
  const float gm = (g0 + g1 + g2) / 3.f;
  d[0] = w * (g0 - gm);
  d[1] = w * (g1 - gm);
  d[2] = w * (g2 - gm);
  return fabsf(r0) + fabsf(r1) + fabsf(r2);
}

struct ProjectBwdArgs {
  int64_t n;
  const float *means, *scales, *quats, *opacities, *colors;
  const float* pose7;
  const uint32_t* counts;
  float* g2d;  // read, then cleared (zero again for the next backward)
  float *g_means, *g_scales, *g_quats, *g_opacities, *g_colors;  // may be NULL; summed over views
  float* pose_acc;  // [n_views][blocks][12] per-workgroup dL/dR_p (9, row-major), dL/dt (3); NULL = skip
  int n_views;
  AdamFused adam;  // adam.on: apply Adam instead of (or as well as) writing the gradients
};
// workgroups of the projection backward (one per 256 Gaussians)
int64_t project_bwd_blocks(int64_t n);
void launch_project_bwd(const Raster& R, const ProjectBwdArgs& a, hipStream_t s);
// Sums the per-workgroup pose partials in a fixed order and converts them.
// Adam on the 7 pose parameters (q: lr_q, t: lr_t), bias-corrected with the
// step count kept in state = [m(8), v(8), step(1)]; element i of a step.
__device__ __forceinline__ void pose_adam_elem(float* pose, float* state, int i, float gi, float t, float lr_q,
                                               float lr_t, float b1, float b2, float eps) {
  const float mi = b1 * state[i] + (1.f - b1) * gi;
  const float vi = b2 * state[8 + i] + (1.f - b2) * gi * gi;
  state[i] = mi;
  state[8 + i] = vi;
  const float bc1 = 1.f - powf(b1, t), bc2 = 1.f - powf(b2, t);
  const float lr = i < 4 ? lr_q : lr_t;
  pose[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

struct PoseAdam {
  float* state;  // NULL: no step
  float lr_q, lr_t, b1, b2, eps;
};

// With adam.state non-NULL (one view), also applies the pose Adam step to
// pose7 (in place) with the gradient just formed.
void launch_pose_finalize(const float* pose7, const float* pose_acc, int64_t blocks, float* dL_dpose7,
                          float* dL_dtwist6, int n_views, hipStream_t s, const PoseAdam* adam = nullptr);
// Longest-list-first order of (view, tile) items for the persistent launches
// (power-of-two length buckets). temp: 64 ints.
void launch_item_order(const int2* ranges, int n_items, int* order, int* temp, hipStream_t s);

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);

// red: reduce_temp_words() uint32, zero before its first use (the loss kernels
// leave it zero again).
int64_t reduce_temp_words();
void launch_loss_l1(const float* C, const float* D, const float* Ct, const float* Dt, int64_t P, float wc, float wd,
                    float* loss, float* gC, float* gD, uint32_t* red, hipStream_t s);
// Adds weight * L_reg (Eq. 11) of scales [n,3] to *loss and, if g != NULL, its
// gradient to g [n,3].
void launch_loss_reg(const float* scales, int64_t n, float weight, float* loss, float* g, uint32_t* red,
                     hipStream_t s);
// Adds weight (1 - SSIM(X, Y)) to *loss and its gradient to gX ([3,H,W]).
void launch_loss_ssim(const float* X, const float* Y, int H, int W, float weight, float* loss, float* gX,
                      uint32_t* red, hipStream_t s);
// temp: track_temp_words() uint32, zero before the first call (every call leaves it zero)
int64_t track_temp_words();
void launch_loss_track(const float* C, const float* D, const float* A, const float* Ct, const float* Dt, int64_t P,
                       float lambda_c, float inlier_mult, float* loss, float* gC, float* gD, float* median,
                       uint32_t* temp, hipStream_t s);
void launch_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                 float bc1, float bc2, hipStream_t s);

void launch_pose_adam(float* pose, float* state, const float* g, float lr_q, float lr_t, float b1, float b2, float eps,
                      hipStream_t s);
// One bias-corrected Adam step (Kingma & Ba) on one value; bc1 = 1 - b1^t,
// bc2 = 1 - b2^t. Contraction is pinned so every kernel that applies it (the
// group step, the single-tensor step and the step fused into the projection
// backward) rounds identically.
__device__ __forceinline__ void adam_one(float& p, float& m, float& v, float g, float lr, float b1, float b2,
                                         float eps, float bc1, float bc2) {
#pragma clang fp contract(off)
  m = b1 * m + (1.f - b1) * g;
  v = b2 * v + (1.f - b2) * g * g;
  p -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

constexpr int kAdamGroups = 8;
struct AdamGroups {
  float* p[kAdamGroups];
  float* m[kAdamGroups];
  float* v[kAdamGroups];
  const float* g[kAdamGroups];
  float lr[kAdamGroups];
  int64_t off[kAdamGroups + 1];
  int n;
};
void launch_adam_multi(const AdamGroups& a, float b1, float b2, float eps, float bc1, float bc2, hipStream_t s);

// Tracking-initialisation CNN (k_initnet.hip). BF16 values travel as uint16_t bits.
int conv_kp(int C);
void launch_conv_fwd(int B, int H, int W, int C, const uint16_t* in, const uint16_t* wk, const float* bias,
                     uint16_t* out, hipStream_t st);
void launch_conv_bwd_data(int B, int H, int W, int C, const uint16_t* dout, const uint16_t* wt, const uint16_t* in,
                          uint16_t* din, hipStream_t st);
void launch_conv_bwd_weight(int B, int H, int W, int C, const uint16_t* dy, const uint16_t* in, float* dw, float* db,
                            hipStream_t st);
void launch_head_fwd(int B, int OH, int OW, const uint16_t* act, const float* wfc, const float* bfc, float* pool,
                     float* out, hipStream_t st);
void launch_head_bwd(int B, int OH, int OW, const float* out, const float* label, const float* scale,
                     const float* pool, const float* wfc, const uint16_t* act, const float* dout, float* dwfc,
                     float* dbfc, uint16_t* dact, float* loss, hipStream_t st);
void launch_cast_weights(const float* w, int C, uint16_t* wk, uint16_t* wt, hipStream_t st);
void launch_pack_input(const float* rc, const float* rd, const float* oc, const float* od, int H, int W, int f,
                       float depth_scale, uint16_t* out, hipStream_t st);
void launch_pose_const_velocity(const float* p0, const float* p1, float* out, hipStream_t s);
void launch_pose_apply_twist(const float* pose, const float* xi, float* out, hipStream_t s);

}  // namespace gsr
