// C ABI of libgsr (declared in include/gsr.h): argument checking, workspace
// management and the launch sequence of each call. No compute happens here;
// every step of the hot path is one of the kernels in k_*.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gsr_internal.h"

struct gsr_state {
  gsr_ctx* ctx = nullptr;
  bool in_use = false;
  gsr::Raster R{};
  int64_t n = 0, P = 0, K = 0;
  gsr_gaussians g{};
  const float* pose7 = nullptr;
  // capacities of the two arenas
  int64_t n_cap = -1, P_cap = -1, tiles_cap = -1, K_cap = -1, views_cap = -1, bin_cap = -1;
  void* arenaA = nullptr;
  void* arenaB = nullptr;
  // arena A: per Gaussian / pixel / tile
  float4* rec_uvab = nullptr;
  float4* rec_cob = nullptr;
  float4* rec_rgbz = nullptr;
  int4* rect = nullptr;
  uint32_t* counts = nullptr;
  int n_wg = 1;                    // binning workgroups per view
  uint32_t* bin_M = nullptr;       // [items][n_wg]: a workgroup's offset inside a (view, tile) range
  uint32_t* bin_T = nullptr;       // [items]: pair totals (zero between forwards)
  int2* bin_R = nullptr;           // [items]: unclipped ranges
  uint32_t* bin_ticket = nullptr;  // zero between forwards
  float* g2d = nullptr;
  float* Tfin = nullptr;
  int* last = nullptr;
  int2* ranges = nullptr;
  uint32_t* d_K = nullptr;
  int* d_overflow = nullptr;
  float* pose_acc = nullptr;  // [views][projection-backward workgroups][12]
  int* queue = nullptr;       // persistent-launch work counter
  int* order = nullptr;       // [views * tiles] longest-list-first item order
  int* order_temp = nullptr;  // 64 ints
  int n_views = 1;
  int blocks = 0;             // persistent workgroups (0 = one per item)
  // arena B: per overlap
  uint64_t* keys = nullptr;     // [K] (depth bits << 32 | record index), slot order
  uint64_t* scratch = nullptr;  // [K] merge buffer for tile ranges longer than LDS holds
  uint32_t* ids = nullptr;      // [K] record indices, per tile in depth order
  // deterministic backward (opts.deterministic): arena D, allocated by the
  // first such backward of the state
  bool det = false;
  void* arenaD = nullptr;
  int64_t det_K_cap = -1, det_n_cap = -1;
  uint32_t* det_goff = nullptr;   // [V n] exclusive scan of the records' tile counts
  uint32_t* det_total = nullptr;  // [1]
  uint32_t* det_scan = nullptr;   // scan temp
  uint32_t* det_rev = nullptr;    // [K] list position of each (record, tile of its rectangle)
  uint32_t* det_mask = nullptr;   // [K] quadrants that stored a sum
  float* det_part = nullptr;      // [K, 16, 10] per (list position, quadrant) sums
};

struct gsr_track_graph {
  gsr_ctx* ctx = nullptr;
  gsr_state* s = nullptr;  // owned (not in the context's pool)
  int32_t n_iters = 0;
  int64_t K_cap = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* buf = nullptr;  // pose, Adam state, gradients, losses, images
  float *pose = nullptr, *adam = nullptr, *dpose = nullptr, *loss = nullptr, *median = nullptr;
  float *color = nullptr, *depth = nullptr, *alpha = nullptr, *gC = nullptr, *gD = nullptr;
  float *obs_c = nullptr, *obs_d = nullptr;
  uint32_t* sel_temp = nullptr;
  int* h_flag = nullptr;
};

// Tracking-initialisation network: FP32 master parameters (flat), BF16
// working copies, activations and gradients for up to max_batch samples.
struct gsr_initnet {
  static constexpr int kLayers = 4;
  static constexpr int kInH = 120, kInW = 160, kInC = 8, kCh = 64, kHeadIn = 3 * 64;  // head: three moments
  gsr_ctx* ctx = nullptr;
  int max_batch = 0;
  void* buf = nullptr;
  int64_t n_params = 0;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  float* w[kLayers] = {};   // into params
  float* b[kLayers] = {};
  float* dw[kLayers] = {};  // into grads
  float* db[kLayers] = {};
  float *wfc = nullptr, *bfc = nullptr, *dwfc = nullptr, *dbfc = nullptr;
  uint16_t* wk[kLayers] = {};
  uint16_t* wt[kLayers] = {};
  uint16_t* act[kLayers + 1] = {};  // act[0] = packed input
  uint16_t* dact[kLayers + 1] = {}; // gradient w.r.t. each layer's pre-activation (masked)
  int H[kLayers + 1] = {}, W[kLayers + 1] = {}, C[kLayers + 1] = {};
  float *pool = nullptr, *out = nullptr, *scratch = nullptr;
  int64_t step = 0;
};

struct gsr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<gsr_state*> pool;
  uint32_t* h_K = nullptr;      // pinned host word for the overlap count
  uint32_t* h_K_dev = nullptr;  // its device-side address (written by the scan kernel)
  hipEvent_t k_ev = nullptr;  // recorded after the scan that writes the overlap count
  uint32_t* red = nullptr;  // grid-reduction scratch of the L1 loss
  uint32_t* track_temp = nullptr;
  unsigned long long* d_stats = nullptr;
  int n_cu = 256;  // compute units of the device
  // stage timing (gsr_profile_*): an event pair around each stage launch
  struct Rec {
    const char* name;
    hipEvent_t a, b;
  };
  bool prof = false;
  std::string prof_only;  // empty: every stage
  std::vector<Rec> recs;
  std::vector<hipEvent_t> spare;
};

namespace {

int fail(gsr_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(gsr_ctx* c, hipError_t e, const char* what) {
  return fail(c, GSR_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define GSR_HIP(ctx, call)                                  \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #call); \
  } while (0)

int check_launch(gsr_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, what);
  return GSR_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(int64_t count) {
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += align_up(sizeof(T) * (size_t)(count > 0 ? count : 1));
    return p;
  }
};

// n, P, tiles are totals over views; nm = entries of the binning matrices.
void carve_A(gsr_state* s, char* base, int64_t n, int64_t P, int64_t tiles, int64_t views, int64_t nm,
             size_t* bytes) {
  Carver c{base};
  s->rec_uvab = c.take<float4>(gsr::kRec * n);  // interleaved records (see gsr_internal.h)
  s->rec_cob = s->rec_uvab ? s->rec_uvab + 1 : nullptr;
  s->rec_rgbz = s->rec_uvab ? s->rec_uvab + 2 : nullptr;
  s->rect = c.take<int4>(n);
  s->counts = c.take<uint32_t>(n);
  s->bin_M = c.take<uint32_t>(nm);
  s->bin_T = c.take<uint32_t>(tiles);
  s->bin_R = c.take<int2>(tiles);
  s->bin_ticket = c.take<uint32_t>(4);
  s->g2d = c.take<float>(10 * n);
  s->Tfin = c.take<float>(P);
  s->last = c.take<int>(P);
  s->ranges = c.take<int2>(tiles);
  s->d_K = c.take<uint32_t>(4);
  s->d_overflow = c.take<int>(4);
  // sum over views of ceil(n_view / 256) <= ceil(n / 256) + views workgroups
  s->pose_acc = c.take<float>(12 * (gsr::project_bwd_blocks(n) + views + 1));
  s->queue = c.take<int>(4);
  s->order = c.take<int>(tiles);
  s->order_temp = c.take<int>(64);
  *bytes = c.off;
}

void carve_B(gsr_state* s, char* base, int64_t K, size_t* bytes) {
  Carver c{base};
  s->keys = c.take<uint64_t>(K);
  s->scratch = c.take<uint64_t>(K);
  s->ids = c.take<uint32_t>(K);
  *bytes = c.off;
}

int ensure_A(gsr_ctx* c, gsr_state* s, int64_t n, int64_t P, int64_t tiles, int64_t views) {
  const int64_t nm_req = tiles * gsr::bin_workgroups(n / std::max<int64_t>(views, 1));
  if (s->arenaA && n <= s->n_cap && P <= s->P_cap && tiles <= s->tiles_cap && views <= s->views_cap &&
      nm_req <= s->bin_cap)
    return GSR_OK;
  if (s->arenaA) GSR_HIP(c, hipFree(s->arenaA));
  s->arenaA = nullptr;
  const int64_t nn = std::max<int64_t>(n + n / 4, 1024), PP = std::max<int64_t>(P, 256),
                tt = std::max<int64_t>(tiles, 16), vv = std::max<int64_t>(views, 1);
  const int64_t nm = std::max<int64_t>(tt * gsr::bin_workgroups(nn / vv), nm_req);
  size_t bytes = 0;
  carve_A(s, nullptr, nn, PP, tt, vv, nm, &bytes);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, GSR_ENOMEM, "device allocation of the per-Gaussian workspace failed");
  }
  s->arenaA = p;
  carve_A(s, (char*)p, nn, PP, tt, vv, nm, &bytes);
  // The per-Gaussian backward sums start at zero and every backward leaves them
  // at zero (the projection backward clears what it reads), so they are
  // cleared only here, when the workspace is allocated.
  gsr::launch_fill_f32(s->g2d, 0.f, 10 * nn, c->stream);
  // likewise the binning's tile totals and ticket (the counting pass's last
  // workgroup returns them to zero)
  gsr::launch_fill_u32(s->bin_T, 0u, tt, c->stream);
  gsr::launch_fill_u32(s->bin_ticket, 0u, 1, c->stream);
  s->bin_cap = nm;
  s->n_cap = nn;
  s->P_cap = PP;
  s->tiles_cap = tt;
  s->views_cap = vv;
  return GSR_OK;
}

int ensure_B(gsr_ctx* c, gsr_state* s, int64_t K) {
  if (s->arenaB && K <= s->K_cap) return GSR_OK;
  if (s->arenaB) GSR_HIP(c, hipFree(s->arenaB));
  s->arenaB = nullptr;
  const int64_t kk = std::max<int64_t>(K + K / 4, 4096);
  size_t bytes = 0;
  carve_B(s, nullptr, kk, &bytes);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, GSR_ENOMEM, "device allocation of the tile-list workspace failed");
  }
  s->arenaB = p;
  carve_B(s, (char*)p, kk, &bytes);
  s->K_cap = kk;
  return GSR_OK;
}

// Arena D of a deterministic backward: sized for the state's current overlap
// count and records (allocation synchronises the device).
int ensure_D(gsr_ctx* c, gsr_state* s) {
  const int64_t n_rec = s->n * s->n_views, K = s->K;
  if (s->arenaD && K <= s->det_K_cap && n_rec <= s->det_n_cap) return GSR_OK;
  if (s->arenaD) GSR_HIP(c, hipFree(s->arenaD));
  s->arenaD = nullptr;
  const int64_t kk = std::max<int64_t>(K + K / 4, 4096), nn = std::max<int64_t>(n_rec + n_rec / 4, 1024);
  Carver cv{nullptr};
  for (int pass = 0; pass < 2; ++pass) {
    s->det_goff = cv.take<uint32_t>(nn);
    s->det_total = cv.take<uint32_t>(1);
    s->det_scan = cv.take<uint32_t>(gsr::scan_temp_words(nn));
    s->det_rev = cv.take<uint32_t>(kk);
    s->det_mask = cv.take<uint32_t>(kk);
    s->det_part = cv.take<float>(kk * 16 * 10);
    if (pass == 0) {
      void* p = nullptr;
      if (hipMalloc(&p, cv.off) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, GSR_ENOMEM, "device allocation of the deterministic backward's workspace failed");
      }
      s->arenaD = p;
      cv = Carver{(char*)p};
    }
  }
  s->det_K_cap = kk;
  s->det_n_cap = nn;
  return GSR_OK;
}

int make_raster(gsr_ctx* c, const gsr_camera* cam, const gsr_opts* o, gsr::Raster* R) {
  if (!cam || !o) return fail(c, GSR_EINVAL, "camera and opts are required");
  if (cam->width <= 0 || cam->height <= 0) return fail(c, GSR_EINVAL, "image size must be positive");
  if (cam->width > 32768 || cam->height > 32768) return fail(c, GSR_EINVAL, "image sides are limited to 32768");
  const float vals[] = {cam->fx, cam->fy, cam->cx, cam->cy, cam->near_z, cam->bg[0], cam->bg[1], cam->bg[2]};
  for (float v : vals)
    if (!std::isfinite(v)) return fail(c, GSR_EINVAL, "camera intrinsics must be finite");
  if (!(cam->fx > 0) || !(cam->fy > 0)) return fail(c, GSR_EINVAL, "focal lengths must be positive");
  const bool shape_ok = (o->tile_w == 16 && o->tile_h == 16) || (o->tile_w == 8 && o->tile_h == 32) ||
                        (o->tile_w == 32 && o->tile_h == 8);
  if (!shape_ok) return fail(c, GSR_EINVAL, "tile shape must be 16x16, 8x32 or 32x8");
  const float ov[] = {o->lowpass, o->alpha_min, o->alpha_max, o->T_min, o->guard};
  for (float v : ov)
    if (!std::isfinite(v)) return fail(c, GSR_EINVAL, "opts must be finite");
  if (!(o->alpha_min > 0) || !(o->alpha_max >= o->alpha_min) || !(o->alpha_max < 1))
    return fail(c, GSR_EINVAL, "need 0 < alpha_min <= alpha_max < 1");
  gsr::Raster& r = *R;
  r.W = cam->width;
  r.H = cam->height;
  r.tw = o->tile_w;
  r.th = o->tile_h;
  r.tw_log2 = o->tile_w == 8 ? 3 : (o->tile_w == 16 ? 4 : 5);
  r.ntx = (r.W + r.tw - 1) / r.tw;
  r.nty = (r.H + r.th - 1) / r.th;
  r.n_tiles = r.ntx * r.nty;
  r.fx = cam->fx;
  r.fy = cam->fy;
  r.cx = cam->cx;
  r.cy = cam->cy;
  r.near_z = cam->near_z;
  r.lowpass = o->lowpass;
  r.amin = o->alpha_min;
  r.log2_amin = std::log2(o->alpha_min);
  r.amax = o->alpha_max;
  r.tmin = o->T_min;
  r.limx = o->guard * std::max(cam->cx, (float)cam->width - cam->cx) / cam->fx;
  r.limy = o->guard * std::max(cam->cy, (float)cam->height - cam->cy) / cam->fy;
  r.bg0 = cam->bg[0];
  r.bg1 = cam->bg[1];
  r.bg2 = cam->bg[2];
  return GSR_OK;
}

hipEvent_t take_event(gsr_ctx* c) {
  if (!c->spare.empty()) {
    hipEvent_t e = c->spare.back();
    c->spare.pop_back();
    return e;
  }
  // Timing-only events: no system-scope fence, whose L2 writeback and
  // invalidation would otherwise stall the stream at every stage boundary.
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// Records an event pair around one stage when profiling is on.
struct Stage {
  gsr_ctx* c;
  const char* name;
  hipEvent_t a = nullptr;
  Stage(gsr_ctx* ctx, const char* nm) : c(ctx), name(nm) {
    if (c->prof && (c->prof_only.empty() || c->prof_only == nm) && (a = take_event(c)))
      (void)hipEventRecord(a, c->stream);
  }
  ~Stage() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) return;
    (void)hipEventRecord(b, c->stream);
    c->recs.push_back({name, a, b});
  }
};

gsr::BinArgs bin_args(gsr_state* s, int64_t cap, uint32_t* K_host = nullptr) {
  return gsr::BinArgs{s->n,     s->n_views, s->n_wg, s->rect, s->bin_M,    s->bin_T,       s->bin_R,
                      s->bin_ticket, s->d_K, K_host, cap, s->keys, s->d_overflow};
}

// Projection, per-(tile, workgroup) pair counts, the tiles' ranges and the
// overlap count K (in s->d_K, and in *K_host when given).
void enqueue_front(gsr_ctx* c, gsr_state* s, hipStream_t st, uint32_t* K_host = nullptr) {
  gsr::ProjectArgs pa{s->n, s->g.means, s->g.scales, s->g.quats, s->g.opacities, s->g.colors, s->pose7,
                      s->rec_uvab, s->rec_cob, s->rec_rgbz, s->rect, s->counts, s->n_views};
  {
    Stage t(c, "project");
    gsr::launch_project(s->R, pa, st);
  }
  {
    Stage t(c, "bin_count");
    s->n_wg = gsr::bin_workgroups(s->n);
    gsr::launch_bin_count(s->R, bin_args(s, 0, K_host), st);
  }
}

// Tile lists (ranges, slot placement, per-tile depth sort) and compositing.
// cap bounds the overlap positions: the exact K (eager) or the capacity
// (captured graphs, where an overflow is flagged on the device).
void enqueue_back(gsr_ctx* c, gsr_state* s, hipStream_t st, int64_t cap, float* color, float* depth, float* alpha) {
  const gsr::Raster& R = s->R;
  const int n_items = R.n_tiles * s->n_views;
  {
    Stage t(c, "tile_bins");
    gsr::launch_tile_bins(R, bin_args(s, cap), n_items, s->ranges, s->scratch, s->ids, st);
    if (s->blocks > 0) gsr::launch_item_order(s->ranges, n_items, s->order, s->order_temp, st);
  }
  gsr::FwdArgs fa{s->ranges, s->ids, s->rec_uvab, s->rec_cob, s->rec_rgbz,
                  color, depth, alpha, s->Tfin, s->last, nullptr,
                  n_items, s->queue, s->blocks > 0 ? s->order : nullptr, s->blocks};
  {
    Stage t(c, "render_fwd");
    gsr::launch_render_fwd(R, fa, st);
  }
}

// Backward of the compositing and the projection. grads may be NULL (pose only).
void enqueue_bwd(gsr_ctx* c, gsr_state* s, hipStream_t st, const float* gC, const float* gD, const float* gA,
                 const gsr_grads* grads, float* dpose7, float* dtwist6, const gsr::AdamFused* adam = nullptr,
                 const gsr::PoseAdam* pose_adam = nullptr) {
  const gsr::Raster& R = s->R;
  const bool want_pose = dpose7 || dtwist6 || pose_adam;
  const int n_items = R.n_tiles * s->n_views;
  // s->g2d is zero here: cleared when allocated, and each projection backward
  // clears the sums it reads
  const bool geom_only = !adam && (!grads || (!grads->opacities && !grads->colors));
  gsr::BwdArgs ba{s->ranges, s->ids, s->rec_uvab, s->rec_cob, s->rec_rgbz, s->Tfin, s->last,
                  gC, gD, gA, s->g2d, geom_only, n_items, s->queue, s->blocks > 0 ? s->order : nullptr, s->blocks,
                  nullptr, nullptr};
  if (s->det) {
    // arena D is in place (ensure_D): list positions of every (record, tile),
    // then the stored quadrant sums, then their fixed-order totals
    const int64_t n_rec = s->n * s->n_views;
    Stage t(c, "render_bwd");
    gsr::launch_exclusive_scan(s->counts, s->det_goff, n_rec, s->det_total, s->det_scan, st);
    gsr::launch_det_rev(R, s->ranges, s->ids, s->rect, s->det_goff, s->det_rev, n_items, st);
    gsr::launch_fill_u32(s->det_mask, 0u, s->K, st);
    ba.part = s->det_part;
    ba.mask = s->det_mask;
    gsr::launch_render_bwd(R, ba, st);
    gsr::launch_det_reduce(s->rect, s->det_goff, s->det_rev, s->det_mask, s->det_part, n_rec, geom_only, s->g2d, st);
  } else {
    Stage t(c, "render_bwd");
    gsr::launch_render_bwd(R, ba, st);
  }
  gsr_grads none{};
  const gsr_grads& G = grads ? *grads : none;
  gsr::ProjectBwdArgs pb{s->n, s->g.means, s->g.scales, s->g.quats, s->g.opacities, s->g.colors, s->pose7,
                         s->counts, s->g2d, G.means, G.scales, G.quats, G.opacities, G.colors,
                         want_pose ? s->pose_acc : nullptr, s->n_views};
  if (adam) pb.adam = *adam;
  {
    Stage t(c, adam ? "project_bwd_adam" : "project_bwd");
    gsr::launch_project_bwd(R, pb, st);
    if (want_pose)
      gsr::launch_pose_finalize(s->pose7, s->pose_acc, gsr::project_bwd_blocks(s->n), dpose7, dtwist6, s->n_views,
                                st, pose_adam);
  }
}

gsr_state* acquire_state(gsr_ctx* c) {
  for (gsr_state* s : c->pool)
    if (!s->in_use) {
      s->in_use = true;
      return s;
    }
  gsr_state* s = new (std::nothrow) gsr_state();
  if (!s) return nullptr;
  s->ctx = c;
  s->in_use = true;
  c->pool.push_back(s);
  return s;
}

}  // namespace

extern "C" {

const char* gsr_strerror(int code) {
  switch (code) {
    case GSR_OK: return "ok";
    case GSR_EINVAL: return "invalid argument";
    case GSR_ENOMEM: return "out of device memory";
    case GSR_EHIP: return "HIP runtime error";
    case GSR_EOVERFLOW: return "fixed-capacity buffer overflow";
    default: return "unknown error";
  }
}

namespace {
// message of the calling thread's last failed context-free call
thread_local std::string t_err;
}  // namespace

const char* gsr_last_error(gsr_ctx* ctx) {
  if (ctx) return ctx->err.c_str();
  return t_err.empty() ? "no context" : t_err.c_str();
}

void gsr_default_opts(gsr_opts* o) {
  if (!o) return;
  o->lowpass = 0.3f;
  o->alpha_min = 1.f / 255.f;
  o->alpha_max = 0.99f;
  o->T_min = 1e-4f;
  o->guard = 1.3f;
  o->tile_w = 16;
  o->tile_h = 16;
  o->deterministic = 0;
}

int gsr_ctx_create(gsr_ctx** out, int device, void* hip_stream) {
  if (!out) return GSR_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return GSR_EINVAL;
  }
  if (hipSetDevice(device) != hipSuccess) return GSR_EHIP;
  gsr_ctx* c = new (std::nothrow) gsr_ctx();
  if (!c) return GSR_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
    c->n_cu = ncu;
  (void)hipGetLastError();
  if (hipHostMalloc((void**)&c->h_K, 64, hipHostMallocDefault) != hipSuccess ||
      hipMalloc((void**)&c->track_temp, sizeof(uint32_t) * gsr::track_temp_words()) != hipSuccess ||
      hipMalloc((void**)&c->red, sizeof(uint32_t) * gsr::reduce_temp_words()) != hipSuccess ||
      hipMalloc((void**)&c->d_stats, 64) != hipSuccess) {
    (void)hipGetLastError();
    if (c->h_K) (void)hipHostFree(c->h_K);
    if (c->track_temp) (void)hipFree(c->track_temp);
    if (c->red) (void)hipFree(c->red);
    if (c->d_stats) (void)hipFree(c->d_stats);
    delete c;
    return GSR_ENOMEM;
  }
  if (hipHostGetDevicePointer((void**)&c->h_K_dev, c->h_K, 0) != hipSuccess || !c->h_K_dev) {
    (void)hipGetLastError();
    gsr_ctx_destroy(c);
    return GSR_EHIP;
  }
  if (hipEventCreateWithFlags(&c->k_ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    gsr_ctx_destroy(c);
    return GSR_EHIP;
  }
  gsr::launch_fill_u32(c->track_temp, 0u, gsr::track_temp_words(), c->stream);
  gsr::launch_fill_u32(c->red, 0u, gsr::reduce_temp_words(), c->stream);
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipGetLastError();
    gsr_ctx_destroy(c);
    return GSR_EHIP;
  }
  *out = c;
  return GSR_OK;
}

int gsr_ctx_destroy(gsr_ctx* c) {
  if (!c) return GSR_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (gsr_state* s : c->pool) {
    if (s->arenaA) (void)hipFree(s->arenaA);
    if (s->arenaB) (void)hipFree(s->arenaB);
    if (s->arenaD) (void)hipFree(s->arenaD);
    delete s;
  }
  if (c->h_K) (void)hipHostFree(c->h_K);
  if (c->track_temp) (void)hipFree(c->track_temp);
  if (c->red) (void)hipFree(c->red);
  if (c->d_stats) (void)hipFree(c->d_stats);
  if (c->k_ev) (void)hipEventDestroy(c->k_ev);
  for (auto& r : c->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : c->spare) (void)hipEventDestroy(e);
  delete c;
  return GSR_OK;
}

int gsr_set_stream(gsr_ctx* c, void* hip_stream) {
  if (!c) return GSR_EINVAL;
  c->stream = (hipStream_t)hip_stream;
  return GSR_OK;
}

int gsr_render_fwd_batch(gsr_ctx* c, const gsr_gaussians* g, int32_t n_views, const gsr_camera* cam,
                         const gsr_opts* opts, int32_t blocks_per_cu, const float* poses7, float* color, float* depth,
                         float* alpha, gsr_state** state) {
  if (!c || !g || !state) return fail(c, GSR_EINVAL, "ctx, gaussians and state are required");
  *state = nullptr;
  if (g->n < 0) return fail(c, GSR_EINVAL, "n must be >= 0");
  if (n_views < 1 || n_views > 1024) return fail(c, GSR_EINVAL, "n_views must be in [1, 1024]");
  if (g->n * n_views >= (int64_t(1) << 31)) return fail(c, GSR_EINVAL, "n * n_views must be < 2^31");
  if (blocks_per_cu < 0 || blocks_per_cu > 64) return fail(c, GSR_EINVAL, "blocks_per_cu must be in [0, 64]");
  if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacities || !g->colors))
    return fail(c, GSR_EINVAL, "Gaussian parameter pointers are required");
  if (g->n > 0 && (reinterpret_cast<uintptr_t>(g->quats) & 15u) != 0)
    return fail(c, GSR_EINVAL, "quats must be 16-byte aligned");
  if (!poses7 || !color || !depth || !alpha) return fail(c, GSR_EINVAL, "poses and the outputs are required");
  gsr::Raster R;
  int rc = make_raster(c, cam, opts, &R);
  if (rc) return rc;
  if ((int64_t)R.n_tiles * n_views >= (int64_t(1) << 31)) return fail(c, GSR_EINVAL, "too many tiles");
  GSR_HIP(c, hipSetDevice(c->device));
  gsr_state* s = acquire_state(c);
  if (!s) return fail(c, GSR_ENOMEM, "host allocation failed");
  const int64_t P = (int64_t)R.W * R.H;
  rc = ensure_A(c, s, g->n * n_views, P * n_views, (int64_t)R.n_tiles * n_views, n_views);
  if (rc) {
    s->in_use = false;
    return rc;
  }
  s->R = R;
  s->n = g->n;
  s->P = P;
  s->g = *g;
  s->pose7 = poses7;
  s->n_views = n_views;
  s->blocks = blocks_per_cu * c->n_cu;
  s->det = opts->deterministic != 0;
  hipStream_t st = c->stream;
  // the scan writes K straight into the pinned host word; the event's
  // system-scope release makes it visible to the host
  enqueue_front(c, s, st, c->h_K_dev);
  GSR_HIP(c, hipEventRecord(c->k_ev, st));
  // With a tile-list workspace from an earlier forward, the second half is
  // queued before the overlap count is known (positions beyond the capacity
  // would be dropped), so the device does not wait for the host; it is redone
  // in the rare case that the count exceeds the capacity.
  const bool speculative = s->arenaB != nullptr && s->K_cap > 0;
  if (speculative) enqueue_back(c, s, st, s->K_cap, color, depth, alpha);
  GSR_HIP(c, hipEventSynchronize(c->k_ev));
  const int64_t K = (int64_t)*static_cast<volatile uint32_t*>(c->h_K);
  s->K = K;
  if (!speculative || K > s->K_cap) {
    if (speculative) GSR_HIP(c, hipStreamSynchronize(st));  // before the workspace is replaced
    rc = ensure_B(c, s, K);
    if (rc) {
      s->in_use = false;
      return rc;
    }
    enqueue_back(c, s, st, K, color, depth, alpha);
  }
  rc = check_launch(c, "gsr_render_fwd kernels");
  if (rc) {
    s->in_use = false;
    return rc;
  }
  *state = s;
  return GSR_OK;
}

int gsr_render_fwd(gsr_ctx* c, const gsr_gaussians* g, const gsr_camera* cam, const gsr_opts* opts,
                   const float* pose7, float* color, float* depth, float* alpha, gsr_state** state) {
  return gsr_render_fwd_batch(c, g, 1, cam, opts, 0, pose7, color, depth, alpha, state);
}

int gsr_render_bwd(gsr_ctx* c, gsr_state* s, const float* dL_dcolor, const float* dL_ddepth, const float* dL_dalpha,
                   const gsr_grads* grads, float* dL_dpose7, float* dL_dtwist6) {
  if (!c || !s || !s->in_use || s->ctx != c) return fail(c, GSR_EINVAL, "invalid state");
  if (!dL_dcolor || !dL_ddepth) return fail(c, GSR_EINVAL, "dL/dcolor and dL/ddepth are required");
  GSR_HIP(c, hipSetDevice(c->device));
  const gsr_grads* G = grads;
  if (G && G->quats && (reinterpret_cast<uintptr_t>(G->quats) & 15u) != 0)
    return fail(c, GSR_EINVAL, "the quaternion gradient must be 16-byte aligned");
  if (s->det) {
    const int rc = ensure_D(c, s);
    if (rc) return rc;
  }
  enqueue_bwd(c, s, c->stream, dL_dcolor, dL_ddepth, dL_dalpha, G, dL_dpose7, dL_dtwist6);
  return check_launch(c, "gsr_render_bwd kernels");
}

int gsr_render_bwd_adam(gsr_ctx* c, gsr_state* s, const float* dL_dcolor, const float* dL_ddepth,
                        const float* dL_dalpha, const gsr_adam5* adam) {
  if (!c || !s || !s->in_use || s->ctx != c) return fail(c, GSR_EINVAL, "invalid state");
  if (!dL_dcolor || !dL_ddepth || !adam) return fail(c, GSR_EINVAL, "dL/dcolor, dL/ddepth and the Adam state are required");
  const float* read[5] = {s->g.means, s->g.scales, s->g.quats, s->g.opacities, s->g.colors};
  gsr::AdamFused A{};
  for (int i = 0; i < 5; ++i) {
    if (adam->params[i] != read[i])
      return fail(c, GSR_EINVAL, "the Adam parameters must be the tensors the forward read");
    if (!adam->exp_avg[i] || !adam->exp_avg_sq[i]) return fail(c, GSR_EINVAL, "Adam moments are required");
    A.p[i] = adam->params[i];
    A.m[i] = adam->exp_avg[i];
    A.v[i] = adam->exp_avg_sq[i];
    A.lr[i] = adam->lr[i];
  }
  if (adam->step < 1) return fail(c, GSR_EINVAL, "the Adam step count is 1-based");
  A.b1 = adam->beta1;
  A.b2 = adam->beta2;
  A.eps = adam->eps;
  A.bc1 = (float)(1.0 - std::pow((double)adam->beta1, (double)adam->step));
  A.bc2 = (float)(1.0 - std::pow((double)adam->beta2, (double)adam->step));
  if (!std::isfinite(adam->scale_reg)) return fail(c, GSR_EINVAL, "scale_reg must be finite");
  A.reg_w = s->g.n > 0 ? (float)((double)adam->scale_reg / (double)s->g.n) : 0.f;
  A.on = true;
  GSR_HIP(c, hipSetDevice(c->device));
  if (s->det) {
    const int rc = ensure_D(c, s);
    if (rc) return rc;
  }
  enqueue_bwd(c, s, c->stream, dL_dcolor, dL_ddepth, dL_dalpha, nullptr, nullptr, nullptr, &A);
  return check_launch(c, "gsr_render_bwd_adam kernels");
}

int gsr_state_release(gsr_ctx* c, gsr_state* s) {
  if (!c || !s || s->ctx != c) return fail(c, GSR_EINVAL, "invalid state");
  s->in_use = false;
  return GSR_OK;
}

int gsr_tile_lists(gsr_ctx* c, const gsr_state* s, int64_t* K, int32_t* ranges, int32_t* ids) {
  if (!c || !s || !s->in_use || s->ctx != c || !K) return fail(c, GSR_EINVAL, "invalid state");
  GSR_HIP(c, hipSetDevice(c->device));
  *K = s->K;
  if (ranges)
    GSR_HIP(c, hipMemcpyAsync(ranges, s->ranges, sizeof(int2) * s->R.n_tiles * s->n_views, hipMemcpyDeviceToDevice,
                              c->stream));
  if (ids && s->K > 0)
    GSR_HIP(c, hipMemcpyAsync(ids, s->ids, sizeof(uint32_t) * s->K, hipMemcpyDeviceToDevice, c->stream));
  GSR_HIP(c, hipStreamSynchronize(c->stream));
  return GSR_OK;
}

int gsr_loss_l1(gsr_ctx* c, const float* color, const float* depth, const float* tgt_color, const float* tgt_depth,
                int64_t P, float w_color, float w_depth, float* loss, float* dL_dcolor, float* dL_ddepth) {
  if (!c) return GSR_EINVAL;
  if (P < 0 || !loss || (P > 0 && (!color || !depth || !tgt_color || !tgt_depth || !dL_dcolor || !dL_ddepth)))
    return fail(c, GSR_EINVAL, "bad loss arguments");
  GSR_HIP(c, hipSetDevice(c->device));
  Stage t(c, "loss_l1");
  gsr::launch_loss_l1(color, depth, tgt_color, tgt_depth, P, w_color, w_depth, loss, dL_dcolor, dL_ddepth, c->red,
                      c->stream);
  return check_launch(c, "gsr_loss_l1");
}

int gsr_seed_candidates(gsr_ctx* c, const gsr_camera* cam, const float* pose7, const float* color,
                        const float* depth, const float* alpha, const float* u, float p_uniform, float p_grad,
                        float grad_thre, float alpha_n, float* points, float* colors, int64_t* n_out) {
  if (!c) return GSR_EINVAL;
  if (!cam || !pose7 || !color || !depth || !u || !points || !colors || !n_out)
    return fail(c, GSR_EINVAL, "bad seeding candidate arguments");
  if (cam->width <= 0 || cam->height <= 0 || cam->width > 65535 || cam->height > 65535 || !std::isfinite(cam->fx) ||
      !std::isfinite(cam->fy) || !std::isfinite(cam->cx) || !std::isfinite(cam->cy) || cam->fx == 0.f ||
      cam->fy == 0.f)
    return fail(c, GSR_EINVAL, "camera: positive size up to 65535 and finite, non-zero focal lengths");
  if (!std::isfinite(p_uniform) || !std::isfinite(p_grad) || !std::isfinite(grad_thre) || !std::isfinite(alpha_n))
    return fail(c, GSR_EINVAL, "seeding probabilities and thresholds must be finite");
  gsr::SeedSample a{color, depth, alpha, u, pose7, cam->width, cam->height, cam->fx, cam->fy, cam->cx, cam->cy,
                    p_uniform, p_grad, grad_thre * grad_thre, alpha_n};
  const int64_t P = (int64_t)cam->width * cam->height;
  GSR_HIP(c, hipSetDevice(c->device));
  uint32_t* temp = nullptr;
  uint32_t* cnt = nullptr;
  GSR_HIP(c, hipMalloc((void**)&temp, sizeof(uint32_t) * gsr::seed_sample_temp_words(P)));
  if (hipHostMalloc((void**)&cnt, sizeof(uint32_t), hipHostMallocMapped) != hipSuccess) {
    (void)hipFree(temp);
    return fail(c, GSR_ENOMEM, "seeding: pinned count");
  }
  uint32_t* cnt_dev = nullptr;
  hipError_t e = hipHostGetDevicePointer((void**)&cnt_dev, cnt, 0);
  if (e == hipSuccess) {
    Stage t(c, "seed_candidates");
    gsr::launch_seed_sample(a, points, colors, temp, cnt_dev, c->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) *n_out = (int64_t)*(volatile uint32_t*)cnt;
  (void)hipFree(temp);
  (void)hipHostFree(cnt);
  if (e != hipSuccess) return fail(c, GSR_EHIP, hipGetErrorString(e));
  return GSR_OK;
}

int gsr_seed_query(gsr_ctx* c, const float* means, int64_t n, const float* points, int64_t m, float rho, float r_max,
                   float* nn_d2, int32_t* keep) {
  if (!c) return GSR_EINVAL;
  if (n < 0 || n > ((int64_t)1 << 27) || m < 0 || m > ((int64_t)1 << 31) || (n > 0 && !means) ||
      (m > 0 && !points) || !std::isfinite(rho) || !std::isfinite(r_max) || !(rho > 0.f) || !(r_max >= rho))
    return fail(c, GSR_EINVAL, "bad seeding query arguments (0 < rho <= r_max, finite)");
  GSR_HIP(c, hipSetDevice(c->device));
  uint32_t* temp = nullptr;
  GSR_HIP(c, hipMalloc((void**)&temp, sizeof(uint32_t) * gsr::seed_temp_words(n)));
  hipError_t e;
  {
    Stage t(c, "seed_grid");
    gsr::launch_seed_grid(means, n, r_max, temp, c->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    Stage t(c, "seed_query");
    gsr::launch_seed_query(n, points, m, rho, r_max, nn_d2, keep, temp, c->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(temp);
  if (e != hipSuccess) return fail(c, GSR_EHIP, hipGetErrorString(e));
  return GSR_OK;
}

int gsr_seed_gaussians(gsr_ctx* c, int64_t m, const float* points, const float* colors, const float* nn_d2,
                       const int32_t* keep, float* const* out, int64_t* n_new) {
  if (!c) return GSR_EINVAL;
  if (m < 0 || m > (int64_t)0x7fffffff || !out || !n_new || (m > 0 && (!points || !colors || !nn_d2 || !keep)))
    return fail(c, GSR_EINVAL, "bad seed_gaussians arguments");
  if (m == 0) {
    *n_new = 0;
    return GSR_OK;
  }
  for (int i = 0; i < 5; ++i)
    if (!out[i]) return fail(c, GSR_EINVAL, "seed_gaussians: all five output arrays are required");
  if ((reinterpret_cast<uintptr_t>(out[2]) & 15u) != 0)
    return fail(c, GSR_EINVAL, "seed_gaussians: the quaternion output must be 16-byte aligned");
  GSR_HIP(c, hipSetDevice(c->device));
  uint32_t* temp = nullptr;
  uint32_t* cnt = nullptr;
  GSR_HIP(c, hipMalloc((void**)&temp, sizeof(uint32_t) * gsr::seed_init_temp_words(m)));
  if (hipHostMalloc((void**)&cnt, sizeof(uint32_t), hipHostMallocMapped) != hipSuccess) {
    (void)hipFree(temp);
    return fail(c, GSR_ENOMEM, "seed_gaussians: pinned count");
  }
  uint32_t* cnt_dev = nullptr;
  hipError_t e = hipHostGetDevicePointer((void**)&cnt_dev, cnt, 0);
  if (e == hipSuccess) {
    Stage t(c, "seed_gaussians");
    const gsr::SeedInit a{m, points, colors, nn_d2, keep, out[0], out[1], out[2], out[3], out[4]};
    gsr::launch_seed_init(a, temp, cnt_dev, c->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) *n_new = (int64_t)*(volatile uint32_t*)cnt;
  (void)hipFree(temp);
  (void)hipHostFree(cnt);
  if (e != hipSuccess) return fail(c, GSR_EHIP, hipGetErrorString(e));
  return GSR_OK;
}

namespace {
// Shared body of gsr_prune and gsr_compact: stable compaction of the Gaussians
// kept by mask (if given) or by opacity >= o_thre.
int compact_impl(gsr_ctx* c, int64_t n, float o_thre, const int32_t* mask, const float* const* in, float* const* out,
                 int64_t* n_kept, const char* stage) {
  if (n < 0 || n > (int64_t)0x7fffffff || !in || !out || !n_kept || (!mask && std::isnan(o_thre)))
    return fail(c, GSR_EINVAL, "bad prune / compact arguments");
  gsr::PruneArgs a{};
  for (int t = 0; t < 15; ++t) {
    if ((in[t] == nullptr) != (out[t] == nullptr))
      return fail(c, GSR_EINVAL, "prune: in[t] and out[t] must both be set or both be NULL");
    if (t < 5 && n > 0 && !in[t]) return fail(c, GSR_EINVAL, "prune: the five parameter tensors are required");
    a.in[t] = in[t];
    a.out[t] = out[t];
  }
  GSR_HIP(c, hipSetDevice(c->device));
  uint32_t* temp = nullptr;
  uint32_t* kept = nullptr;
  GSR_HIP(c, hipMalloc((void**)&temp, sizeof(uint32_t) * gsr::prune_temp_words(n)));
  if (hipHostMalloc((void**)&kept, sizeof(uint32_t), hipHostMallocMapped) != hipSuccess) {
    (void)hipFree(temp);
    return fail(c, GSR_ENOMEM, "prune: pinned count");
  }
  uint32_t* kept_dev = nullptr;
  hipError_t e = hipHostGetDevicePointer((void**)&kept_dev, kept, 0);
  if (e == hipSuccess) {
    Stage t(c, stage);
    gsr::launch_prune(a, n, o_thre, mask, temp, kept_dev, c->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) *n_kept = (int64_t)*(volatile uint32_t*)kept;
  (void)hipFree(temp);
  (void)hipHostFree(kept);
  if (e != hipSuccess) return fail(c, GSR_EHIP, hipGetErrorString(e));
  return GSR_OK;
}
}  // namespace

int gsr_prune(gsr_ctx* c, int64_t n, float o_thre, const float* const* in, float* const* out, int64_t* n_kept) {
  if (!c) return GSR_EINVAL;
  if (std::isnan(o_thre)) return fail(c, GSR_EINVAL, "prune: o_thre is NaN");
  return compact_impl(c, n, o_thre, nullptr, in, out, n_kept, "prune");
}

int gsr_compact(gsr_ctx* c, int64_t n, const int32_t* keep, const float* const* in, float* const* out,
                int64_t* n_kept) {
  if (!c) return GSR_EINVAL;
  if (n > 0 && !keep) return fail(c, GSR_EINVAL, "compact: keep mask required");
  return compact_impl(c, n, 0.f, keep ? keep : (const int32_t*)nullptr, in, out, n_kept, "compact");
}

namespace {
// Copies the five parameter arrays of n Gaussians between device arrays and
// one host buffer [means 3n | scales 3n | quats 4n | opacities n | colors 3n].
int submap_copy(gsr_ctx* c, int64_t n, const float* const* dev_in, float* const* dev_out, const float* host_in,
                float* host_out, const char* what) {
  if (!c) return GSR_EINVAL;
  if (n < 0 || (n > 0 && !(host_in || host_out))) return fail(c, GSR_EINVAL, std::string(what) + ": bad arguments");
  if (n == 0) return GSR_OK;
  static constexpr int kWidth[5] = {3, 3, 4, 1, 3};
  for (int i = 0; i < 5; ++i)
    if ((dev_in && !dev_in[i]) || (dev_out && !dev_out[i]))
      return fail(c, GSR_EINVAL, std::string(what) + ": all five parameter arrays are required");
  GSR_HIP(c, hipSetDevice(c->device));
  int64_t off = 0;
  for (int i = 0; i < 5; ++i) {
    const size_t bytes = sizeof(float) * (size_t)(kWidth[i] * n);
    if (dev_in)
      GSR_HIP(c, hipMemcpyAsync(host_out + off, dev_in[i], bytes, hipMemcpyDeviceToHost, c->stream));
    else
      GSR_HIP(c, hipMemcpyAsync(dev_out[i], host_in + off, bytes, hipMemcpyHostToDevice, c->stream));
    off += kWidth[i] * n;
  }
  return GSR_OK;
}
}  // namespace

int gsr_submap_offload(gsr_ctx* c, int64_t n, const float* const* in, float* host) {
  if (!in) return fail(c, GSR_EINVAL, "submap offload: parameter arrays required");
  return submap_copy(c, n, in, nullptr, nullptr, host, "submap offload");
}

int gsr_submap_restore(gsr_ctx* c, int64_t n, const float* host, float* const* out) {
  if (!out) return fail(c, GSR_EINVAL, "submap restore: parameter arrays required");
  return submap_copy(c, n, nullptr, out, host, nullptr, "submap restore");
}

int gsr_submap_trigger(const float* pose_first7, const float* pose_cur7, float d_thre, float theta_thre,
                       int32_t* start_new) {
  if (!pose_first7 || !pose_cur7 || !start_new || !std::isfinite(d_thre) || !std::isfinite(theta_thre))
    return GSR_EINVAL;
  // camera centres c = -R^T t of the world-to-camera poses; relative rotation angle 2 acos |<q_a, q_b>|
  double qa[4], qb[4], na = 0, nb = 0;
  for (int i = 0; i < 4; ++i) {
    qa[i] = pose_first7[i];
    qb[i] = pose_cur7[i];
    na += qa[i] * qa[i];
    nb += qb[i] * qb[i];
  }
  if (!(na > 0) || !(nb > 0)) return GSR_EINVAL;
  na = std::sqrt(na);
  nb = std::sqrt(nb);
  double dot = 0;
  for (int i = 0; i < 4; ++i) {
    qa[i] /= na;
    qb[i] /= nb;
    dot += qa[i] * qb[i];
  }
  auto centre = [](const double* q, const float* p7, double* cpos) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z),     2 * (x * z + w * y),
                         2 * (x * y + w * z),     1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                         2 * (x * z - w * y),     2 * (y * z + w * x),     1 - 2 * (x * x + y * y)};
    for (int j = 0; j < 3; ++j) cpos[j] = -(R[j] * p7[4] + R[3 + j] * p7[5] + R[6 + j] * p7[6]);
  };
  double ca[3], cb[3];
  centre(qa, pose_first7, ca);
  centre(qb, pose_cur7, cb);
  const double d = std::sqrt((ca[0] - cb[0]) * (ca[0] - cb[0]) + (ca[1] - cb[1]) * (ca[1] - cb[1]) +
                             (ca[2] - cb[2]) * (ca[2] - cb[2]));
  const double angle = 2.0 * std::acos(std::min(1.0, std::fabs(dot)));
  *start_new = (d > d_thre || angle > theta_thre) ? 1 : 0;
  return GSR_OK;
}

int gsr_loss_reg(gsr_ctx* c, const float* scales, int64_t n, float weight, float* loss, float* dL_dscales) {
  if (!c) return GSR_EINVAL;
  if (n < 0 || !loss || !std::isfinite(weight) || (n > 0 && !scales))
    return fail(c, GSR_EINVAL, "bad regulariser arguments");
  GSR_HIP(c, hipSetDevice(c->device));
  Stage t(c, "loss_reg");
  gsr::launch_loss_reg(scales, n, weight, loss, dL_dscales, c->red, c->stream);
  return check_launch(c, "gsr_loss_reg");
}

int gsr_loss_ssim(gsr_ctx* c, const float* color, const float* tgt_color, int32_t width, int32_t height, float weight,
                  float* loss, float* dL_dcolor) {
  if (!c) return GSR_EINVAL;
  if (width < 0 || height < 0 || width > 65535 || height > 65535 || !loss || !std::isfinite(weight) ||
      ((int64_t)width * height > 0 && (!color || !tgt_color || !dL_dcolor)))
    return fail(c, GSR_EINVAL, "bad SSIM loss arguments");
  GSR_HIP(c, hipSetDevice(c->device));
  Stage t(c, "loss_ssim");
  gsr::launch_loss_ssim(color, tgt_color, height, width, weight, loss, dL_dcolor, c->red, c->stream);
  return check_launch(c, "gsr_loss_ssim");
}

int gsr_loss_track(gsr_ctx* c, const float* color, const float* depth, const float* alpha, const float* tgt_color,
                   const float* tgt_depth, int64_t P, float lambda_c, float inlier_mult, float* loss, float* dL_dcolor,
                   float* dL_ddepth, float* median) {
  if (!c) return GSR_EINVAL;
  if (P < 0 || !loss ||
      (P > 0 && (!color || !depth || !alpha || !tgt_color || !tgt_depth || !dL_dcolor || !dL_ddepth)))
    return fail(c, GSR_EINVAL, "bad loss arguments");
  GSR_HIP(c, hipSetDevice(c->device));
  Stage t(c, "loss_track");
  gsr::launch_loss_track(color, depth, alpha, tgt_color, tgt_depth, P, lambda_c, inlier_mult, loss, dL_dcolor,
                         dL_ddepth, median, c->track_temp, c->stream);
  return check_launch(c, "gsr_loss_track");
}

// ---- tracking loss without allocation ---------------------------------------
// The radix-select histograms, the grid-reduction partials and tickets of
// gsr_loss_track_noalloc live in this file-scope device array (one copy per
// device, held until the process ends). Host code never passes `scratch`
// itself to a kernel: that name is a host-side stand-in. Its device address
// is looked up once per device with hipGetSymbolAddress, with that device
// current, and that address is what the kernels get.
namespace {
constexpr int64_t kNoAllocScratchWords = 8192;  // 32 KiB
__device__ __align__(256) uint32_t scratch[kNoAllocScratchWords];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_dev[kMaxDevices] = {};

int noalloc_fail(int code, const std::string& msg) {
  t_err = msg;
  return code;
}

// Device address of `scratch` on the current device (looked up on the first
// call there); NULL with t_err set on failure.
uint32_t* noalloc_scratch(int* code) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    *code = noalloc_fail(GSR_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      *code = noalloc_fail(GSR_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_dev[dev] = static_cast<uint32_t*>(ptr);
  }
  return g_scratch_dev[dev];
}
}  // namespace

int gsr_loss_track_noalloc(void* hip_stream, const float* color, const float* depth, const float* alpha,
                           const float* tgt_color, const float* tgt_depth, int64_t P, float lambda_c,
                           float inlier_mult, float* loss, float* dL_dcolor, float* dL_ddepth, float* median) {
  if (P < 0 || !loss ||
      (P > 0 && (!color || !depth || !alpha || !tgt_color || !tgt_depth || !dL_dcolor || !dL_ddepth)))
    return noalloc_fail(GSR_EINVAL, "gsr_loss_track_noalloc: bad loss arguments");
  if (P > (int64_t)GSR_NOALLOC_MAX_PIXELS)
    return noalloc_fail(GSR_EINVAL, "gsr_loss_track_noalloc: more than GSR_NOALLOC_MAX_PIXELS pixels "
                                    "(the median's histogram counts are 32-bit)");
  const int64_t words = gsr::track_temp_words();
  if (words > kNoAllocScratchWords)
    return noalloc_fail(GSR_EINVAL, "gsr_loss_track_noalloc: the loss needs more scratch than the static array holds");
  int code = GSR_OK;
  uint32_t* temp = noalloc_scratch(&code);
  if (!temp) return code;
  hipStream_t s = (hipStream_t)hip_stream;
  // the previous call (on any stream) leaves its histograms and tickets behind:
  // clear them with a fill kernel (no memset node, so the call can be captured)
  gsr::launch_fill_u32(temp, 0u, words, s);
  gsr::launch_loss_track(color, depth, alpha, tgt_color, tgt_depth, P, lambda_c, inlier_mult, loss, dL_dcolor,
                         dL_ddepth, median, temp, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return noalloc_fail(GSR_EHIP, std::string("gsr_loss_track_noalloc: ") + hipGetErrorString(e));
  return GSR_OK;
}

int gsr_adam(gsr_ctx* c, float* param, float* m, float* v, const float* grad, int64_t n, int64_t step, float lr,
             float b1, float b2, float eps) {
  if (!c) return GSR_EINVAL;
  if (n < 0 || step < 1 || (n > 0 && (!param || !m || !v || !grad))) return fail(c, GSR_EINVAL, "bad Adam arguments");
  GSR_HIP(c, hipSetDevice(c->device));
  const float bc1 = (float)(1.0 - std::pow((double)b1, (double)step));
  const float bc2 = (float)(1.0 - std::pow((double)b2, (double)step));
  Stage t(c, "adam");
  gsr::launch_adam(param, m, v, grad, n, lr, b1, b2, eps, bc1, bc2, c->stream);
  return check_launch(c, "gsr_adam");
}

int gsr_autotune_batch(gsr_ctx* c, const gsr_gaussians* g, int32_t n_views, const gsr_camera* cam, gsr_opts* opts,
                       const float* poses7, const float* dL_dcolor, const float* dL_ddepth, int32_t reps,
                       int32_t* best_blocks_per_cu, float* ms_table) {
  if (!c || !g || !cam || !opts || !poses7 || !dL_dcolor || !dL_ddepth || !best_blocks_per_cu)
    return fail(c, GSR_EINVAL, "bad autotune arguments");
  if (reps < 1 || reps > 1000) return fail(c, GSR_EINVAL, "reps must be in [1, 1000]");
  if (n_views < 1 || n_views > 1024) return fail(c, GSR_EINVAL, "n_views must be in [1, 1024]");
  GSR_HIP(c, hipSetDevice(c->device));
  const int64_t P = (int64_t)cam->width * cam->height;
  if (P <= 0) return fail(c, GSR_EINVAL, "image size must be positive");
  // images, and the parameter gradients a mapping backward writes (the
  // configuration is timed on the backward it will run)
  const int64_t n = g->n > 0 ? g->n : 0;
  float* buf = nullptr;
  if (hipMalloc((void**)&buf, sizeof(float) * (5 * P * n_views + 14 * n)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, GSR_ENOMEM, "autotune scratch allocation failed");
  }
  gsr_grads grads{};
  grads.quats = buf;  // 16-byte aligned: the start of the allocation
  grads.means = buf + 4 * n;
  grads.scales = grads.means + 3 * n;
  grads.opacities = grads.scales + 3 * n;
  grads.colors = grads.opacities + n;
  float* color = buf + 14 * n;
  float* depth = color + 3 * P * n_views;
  float* alpha = depth + P * n_views;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreateWithFlags(&e0, hipEventDisableSystemFence) != hipSuccess ||
      hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(buf);
    return fail(c, GSR_EHIP, "event creation failed");
  }
  const int shapes[3][2] = {{16, 16}, {8, 32}, {32, 8}};
  const int bpc[5] = {0, 1, 2, 4, 8};
  float best = 1e30f;
  int best_s = 0, best_b = 0, rc = GSR_OK;
  const bool prof = c->prof;
  c->prof = false;
  for (int si = 0; si < 3 && rc == GSR_OK; ++si)
    for (int bi = 0; bi < 5 && rc == GSR_OK; ++bi) {
      gsr_opts o = *opts;
      o.tile_w = shapes[si][0];
      o.tile_h = shapes[si][1];
      float total = 0.f;
      for (int r = 0; r <= reps && rc == GSR_OK; ++r) {  // r == 0 warms up
        gsr_state* st = nullptr;
        (void)hipEventRecord(e0, c->stream);
        rc = gsr_render_fwd_batch(c, g, n_views, cam, &o, bpc[bi], poses7, color, depth, alpha, &st);
        if (rc == GSR_OK) rc = gsr_render_bwd(c, st, dL_dcolor, dL_ddepth, nullptr, &grads, nullptr, nullptr);
        (void)hipEventRecord(e1, c->stream);
        if (st) gsr_state_release(c, st);
        if (rc == GSR_OK && hipEventSynchronize(e1) == hipSuccess && r > 0) {
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          total += ms;
        }
      }
      const float avg = total / reps;
      if (ms_table) ms_table[si * 5 + bi] = avg;
      if (rc == GSR_OK && avg < best) {
        best = avg;
        best_s = si;
        best_b = bi;
      }
    }
  c->prof = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  if (rc != GSR_OK) return rc;
  opts->tile_w = shapes[best_s][0];
  opts->tile_h = shapes[best_s][1];
  *best_blocks_per_cu = bpc[best_b];
  return GSR_OK;
}

// ---------------------------------------------------------------------------
// Tracking-initialisation network
// ---------------------------------------------------------------------------

int gsr_initnet_destroy(gsr_ctx* c, gsr_initnet* net) {
  if (!c || !net || net->ctx != c) return fail(c, GSR_EINVAL, "invalid network");
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (net->buf) (void)hipFree(net->buf);
  delete net;
  return GSR_OK;
}

int gsr_initnet_create(gsr_ctx* c, int32_t max_batch, gsr_initnet** out) {
  if (!c || !out || max_batch < 1 || max_batch > 4096) return fail(c, GSR_EINVAL, "max_batch must be in [1, 4096]");
  *out = nullptr;
  GSR_HIP(c, hipSetDevice(c->device));
  gsr_initnet* net = new (std::nothrow) gsr_initnet();
  if (!net) return fail(c, GSR_ENOMEM, "host allocation failed");
  net->ctx = c;
  net->max_batch = max_batch;
  using N = gsr_initnet;
  net->H[0] = N::kInH;
  net->W[0] = N::kInW;
  net->C[0] = N::kInC;
  for (int l = 1; l <= N::kLayers; ++l) {
    net->H[l] = (net->H[l - 1] + 1) / 2;
    net->W[l] = (net->W[l - 1] + 1) / 2;
    net->C[l] = N::kCh;
  }
  int64_t np = 0;
  for (int l = 0; l < N::kLayers; ++l) np += (int64_t)N::kCh * gsr::conv_kp(net->C[l]) + N::kCh;
  np += 6 * N::kHeadIn + 6;
  net->n_params = np;
  const int64_t B = max_batch;
  size_t bytes = 0;
  auto carve = [&](char* base) {
    Carver cv{base};
    net->params = cv.take<float>(np);
    net->grads = cv.take<float>(np);
    net->m = cv.take<float>(np);
    net->v = cv.take<float>(np);
    for (int l = 0; l < N::kLayers; ++l) {
      net->wk[l] = cv.take<uint16_t>((int64_t)N::kCh * gsr::conv_kp(net->C[l]));
      net->wt[l] = cv.take<uint16_t>((int64_t)net->C[l] * 9 * N::kCh);
    }
    for (int l = 0; l <= N::kLayers; ++l) {
      const int64_t sz = B * net->H[l] * net->W[l] * net->C[l];
      net->act[l] = cv.take<uint16_t>(sz);
      net->dact[l] = cv.take<uint16_t>(sz);
    }
    net->pool = cv.take<float>(B * N::kHeadIn);
    net->out = cv.take<float>(B * 6);
    net->scratch = cv.take<float>(B * 6 + 64);
    bytes = cv.off;
  };
  carve(nullptr);
  if (hipMalloc(&net->buf, bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete net;
    return fail(c, GSR_ENOMEM, "device allocation of the network failed");
  }
  carve((char*)net->buf);
  float* p = net->params;
  float* g = net->grads;
  for (int l = 0; l < N::kLayers; ++l) {
    const int64_t nw = (int64_t)N::kCh * gsr::conv_kp(net->C[l]);
    net->w[l] = p;
    net->dw[l] = g;
    p += nw;
    g += nw;
    net->b[l] = p;
    net->db[l] = g;
    p += N::kCh;
    g += N::kCh;
  }
  net->wfc = p;
  net->dwfc = g;
  net->bfc = p + 6 * N::kHeadIn;
  net->dbfc = g + 6 * N::kHeadIn;
  for (float* q : {net->params, net->grads, net->m, net->v}) gsr::launch_fill_f32(q, 0.f, np, c->stream);
  *out = net;
  return check_launch(c, "gsr_initnet_create");
}

int gsr_initnet_count(gsr_ctx* c, gsr_initnet* net, int64_t* n_params) {
  if (!c || !net || net->ctx != c || !n_params) return fail(c, GSR_EINVAL, "invalid network");
  *n_params = net->n_params;
  return GSR_OK;
}

int gsr_initnet_set_params(gsr_ctx* c, gsr_initnet* net, const float* src) {
  if (!c || !net || net->ctx != c || !src) return fail(c, GSR_EINVAL, "invalid network or source");
  GSR_HIP(c, hipSetDevice(c->device));
  GSR_HIP(c, hipMemcpyAsync(net->params, src, sizeof(float) * net->n_params, hipMemcpyDeviceToDevice, c->stream));
  gsr::launch_fill_f32(net->m, 0.f, net->n_params, c->stream);
  gsr::launch_fill_f32(net->v, 0.f, net->n_params, c->stream);
  net->step = 0;
  return check_launch(c, "gsr_initnet_set_params");
}

int gsr_initnet_get_params(gsr_ctx* c, gsr_initnet* net, float* params, float* grads) {
  if (!c || !net || net->ctx != c) return fail(c, GSR_EINVAL, "invalid network");
  GSR_HIP(c, hipSetDevice(c->device));
  if (params)
    GSR_HIP(c, hipMemcpyAsync(params, net->params, sizeof(float) * net->n_params, hipMemcpyDeviceToDevice, c->stream));
  if (grads)
    GSR_HIP(c, hipMemcpyAsync(grads, net->grads, sizeof(float) * net->n_params, hipMemcpyDeviceToDevice, c->stream));
  return GSR_OK;
}

int gsr_initnet_set_input(gsr_ctx* c, gsr_initnet* net, int32_t batch, const uint16_t* src) {
  if (!c || !net || net->ctx != c || !src || batch < 1 || batch > net->max_batch)
    return fail(c, GSR_EINVAL, "bad input arguments");
  GSR_HIP(c, hipSetDevice(c->device));
  const int64_t n = (int64_t)batch * gsr_initnet::kInH * gsr_initnet::kInW * gsr_initnet::kInC;
  GSR_HIP(c, hipMemcpyAsync(net->act[0], src, sizeof(uint16_t) * n, hipMemcpyDeviceToDevice, c->stream));
  return GSR_OK;
}

int gsr_initnet_get_activation(gsr_ctx* c, gsr_initnet* net, int32_t layer, int32_t batch, uint16_t* act,
                               uint16_t* dact) {
  if (!c || !net || net->ctx != c || layer < 0 || layer > gsr_initnet::kLayers || batch < 1 || batch > net->max_batch)
    return fail(c, GSR_EINVAL, "bad activation arguments");
  GSR_HIP(c, hipSetDevice(c->device));
  const int64_t n = (int64_t)batch * net->H[layer] * net->W[layer] * net->C[layer];
  if (act) GSR_HIP(c, hipMemcpyAsync(act, net->act[layer], 2 * n, hipMemcpyDeviceToDevice, c->stream));
  if (dact) GSR_HIP(c, hipMemcpyAsync(dact, net->dact[layer], 2 * n, hipMemcpyDeviceToDevice, c->stream));
  return GSR_OK;
}

int gsr_pack_rgbd_pair(gsr_ctx* c, const float* rend_color, const float* rend_depth, const float* obs_color,
                       const float* obs_depth, int32_t H, int32_t W, float depth_scale, uint16_t* dst) {
  if (!c || !rend_color || !rend_depth || !obs_color || !obs_depth || !dst) return fail(c, GSR_EINVAL, "bad arguments");
  const int f = W / gsr_initnet::kInW;
  if (f < 1 || W != f * gsr_initnet::kInW || H != f * gsr_initnet::kInH)
    return fail(c, GSR_EINVAL, "frames must be an integer multiple of 160 x 120");
  GSR_HIP(c, hipSetDevice(c->device));
  gsr::launch_pack_input(rend_color, rend_depth, obs_color, obs_depth, H, W, f, depth_scale, dst, c->stream);
  return check_launch(c, "gsr_pack_rgbd_pair");
}

int gsr_initnet_forward(gsr_ctx* c, gsr_initnet* net, int32_t batch, float* out) {
  if (!c || !net || net->ctx != c || batch < 1 || batch > net->max_batch)
    return fail(c, GSR_EINVAL, "bad forward arguments");
  GSR_HIP(c, hipSetDevice(c->device));
  hipStream_t st = c->stream;
  Stage t(c, "initnet_fwd");
  for (int l = 0; l < gsr_initnet::kLayers; ++l) {
    gsr::launch_cast_weights(net->w[l], net->C[l], net->wk[l], net->wt[l], st);
    gsr::launch_conv_fwd(batch, net->H[l], net->W[l], net->C[l], net->act[l], net->wk[l], net->b[l], net->act[l + 1],
                         st);
  }
  const int L = gsr_initnet::kLayers;
  gsr::launch_head_fwd(batch, net->H[L], net->W[L], net->act[L], net->wfc, net->bfc, net->pool, net->out, st);
  if (out) GSR_HIP(c, hipMemcpyAsync(out, net->out, sizeof(float) * 6 * batch, hipMemcpyDeviceToDevice, st));
  return check_launch(c, "gsr_initnet_forward");
}

int gsr_initnet_backward(gsr_ctx* c, gsr_initnet* net, int32_t batch, const float* labels, const float* scale,
                         const float* dL_dout, float* loss) {
  if (!c || !net || net->ctx != c || batch < 1 || batch > net->max_batch)
    return fail(c, GSR_EINVAL, "bad backward arguments");
  if (!dL_dout && (!labels || !scale)) return fail(c, GSR_EINVAL, "labels and scale (or dL/dout) are required");
  GSR_HIP(c, hipSetDevice(c->device));
  hipStream_t st = c->stream;
  Stage t(c, "initnet_bwd");
  const int L = gsr_initnet::kLayers;
  gsr::launch_fill_f32(net->grads, 0.f, net->n_params, st);
  float* lp = loss ? loss : net->scratch;
  gsr::launch_fill_f32(lp, 0.f, 1, st);
  gsr::launch_head_bwd(batch, net->H[L], net->W[L], net->out, labels, scale, net->pool, net->wfc, net->act[L], dL_dout,
                       net->dwfc, net->dbfc, net->dact[L], lp, st);
  for (int l = L - 1; l >= 0; --l) {
    // dact[l + 1] holds dL/d(pre-activation of layer l)
    gsr::launch_conv_bwd_weight(batch, net->H[l], net->W[l], net->C[l], net->dact[l + 1], net->act[l], net->dw[l],
                                net->db[l], st);
    if (l > 0)
      gsr::launch_conv_bwd_data(batch, net->H[l], net->W[l], net->C[l], net->dact[l + 1], net->wt[l], net->act[l],
                                net->dact[l], st);
  }
  return check_launch(c, "gsr_initnet_backward");
}

int gsr_initnet_adam(gsr_ctx* c, gsr_initnet* net, float lr, float b1, float b2, float eps) {
  if (!c || !net || net->ctx != c) return fail(c, GSR_EINVAL, "invalid network");
  GSR_HIP(c, hipSetDevice(c->device));
  net->step += 1;
  const float bc1 = (float)(1.0 - std::pow((double)b1, (double)net->step));
  const float bc2 = (float)(1.0 - std::pow((double)b2, (double)net->step));
  gsr::launch_adam(net->params, net->m, net->v, net->grads, net->n_params, lr, b1, b2, eps, bc1, bc2, c->stream);
  return check_launch(c, "gsr_initnet_adam");
}

int gsr_profile_enable(gsr_ctx* c, int on) {
  if (!c) return GSR_EINVAL;
  c->prof = on != 0;
  return GSR_OK;
}

int gsr_profile_only(gsr_ctx* c, const char* stage) {
  if (!c) return GSR_EINVAL;
  if (stage && std::strlen(stage) >= 32) return fail(c, GSR_EINVAL, "stage name too long");
  c->prof_only = stage ? stage : "";
  return GSR_OK;
}

int gsr_profile_read(gsr_ctx* c, int max_stages, char* names, double* total_ms, int64_t* counts, int* n_stages) {
  if (!c || !n_stages || (max_stages > 0 && (!names || !total_ms || !counts)))
    return fail(c, GSR_EINVAL, "bad profile arguments");
  GSR_HIP(c, hipSetDevice(c->device));
  GSR_HIP(c, hipStreamSynchronize(c->stream));
  std::vector<std::string> nm;
  std::vector<double> ms;
  std::vector<int64_t> cnt;
  for (auto& r : c->recs) {
    float t = 0.f;
    (void)hipEventElapsedTime(&t, r.a, r.b);
    size_t i = 0;
    while (i < nm.size() && nm[i] != r.name) ++i;
    if (i == nm.size()) {
      nm.push_back(r.name);
      ms.push_back(0.0);
      cnt.push_back(0);
    }
    ms[i] += t;
    cnt[i] += 1;
    c->spare.push_back(r.a);
    c->spare.push_back(r.b);
  }
  c->recs.clear();
  *n_stages = (int)nm.size();
  for (int i = 0; i < (int)nm.size() && i < max_stages; ++i) {
    std::memset(names + 32 * i, 0, 32);
    std::strncpy(names + 32 * i, nm[i].c_str(), 31);
    total_ms[i] = ms[i];
    counts[i] = cnt[i];
  }
  return GSR_OK;
}

int gsr_state_stats(gsr_ctx* c, gsr_state* s, int64_t out[6]) {
  if (!c || !s || !s->in_use || s->ctx != c || !out) return fail(c, GSR_EINVAL, "invalid state");
  GSR_HIP(c, hipSetDevice(c->device));
  hipStream_t st = c->stream;
  GSR_HIP(c, hipMemsetAsync(c->d_stats, 0, 64, st));
  gsr::FwdArgs fa{s->ranges, s->ids, s->rec_uvab, s->rec_cob, s->rec_rgbz,
                  nullptr, nullptr, nullptr, nullptr, s->last, c->d_stats,
                  s->R.n_tiles * s->n_views, nullptr, nullptr, 0};
  gsr::launch_render_fwd(s->R, fa, st);
  unsigned long long h[3] = {0, 0, 0};
  GSR_HIP(c, hipMemcpyAsync(h, c->d_stats, sizeof(h), hipMemcpyDeviceToHost, st));
  const int64_t m = s->n * s->n_views;
  std::vector<uint32_t> counts((size_t)std::max<int64_t>(m, 1));
  if (m > 0) GSR_HIP(c, hipMemcpyAsync(counts.data(), s->counts, 4 * m, hipMemcpyDeviceToHost, st));
  GSR_HIP(c, hipStreamSynchronize(st));
  int64_t vis = 0;
  for (int64_t i = 0; i < m; ++i) vis += counts[i] > 0;
  out[0] = s->K;
  out[1] = vis;
  out[2] = (int64_t)h[0];
  out[3] = (int64_t)h[1];
  out[4] = (int64_t)h[2];
  out[5] = (int64_t)s->R.n_tiles * s->n_views;
  return check_launch(c, "gsr_state_stats");
}

int gsr_adam_groups(gsr_ctx* c, int32_t n_groups, float* const* params, float* const* exp_avg,
                    float* const* exp_avg_sq, const float* const* grads, const int64_t* counts, const float* lrs,
                    int64_t step, float b1, float b2, float eps) {
  if (!c) return GSR_EINVAL;
  if (n_groups < 1 || n_groups > gsr::kAdamGroups || !params || !exp_avg || !exp_avg_sq || !grads || !counts || !lrs ||
      step < 1)
    return fail(c, GSR_EINVAL, "bad Adam group arguments");
  gsr::AdamGroups a{};
  a.n = n_groups;
  a.off[0] = 0;
  for (int i = 0; i < n_groups; ++i) {
    if (counts[i] < 0 || (counts[i] > 0 && (!params[i] || !exp_avg[i] || !exp_avg_sq[i] || !grads[i])))
      return fail(c, GSR_EINVAL, "bad Adam group");
    a.p[i] = params[i];
    a.m[i] = exp_avg[i];
    a.v[i] = exp_avg_sq[i];
    a.g[i] = grads[i];
    a.lr[i] = lrs[i];
    a.off[i + 1] = a.off[i] + counts[i];
  }
  GSR_HIP(c, hipSetDevice(c->device));
  const float bc1 = (float)(1.0 - std::pow((double)b1, (double)step));
  const float bc2 = (float)(1.0 - std::pow((double)b2, (double)step));
  Stage t(c, "adam");
  gsr::launch_adam_multi(a, b1, b2, eps, bc1, bc2, c->stream);
  return check_launch(c, "gsr_adam_groups");
}

int gsr_pose_adam(gsr_ctx* c, float* pose7, float* state, const float* grad7, float lr_q, float lr_t, float b1,
                  float b2, float eps) {
  if (!c || !pose7 || !state || !grad7) return fail(c, GSR_EINVAL, "pose, state and gradient are required");
  GSR_HIP(c, hipSetDevice(c->device));
  Stage t(c, "pose_adam");
  gsr::launch_pose_adam(pose7, state, grad7, lr_q, lr_t, b1, b2, eps, c->stream);
  return check_launch(c, "gsr_pose_adam");
}

int gsr_pose_apply_twist(gsr_ctx* c, const float* pose7, const float* twist6, float* out) {
  if (!c || !pose7 || !twist6 || !out) return fail(c, GSR_EINVAL, "pose, twist and output are required");
  GSR_HIP(c, hipSetDevice(c->device));
  gsr::launch_pose_apply_twist(pose7, twist6, out, c->stream);
  return check_launch(c, "gsr_pose_apply_twist");
}

int gsr_pose_const_velocity(gsr_ctx* c, const float* p0, const float* p1, float* out) {
  if (!c || !p0 || !p1 || !out) return fail(c, GSR_EINVAL, "pose pointers are required");
  GSR_HIP(c, hipSetDevice(c->device));
  gsr::launch_pose_const_velocity(p0, p1, out, c->stream);
  return check_launch(c, "gsr_pose_const_velocity");
}

int gsr_track_graph_destroy(gsr_ctx* c, gsr_track_graph* tg) {
  if (!c || !tg || tg->ctx != c) return fail(c, GSR_EINVAL, "invalid tracking graph");
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (tg->exec) (void)hipGraphExecDestroy(tg->exec);
  if (tg->graph) (void)hipGraphDestroy(tg->graph);
  if (tg->buf) (void)hipFree(tg->buf);
  if (tg->h_flag) (void)hipHostFree(tg->h_flag);
  if (tg->s) {
    if (tg->s->arenaA) (void)hipFree(tg->s->arenaA);
    if (tg->s->arenaB) (void)hipFree(tg->s->arenaB);
    delete tg->s;
  }
  delete tg;
  return GSR_OK;
}

int gsr_track_graph_set_frame(gsr_ctx* c, gsr_track_graph* tg, const float* obs_color, const float* obs_depth) {
  if (!c || !tg || tg->ctx != c || !obs_color || !obs_depth) return fail(c, GSR_EINVAL, "bad arguments");
  GSR_HIP(c, hipSetDevice(c->device));
  const int64_t P = tg->s->P;
  GSR_HIP(c, hipMemcpyAsync(tg->obs_c, obs_color, sizeof(float) * 3 * P, hipMemcpyDeviceToDevice, c->stream));
  GSR_HIP(c, hipMemcpyAsync(tg->obs_d, obs_depth, sizeof(float) * P, hipMemcpyDeviceToDevice, c->stream));
  return GSR_OK;
}

int gsr_track_graph_create(gsr_ctx* c, const gsr_gaussians* g, const gsr_camera* cam, const gsr_opts* opts,
                           const gsr_track_opts* to, const float* obs_color, const float* obs_depth, int64_t K_cap,
                           gsr_track_graph** out) {
  if (!c || !g || !to || !out || !obs_color || !obs_depth) return fail(c, GSR_EINVAL, "bad arguments");
  *out = nullptr;
  if (g->n <= 0 || g->n >= (int64_t(1) << 31) || !g->means || !g->scales || !g->quats || !g->opacities || !g->colors)
    return fail(c, GSR_EINVAL, "tracking needs a non-empty Gaussian set");
  if ((reinterpret_cast<uintptr_t>(g->quats) & 15u) != 0) return fail(c, GSR_EINVAL, "quats must be 16-byte aligned");
  if (to->n_iters <= 0 || to->n_iters > 100000) return fail(c, GSR_EINVAL, "n_iters must be in [1, 100000]");
  if (K_cap <= 0 || K_cap >= (int64_t(1) << 31)) return fail(c, GSR_EINVAL, "K_cap must be in [1, 2^31)");
  gsr::Raster R;
  int rc = make_raster(c, cam, opts, &R);
  if (rc) return rc;
  if (opts->deterministic) return fail(c, GSR_EINVAL, "the tracking graph has no deterministic backward");
  GSR_HIP(c, hipSetDevice(c->device));
  gsr_track_graph* tg = new (std::nothrow) gsr_track_graph();
  if (!tg) return fail(c, GSR_ENOMEM, "host allocation failed");
  tg->ctx = c;
  tg->n_iters = to->n_iters;
  tg->K_cap = K_cap;
  tg->s = new (std::nothrow) gsr_state();
  if (!tg->s) {
    delete tg;
    return fail(c, GSR_ENOMEM, "host allocation failed");
  }
  gsr_state* s = tg->s;
  s->ctx = c;
  s->in_use = true;
  const int64_t P = (int64_t)R.W * R.H;
  rc = ensure_A(c, s, g->n, P, R.n_tiles, 1);
  if (!rc) rc = ensure_B(c, s, K_cap);
  // graph-owned device buffers
  size_t bytes = 0;
  auto carve = [&](char* base) {
    Carver cv{base};
    tg->pose = cv.take<float>(8);
    tg->adam = cv.take<float>(20);
    tg->dpose = cv.take<float>(8);
    tg->loss = cv.take<float>(tg->n_iters);
    tg->median = cv.take<float>(tg->n_iters);
    tg->color = cv.take<float>(3 * P);
    tg->depth = cv.take<float>(P);
    tg->alpha = cv.take<float>(P);
    tg->gC = cv.take<float>(3 * P);
    tg->gD = cv.take<float>(P);
    tg->obs_c = cv.take<float>(3 * P);
    tg->obs_d = cv.take<float>(P);
    tg->sel_temp = cv.take<uint32_t>(gsr::track_temp_words());
    bytes = cv.off;
  };
  if (!rc) {
    carve(nullptr);
    if (hipMalloc(&tg->buf, bytes) != hipSuccess) {
      (void)hipGetLastError();
      rc = fail(c, GSR_ENOMEM, "device allocation of the tracking buffers failed");
    } else {
      carve((char*)tg->buf);
    }
  }
  if (!rc && hipHostMalloc((void**)&tg->h_flag, 64, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    rc = fail(c, GSR_ENOMEM, "pinned allocation failed");
  }
  if (rc) {
    gsr_track_graph_destroy(c, tg);
    return rc;
  }
  s->R = R;
  s->n = g->n;
  s->P = P;
  s->g = *g;
  s->pose7 = tg->pose;
  s->K = K_cap;
  hipStream_t st = c->stream;
  // every id slot holds an in-range record index from the start
  gsr::launch_fill_u32(s->ids, 0u, K_cap, st);
  gsr::launch_fill_f32(tg->pose, 0.f, 8, st);
  gsr::launch_fill_u32(tg->sel_temp, 0u, gsr::track_temp_words(), st);
  rc = gsr_track_graph_set_frame(c, tg, obs_color, obs_depth);
  if (!rc) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = hip_fail(c, e, "hipStreamSynchronize");
  }
  // capture on a private stream (default priority)
  hipStream_t cap = nullptr;
  if (!rc && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    rc = fail(c, GSR_EHIP, "capture stream creation failed");
  }
  if (!rc) {
    const bool prof = c->prof;
    c->prof = false;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      gsr::launch_fill_f32(tg->adam, 0.f, 20, cap);
      gsr::launch_fill_u32(reinterpret_cast<uint32_t*>(s->d_overflow), 0u, 1, cap);
      const gsr::PoseAdam pa{tg->adam, to->lr_q, to->lr_t, to->beta1, to->beta2, to->eps};
      for (int it = 0; it < tg->n_iters; ++it) {
        enqueue_front(c, s, cap);
        enqueue_back(c, s, cap, K_cap, tg->color, tg->depth, tg->alpha);
        gsr::launch_loss_track(tg->color, tg->depth, tg->alpha, tg->obs_c, tg->obs_d, P, to->lambda_c,
                               to->inlier_mult, tg->loss + it, tg->gC, tg->gD, tg->median + it, tg->sel_temp, cap);
        // the pose backward's last kernel applies the pose Adam step
        enqueue_bwd(c, s, cap, tg->gC, tg->gD, nullptr, nullptr, nullptr, nullptr, nullptr, &pa);
      }
      e = hipStreamEndCapture(cap, &tg->graph);
    }
    c->prof = prof;
    if (e == hipSuccess) e = hipGraphInstantiate(&tg->exec, tg->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = hip_fail(c, e, "tracking graph capture");
    (void)hipStreamDestroy(cap);
  }
  if (rc) {
    gsr_track_graph_destroy(c, tg);
    return rc;
  }
  *out = tg;
  return GSR_OK;
}

int gsr_track_graph_run(gsr_ctx* c, gsr_track_graph* tg, float* pose7, float* losses) {
  if (!c || !tg || tg->ctx != c || !pose7) return fail(c, GSR_EINVAL, "bad arguments");
  GSR_HIP(c, hipSetDevice(c->device));
  hipStream_t st = c->stream;
  Stage t(c, "track_graph");
  GSR_HIP(c, hipMemcpyAsync(tg->pose, pose7, sizeof(float) * 7, hipMemcpyDeviceToDevice, st));
  GSR_HIP(c, hipGraphLaunch(tg->exec, st));
  GSR_HIP(c, hipMemcpyAsync(pose7, tg->pose, sizeof(float) * 7, hipMemcpyDeviceToDevice, st));
  if (losses)
    GSR_HIP(c, hipMemcpyAsync(losses, tg->loss, sizeof(float) * tg->n_iters, hipMemcpyDeviceToDevice, st));
  GSR_HIP(c, hipMemcpyAsync(tg->h_flag, tg->s->d_overflow, sizeof(int), hipMemcpyDeviceToHost, st));
  GSR_HIP(c, hipStreamSynchronize(st));
  if (*tg->h_flag) return fail(c, GSR_EOVERFLOW, "tile-overlap capacity exceeded inside the tracking graph");
  return GSR_OK;
}

}  // extern "C"
