// C ABI of libgsr (declared in include/gsr.h): argument checking, workspace
// management and the launch sequence of each call. No compute happens here;
// every step of the hot path is one of the kernels in k_*.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
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
  int64_t n_cap = -1, P_cap = -1, tiles_cap = -1, K_cap = -1;
  void* arenaA = nullptr;
  void* arenaB = nullptr;
  // arena A: per Gaussian / pixel / tile
  float4* rec_uvab = nullptr;
  float4* rec_cob = nullptr;
  float4* rec_rgbz = nullptr;
  int4* rect = nullptr;
  uint32_t* counts = nullptr;
  uint32_t* offsets = nullptr;
  uint32_t* scan_temp = nullptr;
  float* g2d = nullptr;
  float* Tfin = nullptr;
  int* last = nullptr;
  int2* ranges = nullptr;
  uint32_t* d_K = nullptr;
  int* d_overflow = nullptr;
  float* pose_acc = nullptr;
  // arena B: per overlap
  uint64_t* keys[2] = {nullptr, nullptr};
  uint32_t* vals[2] = {nullptr, nullptr};
  uint32_t* sort_temp = nullptr;
  int sorted = 0;
};

struct gsr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<gsr_state*> pool;
  uint32_t* h_K = nullptr;  // pinned host word for the overlap count
  uint32_t* track_temp = nullptr;
  unsigned long long* d_stats = nullptr;
  // stage timing (gsr_profile_*): an event pair around each stage launch
  struct Rec {
    const char* name;
    hipEvent_t a, b;
  };
  bool prof = false;
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

void carve_A(gsr_state* s, char* base, int64_t n, int64_t P, int64_t tiles, size_t* bytes) {
  Carver c{base};
  s->rec_uvab = c.take<float4>(n);
  s->rec_cob = c.take<float4>(n);
  s->rec_rgbz = c.take<float4>(n);
  s->rect = c.take<int4>(n);
  s->counts = c.take<uint32_t>(n);
  s->offsets = c.take<uint32_t>(n);
  s->scan_temp = c.take<uint32_t>(gsr::scan_temp_words(n));
  s->g2d = c.take<float>(10 * n);
  s->Tfin = c.take<float>(P);
  s->last = c.take<int>(P);
  s->ranges = c.take<int2>(tiles);
  s->d_K = c.take<uint32_t>(4);
  s->d_overflow = c.take<int>(4);
  s->pose_acc = c.take<float>(16);
  *bytes = c.off;
}

void carve_B(gsr_state* s, char* base, int64_t K, size_t* bytes) {
  Carver c{base};
  s->keys[0] = c.take<uint64_t>(K);
  s->keys[1] = c.take<uint64_t>(K);
  s->vals[0] = c.take<uint32_t>(K);
  s->vals[1] = c.take<uint32_t>(K);
  s->sort_temp = c.take<uint32_t>(gsr::radix_temp_words(K));
  *bytes = c.off;
}

int ensure_A(gsr_ctx* c, gsr_state* s, int64_t n, int64_t P, int64_t tiles) {
  if (s->arenaA && n <= s->n_cap && P <= s->P_cap && tiles <= s->tiles_cap) return GSR_OK;
  if (s->arenaA) GSR_HIP(c, hipFree(s->arenaA));
  s->arenaA = nullptr;
  const int64_t nn = std::max<int64_t>(n + n / 4, 1024), PP = std::max<int64_t>(P, 256),
                tt = std::max<int64_t>(tiles, 16);
  size_t bytes = 0;
  carve_A(s, nullptr, nn, PP, tt, &bytes);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, GSR_ENOMEM, "device allocation of the per-Gaussian workspace failed");
  }
  s->arenaA = p;
  carve_A(s, (char*)p, nn, PP, tt, &bytes);
  s->n_cap = nn;
  s->P_cap = PP;
  s->tiles_cap = tt;
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

int bits_for(int64_t v) {
  int b = 1;
  while ((int64_t(1) << b) < v) ++b;
  return b;
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
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
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
    if (c->prof && (a = take_event(c))) (void)hipEventRecord(a, c->stream);
  }
  ~Stage() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) return;
    (void)hipEventRecord(b, c->stream);
    c->recs.push_back({name, a, b});
  }
};

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

const char* gsr_last_error(gsr_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

void gsr_default_opts(gsr_opts* o) {
  if (!o) return;
  o->lowpass = 0.3f;
  o->alpha_min = 1.f / 255.f;
  o->alpha_max = 0.99f;
  o->T_min = 1e-4f;
  o->guard = 1.3f;
  o->tile_w = 16;
  o->tile_h = 16;
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
  if (hipHostMalloc((void**)&c->h_K, 64, hipHostMallocDefault) != hipSuccess ||
      hipMalloc((void**)&c->track_temp, sizeof(uint32_t) * gsr::track_temp_words()) != hipSuccess ||
      hipMalloc((void**)&c->d_stats, 64) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return GSR_ENOMEM;
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
    delete s;
  }
  if (c->h_K) (void)hipHostFree(c->h_K);
  if (c->track_temp) (void)hipFree(c->track_temp);
  if (c->d_stats) (void)hipFree(c->d_stats);
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

int gsr_render_fwd(gsr_ctx* c, const gsr_gaussians* g, const gsr_camera* cam, const gsr_opts* opts,
                   const float* pose7, float* color, float* depth, float* alpha, gsr_state** state) {
  if (!c || !g || !state) return fail(c, GSR_EINVAL, "ctx, gaussians and state are required");
  *state = nullptr;
  if (g->n < 0) return fail(c, GSR_EINVAL, "n must be >= 0");
  if (g->n >= (int64_t(1) << 31)) return fail(c, GSR_EINVAL, "n must be < 2^31");
  if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacities || !g->colors))
    return fail(c, GSR_EINVAL, "Gaussian parameter pointers are required");
  if (g->n > 0 && (reinterpret_cast<uintptr_t>(g->quats) & 15u) != 0)
    return fail(c, GSR_EINVAL, "quats must be 16-byte aligned");
  if (!pose7 || !color || !depth || !alpha) return fail(c, GSR_EINVAL, "pose7 and the outputs are required");
  gsr::Raster R;
  int rc = make_raster(c, cam, opts, &R);
  if (rc) return rc;
  GSR_HIP(c, hipSetDevice(c->device));
  gsr_state* s = acquire_state(c);
  if (!s) return fail(c, GSR_ENOMEM, "host allocation failed");
  const int64_t P = (int64_t)R.W * R.H;
  rc = ensure_A(c, s, g->n, P, R.n_tiles);
  if (rc) {
    s->in_use = false;
    return rc;
  }
  s->R = R;
  s->n = g->n;
  s->P = P;
  s->g = *g;
  s->pose7 = pose7;
  hipStream_t st = c->stream;

  gsr::ProjectArgs pa{g->n, g->means, g->scales, g->quats, g->opacities, g->colors, pose7,
                      s->rec_uvab, s->rec_cob, s->rec_rgbz, s->rect, s->counts};
  {
    Stage t(c, "project");
    gsr::launch_project(R, pa, st);
  }
  {
    Stage t(c, "scan");
    gsr::launch_exclusive_scan(s->counts, s->offsets, g->n, s->d_K, s->scan_temp, st);
  }
  GSR_HIP(c, hipMemcpyAsync(c->h_K, s->d_K, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  GSR_HIP(c, hipStreamSynchronize(st));
  const int64_t K = (int64_t)*c->h_K;
  s->K = K;
  rc = ensure_B(c, s, K);
  if (rc) {
    s->in_use = false;
    return rc;
  }
  gsr::BinArgs ba{g->n, s->rec_rgbz, s->rect, s->counts, s->offsets, s->d_K, K, 0u,
                  s->keys[0], s->vals[0], s->d_overflow};
  {
    Stage t(c, "duplicate");
    gsr::launch_duplicate(R, ba, st);
  }
  {
    Stage t(c, "radix_sort");
    s->sorted = gsr::launch_radix_sort(s->keys, s->vals, s->d_K, K, 32 + bits_for(R.n_tiles), s->sort_temp, st);
  }
  {
    Stage t(c, "tile_ranges");
    gsr::launch_tile_ranges(s->keys[s->sorted], s->d_K, K, s->ranges, R.n_tiles, st);
  }
  gsr::FwdArgs fa{s->ranges, s->vals[s->sorted], s->rec_uvab, s->rec_cob, s->rec_rgbz,
                  color, depth, alpha, s->Tfin, s->last, nullptr};
  {
    Stage t(c, "render_fwd");
    gsr::launch_render_fwd(R, fa, st);
  }
  rc = check_launch(c, "gsr_render_fwd kernels");
  if (rc) {
    s->in_use = false;
    return rc;
  }
  *state = s;
  return GSR_OK;
}

int gsr_render_bwd(gsr_ctx* c, gsr_state* s, const float* dL_dcolor, const float* dL_ddepth, const float* dL_dalpha,
                   const gsr_grads* grads, float* dL_dpose7, float* dL_dtwist6) {
  if (!c || !s || !s->in_use || s->ctx != c) return fail(c, GSR_EINVAL, "invalid state");
  if (!dL_dcolor || !dL_ddepth) return fail(c, GSR_EINVAL, "dL/dcolor and dL/ddepth are required");
  GSR_HIP(c, hipSetDevice(c->device));
  hipStream_t st = c->stream;
  const gsr::Raster& R = s->R;
  const bool want_pose = dL_dpose7 || dL_dtwist6;
  {
    Stage t(c, "fill");
    gsr::launch_fill_f32(s->g2d, 0.f, 10 * s->n, st);
    if (want_pose) gsr::launch_fill_f32(s->pose_acc, 0.f, 12, st);
  }
  gsr::BwdArgs ba{s->ranges, s->vals[s->sorted], s->rec_uvab, s->rec_cob, s->rec_rgbz, s->Tfin, s->last,
                  dL_dcolor, dL_ddepth, dL_dalpha, s->g2d};
  {
    Stage t(c, "render_bwd");
    gsr::launch_render_bwd(R, ba, st);
  }
  gsr_grads none{};
  const gsr_grads& G = grads ? *grads : none;
  if (G.quats && (reinterpret_cast<uintptr_t>(G.quats) & 15u) != 0)
    return fail(c, GSR_EINVAL, "the quaternion gradient must be 16-byte aligned");
  gsr::ProjectBwdArgs pb{s->n, s->g.means, s->g.scales, s->g.quats, s->g.opacities, s->g.colors, s->pose7,
                         s->counts, s->g2d, G.means, G.scales, G.quats, G.opacities, G.colors,
                         want_pose ? s->pose_acc : nullptr};
  {
    Stage t(c, "project_bwd");
    gsr::launch_project_bwd(R, pb, st);
    if (want_pose) gsr::launch_pose_finalize(s->pose7, s->pose_acc, dL_dpose7, dL_dtwist6, st);
  }
  return check_launch(c, "gsr_render_bwd kernels");
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
    GSR_HIP(c, hipMemcpyAsync(ranges, s->ranges, sizeof(int2) * s->R.n_tiles, hipMemcpyDeviceToDevice, c->stream));
  if (ids && s->K > 0)
    GSR_HIP(c, hipMemcpyAsync(ids, s->vals[s->sorted], sizeof(uint32_t) * s->K, hipMemcpyDeviceToDevice, c->stream));
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
  gsr::launch_loss_l1(color, depth, tgt_color, tgt_depth, P, w_color, w_depth, loss, dL_dcolor, dL_ddepth, c->stream);
  return check_launch(c, "gsr_loss_l1");
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

int gsr_profile_enable(gsr_ctx* c, int on) {
  if (!c) return GSR_EINVAL;
  c->prof = on != 0;
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
  gsr::FwdArgs fa{s->ranges, s->vals[s->sorted], s->rec_uvab, s->rec_cob, s->rec_rgbz,
                  nullptr, nullptr, nullptr, nullptr, nullptr, c->d_stats};
  gsr::launch_render_fwd(s->R, fa, st);
  unsigned long long h[3] = {0, 0, 0};
  GSR_HIP(c, hipMemcpyAsync(h, c->d_stats, sizeof(h), hipMemcpyDeviceToHost, st));
  std::vector<uint32_t> counts((size_t)std::max<int64_t>(s->n, 1));
  if (s->n > 0) GSR_HIP(c, hipMemcpyAsync(counts.data(), s->counts, 4 * s->n, hipMemcpyDeviceToHost, st));
  GSR_HIP(c, hipStreamSynchronize(st));
  int64_t vis = 0;
  for (int64_t i = 0; i < s->n; ++i) vis += counts[i] > 0;
  out[0] = s->K;
  out[1] = vis;
  out[2] = (int64_t)h[0];
  out[3] = (int64_t)h[1];
  out[4] = (int64_t)h[2];
  out[5] = s->R.n_tiles;
  return check_launch(c, "gsr_state_stats");
}

}  // extern "C"
