// Per-tile compositing. One 256-thread workgroup per (view, tile) item, one
// pixel per lane, one 8x8 pixel block per wave. Gaussian records of the item's depth-sorted list are staged
// through LDS in batches of 256 (one coalesced fetch per record per
// workgroup). Each wave then ballots, 64 records at a time, which records'
// support boxes overlap its own pixel block, and visits only those, in list
// order, with the record broadcast from LDS. Skipping a record whose box
// misses the block cannot change the result: outside its box a Gaussian has
// alpha < alpha_min.
//
// Forward: front to back (Eq. 3 colour, Eq. 4 alpha, Eq. 6 depth). A lane
// stops before the Gaussian that would take its transmittance below T_min; a
// wave leaves the batch as soon as all its lanes have stopped, and the
// workgroup stops fetching batches once all four waves have.
//
// Backward: back to front from each pixel's last composited Gaussian. The
// transmittance in front of Gaussian j is recomputed as T_j = T_{j+1} /
// (1 - alpha_j) instead of being stored; suffix sums of c alpha T and z alpha T
// give the second terms of dC/dalpha and Eq. 8. The ten per-Gaussian partials
// (sums of q (dx, dy, dx^2, dx dy, dy^2) with q = dL/dp / ln 2 for alpha =
// o 2^p, then opacity, colour, direct depth) of a wave are summed with a field-splitting
// butterfly and added to the [V n, 10] gradient buffer with one 10-lane
// atomic per (Gaussian, wave).
//
// Launch shapes: one workgroup per item (items dealt to XCDs in contiguous
// runs), or a persistent grid whose workgroups pull items from a counter in
// longest-list-first order until the queue is empty (multi-keyframe mapping).
#include "gsr_internal.h"

namespace gsr {

namespace {

struct Block {
  int x0, x1, y0, y1;  // inclusive pixel rectangle of a wave (8x8)
};

struct Pixel {
  int tile, view;
  int px, py;
  bool inside;
  float fpx, fpy;
  int64_t p;    // pixel index inside the view
  int64_t off;  // view * W * H
  Block blk;
};

// Each wave covers one 8x8 pixel block of the tile (a square block meets fewer
// support boxes than a 16x4 or 32x2 strip); the four blocks are row-major in
// the tile, lanes row-major in the block.
__device__ __forceinline__ Pixel item_pixel(const Raster& Rr, int item) {
  Pixel q;
  q.view = item / Rr.n_tiles;
  q.tile = item - q.view * Rr.n_tiles;
  const int tyi = q.tile / Rr.ntx, txi = q.tile - tyi * Rr.ntx;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int bpr_log2 = Rr.tw_log2 - 3;  // 8x8 blocks per tile row: 1, 2 or 4
  const int bx = w & ((1 << bpr_log2) - 1), by = w >> bpr_log2;
  q.blk.x0 = txi * Rr.tw + 8 * bx;
  q.blk.x1 = q.blk.x0 + 7;
  q.blk.y0 = tyi * Rr.th + 8 * by;
  q.blk.y1 = q.blk.y0 + 7;
  q.px = q.blk.x0 + (l & 7);
  q.py = q.blk.y0 + (l >> 3);
  q.inside = q.px < Rr.W && q.py < Rr.H;
  q.fpx = (float)q.px;
  q.fpy = (float)q.py;
  q.p = (int64_t)q.py * Rr.W + q.px;
  q.off = (int64_t)q.view * Rr.W * Rr.H;
  return q;
}

// Does the packed support box (bx = x0 | x1 << 16, by = y0 | y1 << 16) meet the block?
__device__ __forceinline__ bool box_meets(float fbx, float fby, const Block& s) {
  const uint32_t bx = __float_as_uint(fbx), by = __float_as_uint(fby);
  const int x0 = (int)(bx & 0xffffu), x1 = (int)(bx >> 16), y0 = (int)(by & 0xffffu), y1 = (int)(by >> 16);
  return (x0 <= s.x1) & (x1 >= s.x0) & (y0 <= s.y1) & (y1 >= s.y0);  // no short-circuit branches
}

// Can the record reach alpha >= alpha_min anywhere in the block? alpha = o 2^p
// with p = pa dx^2 + pb dx dy + pc dy^2 <= 0 (pa, pc < 0), so it needs
// max over the block of p >= log2(alpha_min / o). If the centre lies in the
// block the maximum is 0; otherwise it lies on the block edge(s) facing the
// centre, where p restricted to the edge is a 1D concave quadratic whose
// maximiser is clamped to the edge. The continuous block contains every pixel
// centre, and the threshold carries a margin of 1e-3 (FP32 rounding of p is
// ~1e-6), so a skipped record has alpha < alpha_min at every pixel: the
// result cannot change, only the work.
__device__ __forceinline__ bool ellipse_meets(const float4& g, const float4& cb, const Block& s, float log2_amin) {
  const float u = g.x, v = g.y, pa = g.z, pb = g.w, pc = cb.x;
  const float thr = log2_amin - __builtin_amdgcn_logf(cb.y) - 1e-3f;  // log2(alpha_min / o)
  const float X0 = (float)s.x0, X1 = (float)s.x1, Y0 = (float)s.y0, Y1 = (float)s.y1;
  const float cx = fminf(fmaxf(u, X0), X1), cy = fminf(fmaxf(v, Y0), Y1);
  float best = (cx == u && cy == v) ? 0.f : -INFINITY;
  if (cx != u) {  // edge x = cx: maximise over y
    const float dX = cx - u;
    const float y = fminf(fmaxf(v - pb * dX * __builtin_amdgcn_rcpf(2.f * pc), Y0), Y1);
    const float dy = y - v;
    best = fmaxf(best, fmaf(pa * dX, dX, fmaf(pb * dX, dy, pc * dy * dy)));
  }
  if (cy != v) {  // edge y = cy: maximise over x
    const float dY = cy - v;
    const float x = fminf(fmaxf(u - pb * dY * __builtin_amdgcn_rcpf(2.f * pa), X0), X1);
    const float dx = x - u;
    best = fmaxf(best, fmaf(pa * dx, dx, fmaf(pb * dx, dY, pc * dY * dY)));
  }
  return best >= thr;
}

__device__ __forceinline__ bool box_holds(float fbx, float fby, int px, int py) {
  const uint32_t bx = __float_as_uint(fbx), by = __float_as_uint(fby);
  return (px >= (int)(bx & 0xffffu)) & (px <= (int)(bx >> 16)) & (py >= (int)(by & 0xffffu)) & (py <= (int)(by >> 16));
}

struct FwdSmem {
  float4 uvab[kTileThreads];
  float4 cob[kTileThreads];
  float4 rgbz[kTileThreads];
};

struct BwdSmem {
  float4 uvab[kTileThreads];
  float4 cob[kTileThreads];
  float4 rgbz[kTileThreads];
  uint32_t gid[kTileThreads];
  int max_last;
};

// STATS = true: instead of writing outputs, count the algorithmic work (for the
// benchmark's roofline): pairs whose pixel lies in the Gaussian's support box
// before the pixel stops, and pairs composited.
template <bool STATS>
__device__ __forceinline__ void fwd_item(const Raster& Rr, const FwdArgs& a, int item, FwdSmem& sm) {
  const int tid = threadIdx.x, lane = tid & 63;
  const Pixel q = item_pixel(Rr, item);
  const int2 rg = a.ranges[item];
  const int start = rg.x, end = rg.y;
  // T > 0: the lane is compositing; T < 0: it has stopped and -T is its final
  // transmittance (T >= T_min > 0 while compositing, so the sign is free).
  float T = q.inside ? 1.f : -1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  int last = 0;
  uint32_t n_eval = 0, n_comp = 0;

  for (int base = start; base < end; base += kTileThreads) {
    if (__syncthreads_count(T > 0.f) == 0) break;
    const int i = base + tid;
    if (i < end) {
      const uint32_t gid = a.ids[i];
      sm.uvab[tid] = a.rec_uvab[kRec * gid];
      sm.cob[tid] = a.rec_cob[kRec * gid];
      sm.rgbz[tid] = a.rec_rgbz[kRec * gid];
    }
    __syncthreads();
    if (!__any(T > 0.f)) continue;
    const int cnt = min(kTileThreads, end - base);
    bool wave_done = false;
    for (int c = 0; c * kWave < cnt && !wave_done; ++c) {
      const int r = c * kWave + lane;
      bool meets = false;
      if (r < cnt) {
        const float4 cb = sm.cob[r];
        meets = box_meets(cb.z, cb.w, q.blk) && ellipse_meets(sm.uvab[r], cb, q.blk, Rr.log2_amin);
      }
      uint64_t m = __ballot(meets);
      while (m) {
        const int j = c * kWave + __builtin_ctzll(m);
        m &= m - 1;
        // Every lane runs the same instructions. A skipped pair (alpha <
        // alpha_min) acts as alpha = 0; a stopped lane has T < 0, so its Tn < T_min
        // and it adds w = 0 and keeps T.
        const float4 g = sm.uvab[j];
        const float4 cb = sm.cob[j];
        const float4 cz = sm.rgbz[j];
        const PairEval pe = eval_pair(q.fpx - g.x, q.fpy - g.y, g.z, g.w, cb.x, cb.y, Rr.amin, Rr.amax);
        if (STATS && T > 0.f && box_holds(cb.z, cb.w, q.px, q.py)) ++n_eval;
        const float al = pe.use ? pe.alpha : 0.f;
        const float Tn = T * (1.f - al);
        const bool comp = Tn >= Rr.tmin;  // false for a stopped lane and at the stop
        const float w = comp ? al * T : 0.f;
        C0 = fmaf(cz.x, w, C0);
        C1 = fmaf(cz.y, w, C1);
        C2 = fmaf(cz.z, w, C2);
        D = fmaf(cz.w, w, D);
        last = (comp && pe.use) ? base - start + j + 1 : last;
        if (STATS && comp && pe.use) ++n_comp;
        T = comp ? Tn : -fabsf(T);
        if (!__any(T > 0.f)) {
          wave_done = true;
          break;
        }
      }
    }
  }
  if (STATS) {
    unsigned long long e = n_eval, cm = n_comp;
    for (int o = 32; o > 0; o >>= 1) {
      e += __shfl_xor(e, o, 64);
      cm += __shfl_xor(cm, o, 64);
    }
    if (lane == 0) {
      atomicAdd(&a.stats[0], e);
      atomicAdd(&a.stats[1], cm);
    }
    return;
  }
  if (q.inside) {
    T = fabsf(T);
    const int64_t P = (int64_t)Rr.W * Rr.H;
    const int64_t p = q.off + q.p;
    float* col = a.color + 3 * q.off;
    col[q.p] = fmaf(T, Rr.bg0, C0);
    col[P + q.p] = fmaf(T, Rr.bg1, C1);
    col[2 * P + q.p] = fmaf(T, Rr.bg2, C2);
    a.depth[p] = D;
    a.alpha[p] = 1.f - T;
    a.Tfin[p] = T;
    a.last[p] = last;
  }
}

template <bool GEOM_ONLY>
__device__ __forceinline__ void bwd_item(const Raster& Rr, const BwdArgs& a, int item, BwdSmem& sm) {
  const int tid = threadIdx.x, lane = tid & 63;
  const Pixel q = item_pixel(Rr, item);
  const int64_t P = (int64_t)Rr.W * Rr.H;
  float T = 1.f, g0 = 0.f, g1 = 0.f, g2 = 0.f, gd = 0.f, ga = 0.f;
  int last = 0;
  if (q.inside) {
    const int64_t p = q.off + q.p;
    const float* gC = a.gC + 3 * q.off;
    T = a.Tfin[p];
    last = a.last[p];
    g0 = gC[q.p];
    g1 = gC[P + q.p];
    g2 = gC[2 * P + q.p];
    gd = a.gD[p];
    ga = a.gA ? a.gA[p] : 0.f;
  }
  // dL/dalpha_j = T_j (g . c_j) - (g . S_j + ga T_fin) / (1 - alpha_j) with the
  // suffix sums S_j = sum_{u > j} c_u alpha_u T_u + T_fin bg (colour) and
  // sum_{u > j} z_u alpha_u T_u (depth), g = (gC, gD). Only the dot product
  // gS = g . S_j is needed; the background enters it through T_fin bg.
  float gS = T * (g0 * Rr.bg0 + g1 * Rr.bg1 + g2 * Rr.bg2);
  const float gA = ga * T;

  __syncthreads();  // the previous item (persistent launch) is done with max_last
  if (tid == 0) sm.max_last = 0;
  __syncthreads();
  if (last > 0) atomicMax(&sm.max_last, last);
  const int wmax = wave_max_int(last);
  __syncthreads();
  const int bmax = sm.max_last;
  const int start = a.ranges[item].x;

  for (int bend = start + bmax; bend > start; bend -= kTileThreads) {
    const int bstart = max(start, bend - kTileThreads);
    __syncthreads();
    const int i = bstart + tid;
    if (i < bend) {
      const uint32_t gid = a.ids[i];
      sm.gid[tid] = gid;
      sm.uvab[tid] = a.rec_uvab[kRec * gid];
      sm.cob[tid] = a.rec_cob[kRec * gid];
      sm.rgbz[tid] = a.rec_rgbz[kRec * gid];
    }
    __syncthreads();
    const int cnt = min(bend, start + wmax) - bstart;  // records this wave may need
    for (int c = (cnt - 1) >> 6; c >= 0; --c) {
      const int r = c * kWave + lane;
      bool meets = false;
      if (r < cnt) {
        const float4 cb = sm.cob[r];
        meets = box_meets(cb.z, cb.w, q.blk) && ellipse_meets(sm.uvab[r], cb, q.blk, Rr.log2_amin);
      }
      uint64_t m = __ballot(meets);
      while (m) {
        const int bit = 63 - __builtin_clzll(m);
        m &= ~(1ull << bit);
        const int li = c * kWave + bit;
        const int pos = bstart + li - start;
        const float4 g = sm.uvab[li];
        const float4 cb = sm.cob[li];
        const float dx = q.fpx - g.x, dy = q.fpy - g.y;
        const PairEval pe = eval_pair(dx, dy, g.z, g.w, cb.x, cb.y, Rr.amin, Rr.amax);
        const bool hit = pos < last && pe.use;
        if (!__any(hit)) continue;
        // Lanes without a hit run the same instructions with alpha = 0: their
        // transmittance and suffix sums are unchanged and their partials are 0.
        const float4 cz = sm.rgbz[li];
        const float al = hit ? pe.alpha : 0.f;
        const float inv = __builtin_amdgcn_rcpf(1.f - al);  // 1 ulp; alpha <= alpha_max < 1
        const float Tj = T * inv;
        const float w = al * Tj;
        float v[10];
        v[6] = w * g0;
        v[7] = w * g1;
        v[8] = w * g2;
        v[9] = w * gd;
        const float gc = fmaf(g0, cz.x, fmaf(g1, cz.y, fmaf(g2, cz.z, gd * cz.w)));
        const float dA = fmaf(Tj, gc, -inv * (gS - gA));
        gS = fmaf(gc, w, gS);
        T = Tj;
        // a clamped alpha does not depend on o or sigma
        const float dAs = (hit && !pe.clamped) ? dA : 0.f;
        v[5] = dAs * pe.e;                       // d alpha / d o = exp(-sigma)
        // q = dL/dp / ln 2 with alpha = o 2^p; the projection backward turns the
        // sums of q (dx, dy, dx^2, dx dy, dy^2) into dL/d(u, v) and the conic terms
        const float gp = dAs * pe.alpha;
        const float gpx = gp * dx, gpy = gp * dy;
        v[0] = gpx;
        v[1] = gpy;
        v[2] = gpx * dx;
        v[3] = gpx * dy;
        v[4] = gpy * dy;
        if (GEOM_ONLY) {
          wave_add6(v, a.g2d + 10 * (int64_t)sm.gid[li], lane);
        } else {
          wave_add10(v, a.g2d + 10 * (int64_t)sm.gid[li], lane);
        }
      }
    }
  }
}

template <bool STATS>
__global__ __launch_bounds__(kTileThreads) void k_render_fwd(Raster Rr, FwdArgs a) {
  __shared__ FwdSmem sm;
  fwd_item<STATS>(Rr, a, xcd_tile(blockIdx.x, gridDim.x), sm);
}

template <bool GEOM_ONLY>
__global__ __launch_bounds__(kTileThreads) void k_render_bwd(Raster Rr, BwdArgs a) {
  __shared__ BwdSmem sm;
  bwd_item<GEOM_ONLY>(Rr, a, xcd_tile(blockIdx.x, gridDim.x), sm);
}

// Persistent workgroups: take the next item from the queue until it is empty.
// Every workgroup reaches the exit once the counter passes n_items.
__device__ __forceinline__ int next_item(int* queue, const int* order, int n_items, int* s_item) {
  __syncthreads();
  if (threadIdx.x == 0) *s_item = atomicAdd(queue, 1);
  __syncthreads();
  const int qi = *s_item;
  if (qi >= n_items) return -1;
  return order ? order[qi] : qi;
}

__global__ __launch_bounds__(kTileThreads) void k_render_fwd_persistent(Raster Rr, FwdArgs a) {
  __shared__ FwdSmem sm;
  __shared__ int s_item;
  for (;;) {
    const int item = next_item(a.queue, a.order, a.n_items, &s_item);
    if (item < 0) break;
    fwd_item<false>(Rr, a, item, sm);
  }
}

template <bool GEOM_ONLY>
__global__ __launch_bounds__(kTileThreads) void k_render_bwd_persistent(Raster Rr, BwdArgs a) {
  __shared__ BwdSmem sm;
  __shared__ int s_item;
  for (;;) {
    const int item = next_item(a.queue, a.order, a.n_items, &s_item);
    if (item < 0) break;
    bwd_item<GEOM_ONLY>(Rr, a, item, sm);
  }
}

// Support-box pairs before each pixel's last composited Gaussian: the pairs
// the backward must evaluate (work counter; reads the forward's `last`).
__global__ __launch_bounds__(kTileThreads) void k_count_bwd_pairs(Raster Rr, FwdArgs a) {
  __shared__ float4 s_cob[kTileThreads];
  const int item = blockIdx.x;
  const Pixel q = item_pixel(Rr, item);
  const int last = q.inside ? a.last[q.off + q.p] : 0;
  const int2 rg = a.ranges[item];
  unsigned long long n = 0;
  for (int base = rg.x; base < rg.y; base += kTileThreads) {
    __syncthreads();
    if (base + (int)threadIdx.x < rg.y) s_cob[threadIdx.x] = a.rec_cob[kRec * a.ids[base + threadIdx.x]];
    __syncthreads();
    const int cnt = min(kTileThreads, rg.y - base);
    for (int j = 0; j < cnt; ++j)
      if (base - rg.x + j < last && box_holds(s_cob[j].z, s_cob[j].w, q.px, q.py)) ++n;
  }
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(&a.stats[2], n);
}

// Longest-list-first item order: bucket items by floor(log2(len + 1)) and
// emit the buckets from the longest down (order inside a bucket is arbitrary).
__global__ void k_order_hist(const int2* __restrict__ ranges, int n_items, int* __restrict__ temp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  const int2 r = ranges[i];
  const int b = 31 - __clz(r.y - r.x + 1);
  atomicAdd(&temp[b], 1);
}

__global__ void k_order_scan(int* temp) {
  if (threadIdx.x != 0) return;
  int s = 0;
  for (int b = 31; b >= 0; --b) {
    const int c = temp[b];
    temp[32 + b] = s;
    s += c;
  }
}

__global__ void k_order_scatter(const int2* __restrict__ ranges, int n_items, int* __restrict__ temp,
                                int* __restrict__ order) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  const int2 r = ranges[i];
  const int b = 31 - __clz(r.y - r.x + 1);
  const int pos = atomicAdd(&temp[32 + b], 1);
  order[pos] = i;
}

}  // namespace

void launch_render_fwd(const Raster& R, const FwdArgs& a, hipStream_t s) {
  if (a.stats) {
    hipLaunchKernelGGL(k_render_fwd<true>, dim3((unsigned)a.n_items), dim3(kTileThreads), 0, s, R, a);
    hipLaunchKernelGGL(k_count_bwd_pairs, dim3((unsigned)a.n_items), dim3(kTileThreads), 0, s, R, a);
  } else if (a.blocks > 0) {
    launch_fill_u32(reinterpret_cast<uint32_t*>(a.queue), 0u, 1, s);
    hipLaunchKernelGGL(k_render_fwd_persistent, dim3((unsigned)a.blocks), dim3(kTileThreads), 0, s, R, a);
  } else {
    hipLaunchKernelGGL(k_render_fwd<false>, dim3((unsigned)a.n_items), dim3(kTileThreads), 0, s, R, a);
  }
}

void launch_render_bwd(const Raster& R, const BwdArgs& a, hipStream_t s) {
  if (a.blocks > 0) {
    launch_fill_u32(reinterpret_cast<uint32_t*>(a.queue), 0u, 1, s);
    if (a.geom_only)
      hipLaunchKernelGGL(k_render_bwd_persistent<true>, dim3((unsigned)a.blocks), dim3(kTileThreads), 0, s, R, a);
    else
      hipLaunchKernelGGL(k_render_bwd_persistent<false>, dim3((unsigned)a.blocks), dim3(kTileThreads), 0, s, R, a);
  } else if (a.geom_only) {
    hipLaunchKernelGGL(k_render_bwd<true>, dim3((unsigned)a.n_items), dim3(kTileThreads), 0, s, R, a);
  } else {
    hipLaunchKernelGGL(k_render_bwd<false>, dim3((unsigned)a.n_items), dim3(kTileThreads), 0, s, R, a);
  }
}

void launch_item_order(const int2* ranges, int n_items, int* order, int* temp, hipStream_t s) {
  launch_fill_u32(reinterpret_cast<uint32_t*>(temp), 0u, 64, s);
  const unsigned g = (unsigned)((n_items + 255) / 256);
  hipLaunchKernelGGL(k_order_hist, dim3(g), dim3(256), 0, s, ranges, n_items, temp);
  hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64), 0, s, temp);
  hipLaunchKernelGGL(k_order_scatter, dim3(g), dim3(256), 0, s, ranges, n_items, temp, order);
}

}  // namespace gsr
