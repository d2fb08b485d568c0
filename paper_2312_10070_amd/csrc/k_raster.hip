// Per-tile compositing. One 256-thread workgroup per tile, one pixel per lane.
// Gaussian records of the tile's depth-sorted list are staged through LDS in
// batches of 256 (one coalesced fetch per record per workgroup). Each wave
// then ballots, 64 records at a time, which records' support boxes overlap its
// own pixel strip, and visits only those, in list order, with the record
// broadcast from LDS. Skipping a record whose box misses the strip cannot
// change the result: outside its box a Gaussian has alpha < alpha_min.
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
// of a wave are summed with a field-splitting butterfly and added to the
// [n, 10] gradient buffer with one 10-lane atomic per (Gaussian, wave).
#include "gsr_internal.h"

namespace gsr {

namespace {

struct Strip {
  int x0, x1, y0, y1;  // inclusive pixel rectangle of a wave
};

__device__ __forceinline__ Strip wave_strip(const Raster& Rr, int txi, int tyi, int wave) {
  const int rows = kWave >> Rr.tw_log2;  // pixel rows per wave
  Strip s;
  s.x0 = txi * Rr.tw;
  s.x1 = s.x0 + Rr.tw - 1;
  s.y0 = tyi * Rr.th + wave * rows;
  s.y1 = s.y0 + rows - 1;
  return s;
}

// Does the packed support box (bx = x0 | x1 << 16, by = y0 | y1 << 16) meet the strip?
__device__ __forceinline__ bool box_meets(float fbx, float fby, const Strip& s) {
  const uint32_t bx = __float_as_uint(fbx), by = __float_as_uint(fby);
  const int x0 = (int)(bx & 0xffffu), x1 = (int)(bx >> 16), y0 = (int)(by & 0xffffu), y1 = (int)(by >> 16);
  return x0 <= s.x1 && x1 >= s.x0 && y0 <= s.y1 && y1 >= s.y0;
}

__device__ __forceinline__ bool box_holds(float fbx, float fby, int px, int py) {
  const uint32_t bx = __float_as_uint(fbx), by = __float_as_uint(fby);
  return px >= (int)(bx & 0xffffu) && px <= (int)(bx >> 16) && py >= (int)(by & 0xffffu) && py <= (int)(by >> 16);
}

// STATS = true: instead of writing outputs, count the algorithmic work (for the
// benchmark's roofline): pairs whose pixel lies in the Gaussian's support box
// before the pixel stops (forward), pairs composited, and pairs in the support
// box before each pixel's last composited Gaussian (what the backward must
// evaluate). Same control flow as the rendering launch.
template <bool STATS>
__global__ __launch_bounds__(kTileThreads) void k_render_fwd(Raster Rr, FwdArgs a);

// Backward-pair counting needs the final `last`; done in a second sweep.
__global__ __launch_bounds__(kTileThreads) void k_count_bwd_pairs(Raster Rr, FwdArgs a) {
  __shared__ float4 s_cob[kTileThreads];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tyi = tile / Rr.ntx, txi = tile - tyi * Rr.ntx;
  const int tid = threadIdx.x;
  const int px = txi * Rr.tw + (tid & (Rr.tw - 1));
  const int py = tyi * Rr.th + (tid >> Rr.tw_log2);
  const bool inside = px < Rr.W && py < Rr.H;
  const int last = inside ? a.last[(int64_t)py * Rr.W + px] : 0;
  const int2 rg = a.ranges[tile];
  unsigned long long n = 0;
  for (int base = rg.x; base < rg.y; base += kTileThreads) {
    __syncthreads();
    if (base + tid < rg.y) s_cob[tid] = a.rec_cob[a.ids[base + tid]];
    __syncthreads();
    const int cnt = min(kTileThreads, rg.y - base);
    for (int j = 0; j < cnt; ++j)
      if (base - rg.x + j < last && box_holds(s_cob[j].z, s_cob[j].w, px, py)) ++n;
  }
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
  if ((tid & 63) == 0) atomicAdd(&a.stats[2], n);
}

// STATS = true: count work instead of writing outputs (see above).
template <bool STATS>
__global__ __launch_bounds__(kTileThreads) void k_render_fwd(Raster Rr, FwdArgs a) {
  __shared__ float4 s_uvab[kTileThreads];
  __shared__ float4 s_cob[kTileThreads];
  __shared__ float4 s_rgbz[kTileThreads];

  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tyi = tile / Rr.ntx, txi = tile - tyi * Rr.ntx;
  const int tid = threadIdx.x, lane = tid & 63;
  const int px = txi * Rr.tw + (tid & (Rr.tw - 1));
  const int py = tyi * Rr.th + (tid >> Rr.tw_log2);
  const bool inside = px < Rr.W && py < Rr.H;
  const float fpx = (float)px, fpy = (float)py;
  const Strip strip = wave_strip(Rr, txi, tyi, tid >> 6);

  const int2 rg = a.ranges[tile];
  const int start = rg.x, end = rg.y;
  bool done = !inside;
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  int last = 0;
  uint32_t n_eval = 0, n_comp = 0;

  for (int base = start; base < end; base += kTileThreads) {
    if (__syncthreads_count(!done) == 0) break;
    const int i = base + tid;
    if (i < end) {
      const uint32_t gid = a.ids[i];
      s_uvab[tid] = a.rec_uvab[gid];
      s_cob[tid] = a.rec_cob[gid];
      s_rgbz[tid] = a.rec_rgbz[gid];
    }
    __syncthreads();
    if (!__any(!done)) continue;
    const int cnt = min(kTileThreads, end - base);
    bool wave_done = false;
    for (int c = 0; c * kWave < cnt && !wave_done; ++c) {
      const int r = c * kWave + lane;
      bool meets = false;
      if (r < cnt) {
        const float4 cb = s_cob[r];
        meets = box_meets(cb.z, cb.w, strip);
      }
      uint64_t m = __ballot(meets);
      while (m) {
        const int j = c * kWave + __builtin_ctzll(m);
        m &= m - 1;
        if (!done) {
          const float4 g = s_uvab[j];
          const float4 cb = s_cob[j];
          const PairEval pe = eval_pair(fpx - g.x, fpy - g.y, g.z, g.w, cb.x, cb.y, Rr.amin, Rr.amax);
          if (STATS && box_holds(cb.z, cb.w, px, py)) ++n_eval;
          if (pe.use) {
            const float Tn = T * (1.f - pe.alpha);
            if (Tn < Rr.tmin) {
              done = true;
            } else {
              const float4 cz = s_rgbz[j];
              const float w = pe.alpha * T;
              C0 = fmaf(cz.x, w, C0);
              C1 = fmaf(cz.y, w, C1);
              C2 = fmaf(cz.z, w, C2);
              D = fmaf(cz.w, w, D);
              T = Tn;
              last = base - start + j + 1;
              if (STATS) ++n_comp;
            }
          }
        }
        if (!__any(!done)) {
          wave_done = true;
          break;
        }
      }
    }
  }
  if (STATS) {
    // counters: [0] support-box pairs before stopping, [1] composited pairs
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
  if (inside) {
    const int64_t P = (int64_t)Rr.W * Rr.H;
    const int64_t p = (int64_t)py * Rr.W + px;
    a.color[p] = fmaf(T, Rr.bg0, C0);
    a.color[P + p] = fmaf(T, Rr.bg1, C1);
    a.color[2 * P + p] = fmaf(T, Rr.bg2, C2);
    a.depth[p] = D;
    a.alpha[p] = 1.f - T;
    a.Tfin[p] = T;
    a.last[p] = last;
  }
}

__global__ __launch_bounds__(kTileThreads) void k_render_bwd(Raster Rr, BwdArgs a) {
  __shared__ float4 s_uvab[kTileThreads];
  __shared__ float4 s_cob[kTileThreads];
  __shared__ float4 s_rgbz[kTileThreads];
  __shared__ uint32_t s_gid[kTileThreads];
  __shared__ int s_max;

  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tyi = tile / Rr.ntx, txi = tile - tyi * Rr.ntx;
  const int tid = threadIdx.x, lane = tid & 63;
  const int px = txi * Rr.tw + (tid & (Rr.tw - 1));
  const int py = tyi * Rr.th + (tid >> Rr.tw_log2);
  const bool inside = px < Rr.W && py < Rr.H;
  const float fpx = (float)px, fpy = (float)py;
  const int64_t P = (int64_t)Rr.W * Rr.H;
  const int64_t p = (int64_t)py * Rr.W + px;
  const Strip strip = wave_strip(Rr, txi, tyi, tid >> 6);

  float T = 1.f, g0 = 0.f, g1 = 0.f, g2 = 0.f, gd = 0.f, ga = 0.f;
  int last = 0;
  if (inside) {
    T = a.Tfin[p];
    last = a.last[p];
    g0 = a.gC[p];
    g1 = a.gC[P + p];
    g2 = a.gC[2 * P + p];
    gd = a.gD[p];
    ga = a.gA ? a.gA[p] : 0.f;
  }
  const float Tfin = T;
  // suffix sums: the background enters dC/dalpha through T_final * bg
  float S0 = T * Rr.bg0, S1 = T * Rr.bg1, S2 = T * Rr.bg2, SD = 0.f;

  if (tid == 0) s_max = 0;
  __syncthreads();
  if (last > 0) atomicMax(&s_max, last);
  const int wmax = wave_max_int(last);
  __syncthreads();
  const int bmax = s_max;
  const int start = a.ranges[tile].x;

  for (int bend = start + bmax; bend > start; bend -= kTileThreads) {
    const int bstart = max(start, bend - kTileThreads);
    __syncthreads();
    const int i = bstart + tid;
    if (i < bend) {
      const uint32_t gid = a.ids[i];
      s_gid[tid] = gid;
      s_uvab[tid] = a.rec_uvab[gid];
      s_cob[tid] = a.rec_cob[gid];
      s_rgbz[tid] = a.rec_rgbz[gid];
    }
    __syncthreads();
    const int cnt = min(bend, start + wmax) - bstart;  // records this wave may need
    for (int c = (cnt - 1) >> 6; c >= 0; --c) {
      const int r = c * kWave + lane;
      bool meets = false;
      if (r < cnt) {
        const float4 cb = s_cob[r];
        meets = box_meets(cb.z, cb.w, strip);
      }
      uint64_t m = __ballot(meets);
      while (m) {
        const int bit = 63 - __builtin_clzll(m);
        m &= ~(1ull << bit);
        const int li = c * kWave + bit;
        const int pos = bstart + li - start;
        float v[10];
#pragma unroll
        for (int f = 0; f < 10; ++f) v[f] = 0.f;
        bool hit = false;
        if (pos < last) {
          const float4 g = s_uvab[li];
          const float4 cb = s_cob[li];
          const float dx = fpx - g.x, dy = fpy - g.y;
          const PairEval pe = eval_pair(dx, dy, g.z, g.w, cb.x, cb.y, Rr.amin, Rr.amax);
          if (pe.use) {
            hit = true;
            const float4 cz = s_rgbz[li];
            const float inv = 1.f / (1.f - pe.alpha);
            const float Tj = T * inv;
            const float w = pe.alpha * Tj;
            v[6] = w * g0;
            v[7] = w * g1;
            v[8] = w * g2;
            v[9] = w * gd;
            float dA = g0 * (cz.x * Tj - S0 * inv) + g1 * (cz.y * Tj - S1 * inv) + g2 * (cz.z * Tj - S2 * inv);
            dA += gd * (cz.w * Tj - SD * inv);
            dA += ga * Tfin * inv;
            S0 = fmaf(cz.x, w, S0);
            S1 = fmaf(cz.y, w, S1);
            S2 = fmaf(cz.z, w, S2);
            SD = fmaf(cz.w, w, SD);
            T = Tj;
            if (!pe.clamped) {
              v[5] = dA * pe.e;                       // d alpha / d o = exp(-sigma)
              const float gp = dA * pe.alpha * kLn2;  // dL/dp with alpha = o 2^p
              const float gpx = gp * dx, gpy = gp * dy;
              v[2] = gpx * dx;
              v[3] = gpx * dy;
              v[4] = gpy * dy;
              v[0] = -(2.f * g.z * gpx + g.w * gpy);
              v[1] = -(g.w * gpx + 2.f * cb.x * gpy);
            }
          }
        }
        if (__any(hit)) wave_add10(v, a.g2d + 10 * (int64_t)s_gid[li], lane);
      }
    }
  }
}

}  // namespace

void launch_render_fwd(const Raster& R, const FwdArgs& a, hipStream_t s) {
  if (a.stats) {
    hipLaunchKernelGGL(k_render_fwd<true>, dim3((unsigned)R.n_tiles), dim3(kTileThreads), 0, s, R, a);
    hipLaunchKernelGGL(k_count_bwd_pairs, dim3((unsigned)R.n_tiles), dim3(kTileThreads), 0, s, R, a);
  } else
    hipLaunchKernelGGL(k_render_fwd<false>, dim3((unsigned)R.n_tiles), dim3(kTileThreads), 0, s, R, a);
}

void launch_render_bwd(const Raster& R, const BwdArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_render_bwd, dim3((unsigned)R.n_tiles), dim3(kTileThreads), 0, s, R, a);
}

}  // namespace gsr
