// Losses and their upstream gradients (Eq. 9, Eq. 10 with its L1 and SSIM
// terms, and the masked tracking loss of Eq. 15), the exact median the inlier
// mask needs (radix select on float bits, all on the device), and Adam.
#include <cmath>

#include "gsr_internal.h"

namespace gsr {

namespace {

__device__ __forceinline__ float sgnf(float r) { return (float)((r > 0.f) - (r < 0.f)); }

constexpr int kRedSlots = 4096;  // most workgroups a grid_sum launch may have
constexpr int kRedGroup = 32;    // workgroups per first-level ticket
constexpr int kRedGroups = kRedSlots / kRedGroup;
constexpr int kLine = 16;        // words per 64-byte line: one ticket per line
// red layout (uint32 words): partials | group sums | group tickets | final ticket
constexpr int kRedSums = kRedSlots, kRedTickets = kRedSums + kRedGroups;
constexpr int kRedFinal = kRedTickets + kRedGroups * kLine;
constexpr int kRedWords = kRedFinal + kLine;

__device__ __forceinline__ float block_sum(float v) {
  __shared__ float part[4];
  const float s = wave_sum_all(v);
  __syncthreads();  // part[] may still be read from a previous call
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  return part[0] + part[1] + part[2] + part[3];
}

// Stores `value` to the device-coherent level, waits for it, then takes a
// ticket; returns true for the last of `n` takers (who resets the ticket).
// No release fence: that would also write back the workgroup's unrelated stores.
__device__ __forceinline__ bool publish_and_count(float* slot, float value, uint32_t* ticket, uint32_t n) {
  __hip_atomic_store(slot, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  const uint32_t t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (t != n - 1) return false;
  __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// Sum of v over the whole grid into *out (overwritten), in a fixed order and
// with at most kRedGroup same-address atomics in a row (those serialise in
// L2): every workgroup publishes its partial; the last of each group of
// kRedGroup workgroups sums the group's partials and publishes that; the last
// group sums the group sums. Tickets return to zero. red: kRedWords words,
// zero before the first launch. With `accumulate`, *out becomes
// *out + (offset + scale * total) instead. With `clear`, the last workgroup
// (which runs after every other one has published its partial, so after all
// their earlier reads) zeroes clear[0, n_clear).
__device__ __forceinline__ void grid_sum(float v, float* out, uint32_t* red, bool accumulate = false,
                                         float scale = 1.f, float offset = 0.f, uint32_t* clear = nullptr,
                                         int n_clear = 0) {
  __shared__ bool go;
  float* f = reinterpret_cast<float*>(red);
  const uint32_t b = blockIdx.x, n = gridDim.x;
  const uint32_t g = b / kRedGroup, n_groups = (n + kRedGroup - 1) / kRedGroup;
  const uint32_t in_group = min((uint32_t)kRedGroup, n - g * kRedGroup);
  const float s = block_sum(v);
  if (threadIdx.x == 0) go = publish_and_count(f + b, s, red + kRedTickets + kLine * g, in_group);
  __syncthreads();
  if (!go) return;
  float acc = threadIdx.x < in_group
                  ? __hip_atomic_load(f + g * kRedGroup + threadIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                  : 0.f;
  const float gs = block_sum(acc);
  if (threadIdx.x == 0) go = publish_and_count(f + kRedSums + g, gs, red + kRedFinal, n_groups);
  __syncthreads();
  if (!go) return;
  acc = threadIdx.x < n_groups
            ? __hip_atomic_load(f + kRedSums + threadIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
            : 0.f;
  const float total = block_sum(acc);
  if (threadIdx.x == 0) *out = accumulate ? *out + (offset + scale * total) : total;
  for (int i = threadIdx.x; i < n_clear; i += blockDim.x) clear[i] = 0u;
}

__device__ __forceinline__ float4 ld4(const float* p, int64_t i) { return reinterpret_cast<const float4*>(p)[i]; }
__device__ __forceinline__ void st4(float* p, int64_t i, float4 v) { reinterpret_cast<float4*>(p)[i] = v; }
__device__ __forceinline__ float l1_term(float r, float w, float* g) {
  *g = sgnf(r) * w;
  return fabsf(r) * w;
}

// P4 = P / 4 when every plane is 16-byte aligned (float4 path for pixels
// [0, 4 P4)), else 0; the rest is handled one pixel at a time.
__global__ __launch_bounds__(256) void k_loss_l1(const float* __restrict__ C, const float* __restrict__ D,
                                                const float* __restrict__ Ct, const float* __restrict__ Dt, int64_t P,
                                                int64_t P4, float wc3, float wd1, float* __restrict__ loss,
                                                float* __restrict__ gC, float* __restrict__ gD,
                                                uint32_t* __restrict__ red) {
  float acc = 0.f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P4; i += stride) {
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      const float* X = ch < 3 ? C + ch * P : D;
      const float* Y = ch < 3 ? Ct + ch * P : Dt;
      float* G = ch < 3 ? gC + ch * P : gD;
      const float w = ch < 3 ? wc3 : wd1;
      const float4 x = ld4(X, i), y = ld4(Y, i);
      float4 g;
      acc += l1_term(x.x - y.x, w, &g.x) + l1_term(x.y - y.y, w, &g.y) + l1_term(x.z - y.z, w, &g.z) +
             l1_term(x.w - y.w, w, &g.w);
      st4(G, i, g);
    }
  }
  for (int64_t i = 4 * P4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += stride) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float r = C[ch * P + i] - Ct[ch * P + i];
      acc += fabsf(r) * wc3;
      gC[ch * P + i] = sgnf(r) * wc3;
    }
    const float rd = D[i] - Dt[i];
    acc += fabsf(rd) * wd1;
    gD[i] = sgnf(rd) * wd1;
  }
  grid_sum(acc, loss, red);
}

// ---- exact lower median of e = |D - D*| over pixels with D* > 0 ----------
// Radix select on the float bits of e (non-negative, so the bits order like
// the values), 8 bits per pass from the top. Pass p builds the 256-bin
// histogram hist[p] of the digit at bits [24 - 8p, 32 - 8p) among the pixels
// whose higher digits equal the prefix chosen so far; every workgroup of pass
// p (and of the loss kernel) re-derives that prefix from hist[0..p-1] with a
// wave scan, so no separate single-workgroup "pick" launches are needed.
constexpr int kSelPasses = 4;
constexpr int kSelWords = kSelPasses * 256;

struct SelState {
  uint32_t prefix, mask, rank, count;
};

// Digit of the pass whose histogram is h holding rank k (lower median rule):
// lane L covers bins 4L..4L+3. Returns the digit and the rank inside it.
__device__ __forceinline__ void pick_digit(const uint32_t* __restrict__ h, uint32_t k, uint32_t& digit,
                                           uint32_t& k_in, uint32_t& total) {
  const int lane = threadIdx.x & 63;
  const uint4 c = reinterpret_cast<const uint4*>(h)[lane];
  const uint32_t s = c.x + c.y + c.z + c.w;
  uint32_t incl = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  total = __shfl(incl, 63, 64);
  const uint32_t excl = incl - s;
  const uint64_t m = __ballot(k >= excl && k < incl);
  if (m == 0) {  // no valid pixel: the median is unused
    digit = 255;
    k_in = 0;
    return;
  }
  const int L = __builtin_ctzll(m);
  uint32_t kk = k - __shfl(excl, L, 64);
  const uint32_t c0 = __shfl(c.x, L, 64), c1 = __shfl(c.y, L, 64), c2 = __shfl(c.z, L, 64);
  uint32_t d = 4 * L;
  if (kk >= c0) { kk -= c0; ++d;
    if (kk >= c1) { kk -= c1; ++d;
      if (kk >= c2) { kk -= c2; ++d; } } }
  digit = d;
  k_in = kk;
}

// State after the picks of passes 0..passes-1 (wave-uniform; every wave computes it).
__device__ __forceinline__ SelState select_state(const uint32_t* __restrict__ st, int passes) {
  SelState r{0u, 0u, 0u, 0u};
  for (int p = 0; p < passes; ++p) {
    uint32_t d, kin, total;
    pick_digit(st + 256 * p, r.rank, d, kin, total);
    if (p == 0) {
      r.count = total;
      // rank of the lower median among `total` values
      const uint32_t k0 = total > 0 ? (total - 1) / 2 : 0;
      pick_digit(st, k0, d, kin, total);
    }
    const int shift = 24 - 8 * p;
    r.prefix |= d << shift;
    r.mask |= 0xffu << shift;
    r.rank = kin;
  }
  return r;
}

__global__ __launch_bounds__(256) void k_select_hist(const float* __restrict__ D, const float* __restrict__ Dt, int64_t P,
                                                    int pass, uint32_t* __restrict__ st) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  const SelState sel = select_state(st, pass);
  const int shift = 24 - 8 * pass;
  __syncthreads();
  // four pixels per thread and round: their loads are in flight together
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < P; i0 += 4 * stride) {
    float d[4], dt[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = min(i0 + u * stride, P - 1);
      d[u] = D[i];
      dt[u] = Dt[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i0 + u * stride < P && dt[u] > 0.f) {
        const uint32_t b = __float_as_uint(fabsf(d[u] - dt[u]));
        if ((b & sel.mask) == sel.prefix) atomicAdd(&h[(b >> shift) & 0xffu], 1u);
      }
    }
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&st[256 * pass + threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(256) void k_loss_track(const float* __restrict__ C, const float* __restrict__ D,
                                                   const float* __restrict__ A, const float* __restrict__ Ct,
                                                   const float* __restrict__ Dt, int64_t P, float lambda_c,
                                                   float inlier_mult, uint32_t* __restrict__ st,
                                                   float* __restrict__ loss, float* __restrict__ gC,
                                                   float* __restrict__ gD, float* __restrict__ median,
                                                   uint32_t* __restrict__ red) {
  const SelState sel = select_state(st, kSelPasses);
  const bool any = sel.count > 0;
  const float med = any ? __uint_as_float(sel.prefix) : 0.f;
  if (median && blockIdx.x == 0 && threadIdx.x == 0) *median = med;
  const float thr = inlier_mult * med;
  const float lc = lambda_c, ld = 1.f - lambda_c;
  float acc = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
    const float dt = Dt[i];
    const float rd = D[i] - dt;
    const bool inl = any && dt > 0.f && fabsf(rd) <= thr;
    const float a = A[i];
    const float w = inl ? a * a * a : 0.f;
    float l = 0.f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float r = C[ch * P + i] - Ct[ch * P + i];
      l += fabsf(r);
      gC[ch * P + i] = w * lc * sgnf(r);
    }
    gD[i] = w * ld * sgnf(rd);
    acc += w * (lc * l + ld * fabsf(rd));
  }
  // the histograms are read by now: the last workgroup clears them for the next call
  grid_sum(acc, loss, red, false, 1.f, 0.f, st, kSelWords);
}

// ---- SSIM term of the mapping colour loss (Eq. 10) ------------------------
// SSIM after Wang et al. 2004: per channel, an 11x11 Gaussian window (sigma
// 1.5, unit sum, applied as two 11-tap passes), zero padding, C1 = 1e-4,
// C2 = 9e-4 for values in [0, 1]. A workgroup takes one 32x32 block of one
// channel at a time and keeps everything in LDS: the five windowed moments
// (mu_x, mu_y, E[x^2], E[y^2], E[xy]) over the block and a 5-pixel apron, the
// partials of SSIM(p) with respect to them on that apron (zero outside the
// image), and the windowed sums of those partials over the block, which give
//   d mean SSIM / d x_q = (1/n) sum_p w(q - p) (A_p + 2 x_q B_p + y_q C_p)
// with A = dS/dmu_x, B = dS/dE[x^2], C = dS/dE[xy] (the moments taken as
// independent: sigma_x^2 = E[x^2] - mu_x^2, sigma_xy = E[xy] - mu_x mu_y).
// Global memory sees the two images (with a 10-pixel apron, mostly from L2),
// the gradient read-modify-write and one partial per workgroup.
constexpr int kSsR = 5;                // window half-width
constexpr int kSsT = 32;               // output block edge
constexpr int kSsS = kSsT + 2 * kSsR;  // 42: moments and partials edge
constexpr int kSsI = kSsT + 4 * kSsR;  // 52: input edge
constexpr int kSsTaps = 2 * kSsR + 1;
static_assert(kSsS % 3 == 0 && kSsT % 2 == 0 && kSsT * 8 == 256, "SSIM work split");

struct SsimWin {
  float w[kSsTaps];
};

struct SsimSmem {
  union {
    struct {
      float x[kSsI * kSsI], y[kSsI * kSsI];  // inputs (steps 1-2)
    } in;
    float part[3][kSsS * kSsS];  // A, B, C on the apron (steps 3-4)
  } a;
  union {
    float hm[5][kSsI * kSsS];  // row sums of the five moments, 52 rows x 42 (steps 2-3)
    float hp[3][kSsS * kSsT];  // row sums of A, B, C, 42 rows x 32 (steps 4-5)
  } b;
};

constexpr int kSsLd = (kSsI * kSsI + 255) / 256;  // input elements per thread and image

// One block's inputs (block and 10-pixel apron) into registers: element
// threadIdx.x + 256 j of the 52 x 52 window goes to v[j], read at the nearest
// in-image pixel; bit j of the result says whether it lies in the image (else
// it counts as zero). The loads are unconditional so that nothing waits for
// them before the values are stored.
__device__ __forceinline__ uint32_t ssim_load(const float* __restrict__ X, const float* __restrict__ Y, int H, int W,
                                              int tiles_x, int n_tiles, int item, float (&vx)[kSsLd],
                                              float (&vy)[kSsLd]) {
  const int ch = item / n_tiles, tile = item - ch * n_tiles;
  const int ty0 = (tile / tiles_x) * kSsT, tx0 = (tile % tiles_x) * kSsT;
  const int64_t base = (int64_t)ch * H * W;
  uint32_t in_mask = 0;
#pragma unroll
  for (int j = 0; j < kSsLd; ++j) {
    const int i = threadIdx.x + 256 * j;
    const int r = i / kSsI, c = i - r * kSsI;
    const int gy = ty0 - 2 * kSsR + r, gx = tx0 - 2 * kSsR + c;
    in_mask |= (uint32_t)(i < kSsI * kSsI && gy >= 0 && gy < H && gx >= 0 && gx < W) << j;
    const int64_t o = base + (int64_t)min(max(gy, 0), H - 1) * W + min(max(gx, 0), W - 1);
    vx[j] = X[o];
    vy[j] = Y[o];
  }
  return in_mask;
}

// lsum accumulates SSIM(p) over the pixels of the blocks this workgroup owns;
// *loss += loffset + lscale * (sum over the grid); gX += gscale * d(sum SSIM)/dx.
// A workgroup normally owns one block (the grid has one workgroup per block up
// to the reduction's limit), so the other workgroup on its CU hides its input
// latency; the gradient step's own global reads are issued a step early.
__global__ __launch_bounds__(256, 2) void k_loss_ssim(const float* __restrict__ X, const float* __restrict__ Y, int H,
                                                      int W, int tiles_x, int n_tiles, SsimWin win, float gscale,
                                                      float lscale, float loffset, float* __restrict__ loss,
                                                      float* __restrict__ gX, uint32_t* __restrict__ red) {
  __shared__ SsimSmem sm;
  constexpr float c1 = 1e-4f, c2 = 9e-4f;
  const int tid = threadIdx.x;
  const int64_t plane = (int64_t)H * W;
  const int n_items = 3 * n_tiles;
  float lsum = 0.f;
  // Workgroups are dealt to the 8 XCDs in turn (b mod 8), each with its own L2:
  // XCD x takes the x-th contiguous eighth of the blocks, so neighbouring
  // blocks, which share their aprons, meet in one L2. A bijection on
  // [0, n_items) whenever the grid is n_items or a multiple of 8.
  const int xq = n_items >> 3, xr = n_items & 7;
  for (int v = blockIdx.x; v < n_items; v += gridDim.x) {
    const int xcd = v & 7, local = v >> 3;
    const int item = xcd * xq + min(xcd, xr) + local;
    const int ch = item / n_tiles, tile = item - ch * n_tiles;
    const int ty0 = (tile / tiles_x) * kSsT, tx0 = (tile % tiles_x) * kSsT;
    float vx[kSsLd], vy[kSsLd];
    const uint32_t in_mask = ssim_load(X, Y, H, W, tiles_x, n_tiles, item, vx, vy);
    __syncthreads();  // the previous block's last step still reads sm.b
    // 1: the inputs to LDS
#pragma unroll
    for (int j = 0; j < kSsLd; ++j) {
      const int i = tid + 256 * j;
      if (i < kSsI * kSsI) {
        const bool in = (in_mask >> j) & 1u;
        sm.a.in.x[i] = in ? vx[j] : 0.f;
        sm.a.in.y[i] = in ? vy[j] : 0.f;
      }
    }
    __syncthreads();
    // 2: row sums of x, y, x^2, y^2, xy; 14 adjacent outputs per thread (156 threads)
    if (tid < kSsI * 3) {
      const int r = tid / 3, c0 = 14 * (tid - 3 * r);
      float acc[5][14] = {};
#pragma unroll
      for (int k = 0; k < kSsTaps + 13; ++k) {
        const float xv = sm.a.in.x[r * kSsI + c0 + k], yv = sm.a.in.y[r * kSsI + c0 + k];
        const float m[5] = {xv, yv, xv * xv, yv * yv, xv * yv};
#pragma unroll
        for (int o = 0; o < 14; ++o) {
          const int t = k - o;
          if (t < 0 || t >= kSsTaps) continue;
#pragma unroll
          for (int q = 0; q < 5; ++q) acc[q][o] = fmaf(win.w[t], m[q], acc[q][o]);
        }
      }
#pragma unroll
      for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int o = 0; o < 14; ++o) sm.b.hm[q][r * kSsS + c0 + o] = acc[q][o];
    }
    __syncthreads();
    // 3: column sums give the moments at apron position (r, c), pixel
    //    (ty0 - 5 + r, tx0 - 5 + c); then SSIM and its partials there
    //    (7 rows per thread, 252 threads)
    if (tid < kSsS * 6) {
      const int sg = tid / kSsS, c = tid - sg * kSsS, r0 = 7 * sg;
      float acc[5][7] = {};
#pragma unroll
      for (int k = 0; k < kSsTaps + 6; ++k) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const float v = sm.b.hm[q][(r0 + k) * kSsS + c];
#pragma unroll
          for (int o = 0; o < 7; ++o) {
            const int t = k - o;
            if (t >= 0 && t < kSsTaps) acc[q][o] = fmaf(win.w[t], v, acc[q][o]);
          }
        }
      }
      const int gx = tx0 - kSsR + c;
#pragma unroll
      for (int o = 0; o < 7; ++o) {
        const int r = r0 + o, gy = ty0 - kSsR + r;
        float pa = 0.f, pb = 0.f, pc = 0.f;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
          const float mx = acc[0][o], my = acc[1][o];
          const float vxx = acc[2][o] - mx * mx, vyy = acc[3][o] - my * my, cxy = acc[4][o] - mx * my;
          const float a1 = 2.f * mx * my + c1, a2 = 2.f * cxy + c2;
          const float rb1 = __builtin_amdgcn_rcpf(mx * mx + my * my + c1);
          const float rb2 = __builtin_amdgcn_rcpf(vxx + vyy + c2);
          const float s = a1 * a2 * (rb1 * rb2);
          if (r >= kSsR && r < kSsR + kSsT && c >= kSsR && c < kSsR + kSsT) lsum += s;
          // partials of s = a1 a2 / (b1 b2), written without dividing by a1 or a2
          pb = -s * rb2;                // dS/dsigma_x^2 = dS/dE[x^2]
          pc = 2.f * a1 * rb1 * rb2;    // dS/dsigma_xy = dS/dE[xy]
          pa = 2.f * rb1 * (my * a2 * rb2 - mx * s) - 2.f * mx * pb - my * pc;  // total dS/dmu_x
        }
        sm.a.part[0][r * kSsS + c] = pa;
        sm.a.part[1][r * kSsS + c] = pb;
        sm.a.part[2][r * kSsS + c] = pc;
      }
    }
    // the gradient step's pixels (ty0 + r5 + o, tx0 + c5), read a step early at
    // the nearest in-image pixel (only in-image ones are used)
    const int c5 = tid & (kSsT - 1), r5 = 4 * (tid >> 5);
    const float* x = X + ch * plane;
    const float* y = Y + ch * plane;
    float* g = gX + ch * plane;
    float xs[4], ys[4], gs[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      const int64_t q = (int64_t)min(ty0 + r5 + o, H - 1) * W + min(tx0 + c5, W - 1);
      xs[o] = x[q];
      ys[o] = y[q];
      gs[o] = g[q];
    }
    __syncthreads();
    // 4: row sums of A, B, C for output column c (pixel tx0 + c); 8 per thread (168 threads)
    if (tid < kSsS * 4) {
      const int r = tid >> 2, c0 = 8 * (tid & 3);
      float acc[3][8] = {};
#pragma unroll
      for (int k = 0; k < kSsTaps + 7; ++k) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const float v = sm.a.part[q][r * kSsS + c0 + k];
#pragma unroll
          for (int o = 0; o < 8; ++o) {
            const int t = k - o;
            if (t >= 0 && t < kSsTaps) acc[q][o] = fmaf(win.w[t], v, acc[q][o]);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int o = 0; o < 8; ++o) sm.b.hp[q][r * kSsT + c0 + o] = acc[q][o];
    }
    __syncthreads();
    // 5: column sums; gradient at pixel (ty0 + r5 + o, tx0 + c5), four rows per thread
    {
      float acc[3][4] = {};
#pragma unroll
      for (int k = 0; k < kSsTaps + 3; ++k) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const float v = sm.b.hp[q][(r5 + k) * kSsT + c5];
#pragma unroll
          for (int o = 0; o < 4; ++o) {
            const int t = k - o;
            if (t >= 0 && t < kSsTaps) acc[q][o] = fmaf(win.w[t], v, acc[q][o]);
          }
        }
      }
      const int gx = tx0 + c5;
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        const int gy = ty0 + r5 + o;
        if (gy < H && gx < W)
          g[(int64_t)gy * W + gx] = gs[o] + gscale * (acc[0][o] + 2.f * xs[o] * acc[1][o] + ys[o] * acc[2][o]);
      }
    }
  }
  grid_sum(lsum, loss, red, true, lscale, loffset);
}

// ---- isotropic scale regulariser (Eq. 11) -----------------------------------
// *loss += lscale * sum_k sum_i |s_k,i - sbar_k|; g (if non-NULL) += the gradient
// with weight w per Gaussian (the same reg_term the fused mapping step applies).
__global__ __launch_bounds__(256) void k_loss_reg(const float* __restrict__ S, int64_t n, float w, float lscale,
                                                 float* __restrict__ loss, float* __restrict__ g,
                                                 uint32_t* __restrict__ red) {
  float acc = 0.f;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    float d[3];
    acc += reg_term(S[3 * k], S[3 * k + 1], S[3 * k + 2], w, d);
    if (g) {
      g[3 * k] += d[0];
      g[3 * k + 1] += d[1];
      g[3 * k + 2] += d[2];
    }
  }
  grid_sum(acc, loss, red, true, lscale, 0.f);
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                             const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                                             float eps, float bc1, float bc2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float pi = p[i], mi = m[i], vi = v[i];
    adam_one(pi, mi, vi, g[i], lr, b1, b2, eps, bc1, bc2);
    p[i] = pi;
    m[i] = mi;
    v[i] = vi;
  }
}

// Adam over up to kAdamGroups parameter tensors in one launch (each with its
// own step size): grid row y = group, float4 loads where the group's four
// arrays are 16-byte aligned, then a scalar tail.
__global__ __launch_bounds__(256) void k_adam_multi(AdamGroups a, float b1, float b2, float eps, float bc1, float bc2) {
  const int gi = blockIdx.y;
  const int64_t n = a.off[gi + 1] - a.off[gi];
  float* __restrict__ P = a.p[gi];
  float* __restrict__ M = a.m[gi];
  float* __restrict__ V = a.v[gi];
  const float* __restrict__ G = a.g[gi];
  const float lr = a.lr[gi];
  const bool vec = ((reinterpret_cast<uintptr_t>(P) | reinterpret_cast<uintptr_t>(M) | reinterpret_cast<uintptr_t>(V) |
                     reinterpret_cast<uintptr_t>(G)) & 15u) == 0;
  const int64_t n4 = vec ? n / 4 : 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    float4 p = reinterpret_cast<float4*>(P)[i], m = reinterpret_cast<float4*>(M)[i];
    float4 v = reinterpret_cast<float4*>(V)[i];
    const float4 g = reinterpret_cast<const float4*>(G)[i];
    adam_one(p.x, m.x, v.x, g.x, lr, b1, b2, eps, bc1, bc2);
    adam_one(p.y, m.y, v.y, g.y, lr, b1, b2, eps, bc1, bc2);
    adam_one(p.z, m.z, v.z, g.z, lr, b1, b2, eps, bc1, bc2);
    adam_one(p.w, m.w, v.w, g.w, lr, b1, b2, eps, bc1, bc2);
    reinterpret_cast<float4*>(P)[i] = p;
    reinterpret_cast<float4*>(M)[i] = m;
    reinterpret_cast<float4*>(V)[i] = v;
  }
  for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    float p = P[i], m = M[i], v = V[i];
    adam_one(p, m, v, G[i], lr, b1, b2, eps, bc1, bc2);
    P[i] = p;
    M[i] = m;
    V[i] = v;
  }
}

// Adam on the 7 pose parameters (q: lr_q, t: lr_t) with the step count kept
// on the device, so a captured graph can run many iterations. state = [m(8),
// v(8), step(1)].
__global__ void k_pose_adam(float* __restrict__ pose, float* __restrict__ state, const float* __restrict__ g,
                            float lr_q, float lr_t, float b1, float b2, float eps) {
  const int i = threadIdx.x;
  const float t = state[16] + 1.f;
  __syncthreads();
  if (i < 7) pose_adam_elem(pose, state, i, g[i], t, lr_q, lr_t, b1, b2, eps);
  __syncthreads();
  if (i == 0) state[16] = t;
}

// Constant-speed initialisation (Eq. 13) on (q, t): t = 2 t1 - t0; q =
// normalise(2 q1 - q0') with q0 flipped into q1's hemisphere.
__global__ void k_pose_const_velocity(const float* __restrict__ p0, const float* __restrict__ p1,
                                      float* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const float dot = p0[0] * p1[0] + p0[1] * p1[1] + p0[2] * p1[2] + p0[3] * p1[3];
  const float sgn = dot < 0.f ? -1.f : 1.f;
  float q[4], n2 = 0.f;
  for (int i = 0; i < 4; ++i) {
    q[i] = 2.f * p1[i] - sgn * p0[i];
    n2 += q[i] * q[i];
  }
  const float inv = n2 > 0.f ? 1.f / sqrtf(n2) : 0.f;
  for (int i = 0; i < 4; ++i) out[i] = n2 > 0.f ? q[i] * inv : p1[i];
  for (int i = 4; i < 7; ++i) out[i] = 2.f * p1[i] - p0[i];
}

// Left perturbation of a pose by a twist xi = (rho, phi): R' = Exp(phi) R,
// t' = Exp(phi) t + rho; the quaternion is dq * q / |q| with dq the unit
// quaternion of the rotation vector phi.
__global__ void k_pose_apply_twist(const float* __restrict__ pose, const float* __restrict__ xi,
                                   float* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const float px = xi[3], py = xi[4], pz = xi[5];
  const float th = sqrtf(px * px + py * py + pz * pz);
  const float h = 0.5f * th;
  const float sc = th > 1e-12f ? sinf(h) / th : 0.5f;
  const float dw = cosf(h), dx = sc * px, dy = sc * py, dz = sc * pz;
  float qw = pose[0], qx = pose[1], qy = pose[2], qz = pose[3];
  const float n = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  const float in = n > 0.f ? 1.f / n : 0.f;
  qw *= in; qx *= in; qy *= in; qz *= in;
  out[0] = dw * qw - dx * qx - dy * qy - dz * qz;
  out[1] = dw * qx + dx * qw + dy * qz - dz * qy;
  out[2] = dw * qy - dx * qz + dy * qw + dz * qx;
  out[3] = dw * qz + dx * qy - dy * qx + dz * qw;
  float R[9];
  quat_rot(dw, dx, dy, dz, R);
  for (int i = 0; i < 3; ++i) out[4 + i] = R[3 * i] * pose[4] + R[3 * i + 1] * pose[5] + R[3 * i + 2] * pose[6] + xi[i];
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

unsigned grid_for(int64_t n, int64_t cap) {
  int64_t b = (n + 255) / 256;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

int64_t reduce_temp_words() { return kRedWords; }

void launch_loss_l1(const float* C, const float* D, const float* Ct, const float* Dt, int64_t P, float wc, float wd,
                    float* loss, float* gC, float* gD, uint32_t* red, hipStream_t s) {
  if (P <= 0) {
    launch_fill_f32(loss, 0.f, 1, s);
    return;
  }
  const bool vec = P % 4 == 0 && aligned16(C) && aligned16(D) && aligned16(Ct) && aligned16(Dt) && aligned16(gC) &&
                   aligned16(gD);
  const int64_t P4 = vec ? P / 4 : 0;
  hipLaunchKernelGGL(k_loss_l1, dim3(grid_for(vec ? P4 : P, kRedSlots)), dim3(256), 0, s, C, D, Ct, Dt, P, P4,
                     wc / (3.f * (float)P), wd / (float)P, loss, gC, gD, red);
}

void launch_loss_ssim(const float* X, const float* Y, int H, int W, float weight, float* loss, float* gX,
                      uint32_t* red, hipStream_t s) {
  if (H <= 0 || W <= 0) return;  // an empty image adds nothing
  SsimWin win;
  double g[kSsTaps], sum = 0.0;
  for (int k = 0; k < kSsTaps; ++k) {
    const double d = k - kSsR;
    g[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += g[k];
  }
  for (int k = 0; k < kSsTaps; ++k) win.w[k] = (float)(g[k] / sum);
  const int tiles_x = (W + kSsT - 1) / kSsT, tiles_y = (H + kSsT - 1) / kSsT;
  const int n_tiles = tiles_x * tiles_y;
  const double n = 3.0 * (double)H * (double)W;
  const int grid = 3 * n_tiles < kRedSlots ? 3 * n_tiles : kRedSlots;
  hipLaunchKernelGGL(k_loss_ssim, dim3(grid), dim3(256), 0, s, X, Y, H, W, tiles_x, n_tiles, win,
                     (float)(-weight / n), (float)(-weight / n), weight, loss, gX, red);
}

void launch_loss_reg(const float* scales, int64_t n, float weight, float* loss, float* g, uint32_t* red,
                     hipStream_t s) {
  if (n <= 0) return;  // nothing to add
  const float w = (float)((double)weight / (double)n);
  hipLaunchKernelGGL(k_loss_reg, dim3(grid_for(n, 2048)), dim3(256), 0, s, scales, n, w, w, loss, g, red);
}

int64_t track_temp_words() { return kSelWords + kRedWords; }

void launch_loss_track(const float* C, const float* D, const float* A, const float* Ct, const float* Dt, int64_t P,
                       float lambda_c, float inlier_mult, float* loss, float* gC, float* gD, float* median,
                       uint32_t* temp, hipStream_t s) {
  if (P <= 0) {
    launch_fill_f32(loss, 0.f, 1, s);
    return;
  }
  // temp's histograms are zero here: cleared when allocated and by the loss
  // kernel of the previous call, after its last read
  const unsigned g = grid_for(P, 256);
  for (int pass = 0; pass < kSelPasses; ++pass)
    hipLaunchKernelGGL(k_select_hist, dim3(g), dim3(256), 0, s, D, Dt, P, pass, temp);
  hipLaunchKernelGGL(k_loss_track, dim3(grid_for(P, kRedSlots)), dim3(256), 0, s, C, D, A, Ct, Dt, P, lambda_c,
                     inlier_mult, temp, loss, gC, gD, median, temp + kSelWords);
}

void launch_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                 float bc1, float bc2, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n, 4096)), dim3(256), 0, s, p, m, v, g, n, lr, b1, b2, eps, bc1, bc2);
}

}  // namespace gsr

namespace gsr {
void launch_pose_adam(float* pose, float* state, const float* g, float lr_q, float lr_t, float b1, float b2, float eps,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_pose_adam, dim3(1), dim3(64), 0, s, pose, state, g, lr_q, lr_t, b1, b2, eps);
}
void launch_adam_multi(const AdamGroups& a, float b1, float b2, float eps, float bc1, float bc2, hipStream_t s) {
  if (a.n <= 0 || a.off[a.n] <= 0) return;
  int64_t most = 0;
  for (int i = 0; i < a.n; ++i) most = std::max<int64_t>(most, a.off[i + 1] - a.off[i]);
  hipLaunchKernelGGL(k_adam_multi, dim3(grid_for((most + 3) / 4, 2048), (unsigned)a.n), dim3(256), 0, s, a, b1, b2,
                     eps, bc1, bc2);
}
void launch_pose_const_velocity(const float* p0, const float* p1, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pose_const_velocity, dim3(1), dim3(64), 0, s, p0, p1, out);
}
void launch_pose_apply_twist(const float* pose, const float* xi, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pose_apply_twist, dim3(1), dim3(64), 0, s, pose, xi, out);
}
}  // namespace gsr
