// Tile binning: exclusive scan of per-Gaussian tile counts, duplication into
// 64-bit (tile, depth) keys, a stable least-significant-digit radix sort and
// the per-tile [start, end) ranges. This realises the depth order of the "m
// ordered Gaussians" of Eq. 3 and Eq. 6 per tile. All passes read the
// overlap count K from device memory, so the same launches work with exact
// or capacity-sized grids (the latter for captured graphs).
#include "gsr_internal.h"

namespace gsr {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;  // 2048 keys per workgroup
constexpr int kDigits = 256;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total, uint32_t* s_wave) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_wave[w] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kScanThreads / 64; ++i) {
    if (i < w) base += s_wave[i];
    tot += s_wave[i];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                             uint32_t* __restrict__ partials) {
  __shared__ uint32_t s_wave[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  uint32_t tot;
  block_exclusive_scan(s, &tot, s_wave);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// One workgroup scans all partials (exclusive, in place) and writes the total.
__global__ __launch_bounds__(kScanThreads) void k_scan_partials(uint32_t* __restrict__ partials, int64_t np,
                                                               uint32_t* __restrict__ total) {
  __shared__ uint32_t s_wave[4];
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < np; b0 += kScanTile) {
    const int64_t base = b0 + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      v[i] = (base + i < np) ? partials[base + i] : 0u;
      s += v[i];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(s, &tot, s_wave) + carry;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (base + i < np) partials[base + i] = ex;
      ex += v[i];
    }
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                           int64_t n, const uint32_t* __restrict__ partials) {
  __shared__ uint32_t s_wave[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0u;
    s += v[i];
  }
  uint32_t tot;
  uint32_t ex = block_exclusive_scan(s, &tot, s_wave) + partials[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
}

// One thread per Gaussian: a key per overlapped tile, row-major over its
// rectangle. Key = (tile id) << 32 | float bits of the camera depth (z > 0,
// so the bits order like the values); value = Gaussian index. Writing in
// index order makes the stable sort break depth ties by index.
__global__ __launch_bounds__(256) void k_duplicate(Raster Rr, BinArgs a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // view * n + Gaussian
  if (k >= a.n * a.n_views) return;
  const uint32_t cnt = a.counts[k];
  if (cnt == 0) return;
  const uint64_t off = a.offsets[k];
  if (off + cnt > (uint64_t)a.K_cap) {
    atomicOr(a.overflow, 1);
    return;
  }
  const int4 r = a.rect[k];
  const uint32_t zb = __float_as_uint(a.rec_rgbz[k].w);
  const uint32_t tile_base = (uint32_t)(k / a.n) * (uint32_t)Rr.n_tiles;
  uint64_t* kp = a.keys + off;
  uint32_t* vp = a.vals + off;
  int i = 0;
  for (int ty = r.y; ty <= r.w; ++ty)
    for (int tx = r.x; tx <= r.z; ++tx) {
      const uint32_t tile = tile_base + (uint32_t)(ty * Rr.ntx + tx);
      kp[i] = ((uint64_t)tile << 32) | zb;
      vp[i] = (uint32_t)k;
      ++i;
    }
}

__device__ __forceinline__ uint32_t clamp_K(const uint32_t* d_K, int64_t cap) {
  const uint32_t K = *d_K;
  return (int64_t)K < cap ? K : (uint32_t)cap;
}

// Lanes of the wave holding the same 8-bit digit as this lane (ballot match).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                            const uint32_t* __restrict__ d_K, int64_t cap, int shift,
                                                            uint32_t* __restrict__ hist, int nb) {
  __shared__ uint32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t K = clamp_K(d_K, cap);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const uint64_t lt = (1ull << (threadIdx.x & 63)) - 1ull;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t idx = base + r * kSortThreads + threadIdx.x;
    const bool valid = idx < (int64_t)K;
    const uint32_t d = valid ? (uint32_t)(keys[idx] >> shift) & 0xffu : 0u;
    const uint64_t m = match_digit(d, valid);
    if (valid && (m & lt) == 0) atomicAdd(&h[d], (uint32_t)__popcll(m));
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: element order inside the workgroup is (round, lane) order,
// which is index order, and every rank respects it.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint64_t* __restrict__ kin,
                                                               const uint32_t* __restrict__ vin,
                                                               uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                               const uint32_t* __restrict__ d_K, int64_t cap, int shift,
                                                               const uint32_t* __restrict__ hist, int nb) {
  __shared__ uint32_t run[kDigits];
  __shared__ uint32_t wc[kSortThreads / 64][kDigits];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  run[threadIdx.x] = hist[(int64_t)threadIdx.x * nb + blockIdx.x];
  const uint32_t K = clamp_K(d_K, cap);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
#pragma unroll
    for (int i = 0; i < kSortThreads / 64; ++i) wc[i][threadIdx.x] = 0;
    __syncthreads();
    const int64_t idx = base + r * kSortThreads + threadIdx.x;
    const bool valid = idx < (int64_t)K;
    uint64_t key = 0;
    uint32_t d = 0;
    if (valid) {
      key = kin[idx];
      d = (uint32_t)(key >> shift) & 0xffu;
    }
    const uint64_t m = match_digit(d, valid);
    const uint32_t rank = (uint32_t)__popcll(m & lt);
    if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int i = 0; i < w; ++i) pos += wc[i][d];
      kout[pos] = key;
      vout[pos] = vin[idx];
    }
    __syncthreads();
    run[threadIdx.x] += wc[0][threadIdx.x] + wc[1][threadIdx.x] + wc[2][threadIdx.x] + wc[3][threadIdx.x];
  }
}

// Tiles outside [0, n_ranges) (possible only for stale keys after a capacity
// overflow, which the caller reports) are ignored.
__global__ __launch_bounds__(256) void k_tile_ranges(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ d_K,
                                                    int64_t cap, int2* __restrict__ ranges, int64_t n_ranges) {
  const uint32_t K = clamp_K(d_K, cap);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)K) return;
  const uint32_t t = (uint32_t)(keys[i] >> 32);
  if ((int64_t)t >= n_ranges) return;
  if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != t) ranges[t].x = (int)i;
  if (i == (int64_t)K - 1 || (uint32_t)(keys[i + 1] >> 32) != t) ranges[t].y = (int)(i + 1);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_f32(float* p, float v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

unsigned fill_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

int64_t scan_temp_words(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* temp,
                           hipStream_t s) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, total, 0u, (int64_t)1);
    return;
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, temp);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, s, temp, nb, total);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n, (const uint32_t*)temp);
}

void launch_duplicate(const Raster& R, const BinArgs& a, hipStream_t s) {
  const int64_t m = a.n * a.n_views;
  if (m <= 0) return;
  hipLaunchKernelGGL(k_duplicate, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, R, a);
}

int64_t radix_temp_words(int64_t cap) {
  const int64_t nb = (cap + kSortTile - 1) / kSortTile;
  const int64_t nh = (int64_t)kDigits * (nb > 0 ? nb : 1);
  return nh + scan_temp_words(nh) + 1;
}

int launch_radix_sort(uint64_t* keys[2], uint32_t* vals[2], const uint32_t* d_K, int64_t cap, int bits,
                      uint32_t* temp, hipStream_t s) {
  const int64_t nb = (cap + kSortTile - 1) / kSortTile;
  if (nb == 0) return 0;
  const int64_t nh = (int64_t)kDigits * nb;
  uint32_t* hist = temp;
  uint32_t* stemp = temp + nh;
  uint32_t* total = stemp + scan_temp_words(nh);
  int cur = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, s, (const uint64_t*)keys[cur], d_K,
                       cap, shift, hist, (int)nb);
    launch_exclusive_scan(hist, hist, nh, total, stemp, s);
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0, s, (const uint64_t*)keys[cur],
                       (const uint32_t*)vals[cur], keys[cur ^ 1], vals[cur ^ 1], d_K, cap, shift,
                       (const uint32_t*)hist, (int)nb);
    cur ^= 1;
  }
  return cur;
}

void launch_tile_ranges(const uint64_t* keys, const uint32_t* d_K, int64_t cap, int2* ranges, int64_t n_ranges,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(2 * n_ranges)), dim3(256), 0, s, (uint32_t*)ranges, 0u,
                     2 * n_ranges);
  if (cap <= 0) return;
  hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, keys, d_K, cap, ranges,
                     n_ranges);
}

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}

void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f32, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}

}  // namespace gsr
