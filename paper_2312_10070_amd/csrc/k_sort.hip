// Tile binning. The projection counts, per tile, the Gaussians whose tile
// rectangle holds it; an exclusive scan of those counts gives each tile's
// [start, end) range in the overlap list (and the overlap count K). Every
// (Gaussian, tile) pair then takes a slot of its tile's range with an atomic
// counter and writes the key (float bits of the camera depth << 32 | record
// index); the slot order is arbitrary. Finally one workgroup per tile sorts
// its range by key in LDS (a bitonic network; a range longer than LDS holds
// is sorted in LDS-sized runs that are merged pairwise in global memory) and
// writes the record indices. Keys are unique within a tile, so the result is
// the depth order of the "m ordered Gaussians" of Eq. 3 and Eq. 6 with ties
// broken by index: exactly what a stable sort of (tile, depth) gives.
// No launch grid depends on K: positions at or beyond the capacity are
// dropped and flagged, so the same launches serve captured graphs.
#include "gsr_internal.h"

namespace gsr {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048


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

constexpr int kSortCap = 2048;  // keys a workgroup sorts in LDS (16 KB)
constexpr int kBinThreads = 256;

__global__ __launch_bounds__(256) void k_bin_gather(const uint32_t* __restrict__ cnt, int64_t n_items,
                                                   uint32_t* __restrict__ cntT) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // = item * kBinCopies + copy
  if (i >= n_items * kBinCopies) return;
  const int64_t t = i / kBinCopies, c = i - t * kBinCopies;
  cntT[i] = cnt[c * n_items + t];
}

// ranges[t] = [start of copy 0, end of the last copy) clipped to the
// capacity; fill[c][t] = start of copy c's sub-range.
__global__ __launch_bounds__(256) void k_tile_init(const uint32_t* __restrict__ cntT,
                                                  const uint32_t* __restrict__ startT, int64_t n_items, int64_t cap,
                                                  int2* __restrict__ ranges, uint32_t* __restrict__ fill) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_items) return;
  const int64_t b = t * kBinCopies;
  const int64_t s0 = startT[b], s1 = (int64_t)startT[b + kBinCopies - 1] + cntT[b + kBinCopies - 1];
  ranges[t] = make_int2((int)(s0 < cap ? s0 : cap), (int)(s1 < cap ? s1 : cap));
  for (int c = 0; c < kBinCopies; ++c) fill[c * n_items + t] = startT[b + c];
}

// One thread per (view, Gaussian): a slot in every tile of its rectangle.
__global__ __launch_bounds__(256) void k_tile_place(Raster Rr, PlaceArgs a) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // view * n + Gaussian
  if (o >= a.n * a.n_views) return;
  if (a.counts[o] == 0) return;
  const int4 r = a.rect[o];
  const uint64_t key_lo = (uint64_t)(uint32_t)o;
  const uint64_t zb = (uint64_t)__float_as_uint(a.rec_rgbz[o].w) << 32;
  const int64_t view = o / a.n;
  uint32_t* fill = a.fill + bin_copy(o - view * a.n) * a.n_items + view * Rr.n_tiles;
  for (int ty = r.y; ty <= r.w; ++ty)
    for (int tx = r.x; tx <= r.z; ++tx) {
      const uint32_t pos = atomicAdd(fill + ty * Rr.ntx + tx, 1u);
      if ((int64_t)pos < a.cap) {
        a.keys[pos] = zb | key_lo;
      } else {
        atomicOr(a.overflow, 1);
      }
    }
}

// Bitonic sort of s[0, n2) ascending (n2 a power of two <= kSortCap), all
// threads of the workgroup; ends with a barrier.
__device__ __forceinline__ void lds_bitonic(uint64_t* s, int n2) {
  const int half = n2 >> 1;
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int p = threadIdx.x; p < half; p += kBinThreads) {
        const int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));  // pairs (i, i + j) with bit j of i clear
        const int l = i + j;
        const uint64_t x = s[i], y = s[l];
        const bool up = (i & k) == 0;
        if ((x > y) == up) {
          s[i] = y;
          s[l] = x;
        }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ int pow2_at_least(int v) {
  int n = 2;
  while (n < v) n <<= 1;
  return n;
}

// Sorts keys[b, b + len) (len <= kSortCap) through LDS; writes the sorted keys
// to out_keys (may alias keys) and/or their low words to out_ids.
__device__ void sort_run(const uint64_t* keys, int64_t b, int len, uint64_t* s, uint64_t* out_keys,
                         uint32_t* out_ids) {
  const int n2 = pow2_at_least(len);
  for (int i = threadIdx.x; i < n2; i += kBinThreads) s[i] = i < len ? keys[b + i] : ~0ull;
  __syncthreads();
  lds_bitonic(s, n2);
  for (int i = threadIdx.x; i < len; i += kBinThreads) {
    if (out_keys) out_keys[b + i] = s[i];
    if (out_ids) out_ids[b + i] = (uint32_t)s[i];
  }
  __syncthreads();
}

// Merges the sorted runs a[0, na) and b[0, nb) (distinct keys) into out; the
// output is split evenly over the workgroup's threads by merge-path search.
__device__ void merge_runs(const uint64_t* a, int na, const uint64_t* b, int nb, uint64_t* out) {
  const int total = na + nb;
  const int per = (total + kBinThreads - 1) / kBinThreads;
  const int d0 = min(total, (int)threadIdx.x * per), d1 = min(total, d0 + per);
  if (d0 >= d1) return;
  int lo = max(0, d0 - nb), hi = min(d0, na);
  while (lo < hi) {  // the first i with a[i] > b[d0 - 1 - i]
    const int mid = (lo + hi) >> 1;
    if (a[mid] < b[d0 - 1 - mid]) lo = mid + 1;
    else hi = mid;
  }
  int i = lo, j = d0 - lo;
  for (int d = d0; d < d1; ++d) {
    const bool take_a = j >= nb || (i < na && a[i] < b[j]);
    out[d] = take_a ? a[i++] : b[j++];
  }
}

// One workgroup per (view, tile) item.
__global__ __launch_bounds__(kBinThreads) void k_tile_sort(const int2* __restrict__ ranges, uint64_t* __restrict__ keys,
                                                          uint64_t* __restrict__ scratch, uint32_t* __restrict__ ids) {
  __shared__ uint64_t s[kSortCap];
  const int2 rg = ranges[blockIdx.x];
  const int64_t b = rg.x;
  const int len = rg.y - rg.x;
  if (len <= 0) return;
  if (len <= kSortCap) {
    sort_run(keys, b, len, s, nullptr, ids);
    return;
  }
  // long range: sorted runs of kSortCap, then pairwise merges (ping-pong)
  for (int c0 = 0; c0 < len; c0 += kSortCap) sort_run(keys, b + c0, min(kSortCap, len - c0), s, keys, nullptr);
  uint64_t* src = keys + b;
  uint64_t* dst = scratch + b;
  for (int w = kSortCap; w < len; w <<= 1) {
    for (int lo = 0; lo < len; lo += 2 * w) {
      const int mid = min(lo + w, len), hi = min(lo + 2 * w, len);
      merge_runs(src + lo, mid - lo, src + mid, hi - mid, dst + lo);
    }
    __threadfence_block();
    __syncthreads();
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  for (int i = threadIdx.x; i < len; i += kBinThreads) ids[b + i] = (uint32_t)src[i];
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

void launch_bin_gather(const uint32_t* tile_cnt, int64_t n_items, uint32_t* cntT, hipStream_t s) {
  const int64_t m = n_items * kBinCopies;
  if (m <= 0) return;
  hipLaunchKernelGGL(k_bin_gather, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, tile_cnt, n_items, cntT);
}

void launch_tile_bins(const Raster& R, const PlaceArgs& a, const uint32_t* cntT, const uint32_t* startT,
                      int64_t n_items, int2* ranges, uint64_t* scratch, uint32_t* ids, hipStream_t s) {
  if (n_items <= 0) return;
  hipLaunchKernelGGL(k_tile_init, dim3((unsigned)((n_items + 255) / 256)), dim3(256), 0, s, cntT, startT,
                     n_items, a.cap, ranges, a.fill);
  const int64_t m = a.n * a.n_views;
  if (m > 0)
    hipLaunchKernelGGL(k_tile_place, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, R, a);
  hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)n_items), dim3(kBinThreads), 0, s, (const int2*)ranges, a.keys,
                     scratch, ids);
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
