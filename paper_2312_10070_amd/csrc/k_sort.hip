// Tile binning in two passes. Each binning workgroup owns a contiguous run of
// Gaussians and counts their (Gaussian, tile) pairs per tile in an LDS
// histogram; for every tile it meets it reserves a sub-range of the tile's
// range with one atomic on the tile's total and keeps the offset in column w
// of a [tile][workgroup] matrix M. The last workgroup to finish scans the
// tile totals into the tiles' [start, end) ranges and the overlap count K
// (and zeroes the totals for the next launch). The placing workgroup then
// walks its Gaussians again, takes positions from LDS counters seeded with
// start + its offset, and writes the keys (float bits of the camera depth <<
// 32 | record index) in arbitrary order. Finally each
// tile's range is sorted by key and its record indices written: by one wave
// in registers (a bitonic network of up to 2048 keys), or for longer ranges
// by the waves of a workgroup side by side (runs of 1024 keys, merged
// pairwise in global memory). Keys are unique within a
// tile, so the result is the depth order of the "m ordered Gaussians" of
// Eq. 3 and Eq. 6 with ties broken by index: exactly what a stable sort of
// (tile, depth) gives. No launch grid depends on K: positions at or beyond
// the capacity are dropped and flagged, so the same launches serve captured
// graphs.
#include "gsr_internal.h"

namespace gsr {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048


// Gaussians whose rectangles a binning thread loads together (the loads are
// in flight at once instead of one round trip per Gaussian).
constexpr int kRectBatch = 4;

// rect of Gaussians g0 + j blockDim.x (j < kRectBatch) of view `view`, zero
// past g1; every load is issued before any value is used.
__device__ __forceinline__ void load_rects(const BinArgs& a, int64_t view, int64_t g0, int64_t g1, int4 (&r)[kRectBatch]) {
  // (indices past g1 load Gaussian g1 - 1 >= g0 and are then zeroed: no branch between the loads)
#pragma unroll
  for (int j = 0; j < kRectBatch; ++j) {
    const int64_t g = g0 + (int64_t)j * blockDim.x;
    r[j] = a.rect[view * a.n + (g < g1 ? g : g1 - 1)];
  }
#pragma unroll
  for (int j = 0; j < kRectBatch; ++j) {
    asm volatile("" : "+v"(r[j].x), "+v"(r[j].y), "+v"(r[j].z), "+v"(r[j].w));
    if (g0 + (int64_t)j * blockDim.x >= g1) r[j] = make_int4(0, 0, 0, 0);
  }
}

// Exclusive scan of v over a workgroup of T threads; *total = the sum.
template <int T>
__device__ __forceinline__ uint32_t block_exclusive_scan_t(uint32_t v, uint32_t* total, uint32_t* s_wave) {
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
  for (int i = 0; i < T / 64; ++i) {
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
  block_exclusive_scan_t<kScanThreads>(s, &tot, s_wave);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// One workgroup scans all partials (exclusive, in place) and writes the total
// (and, if total_host is set, the same word to pinned host memory).
__global__ __launch_bounds__(kScanThreads) void k_scan_partials(uint32_t* __restrict__ partials, int64_t np,
                                                               uint32_t* __restrict__ total,
                                                               uint32_t* __restrict__ total_host) {
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
    uint32_t ex = block_exclusive_scan_t<kScanThreads>(s, &tot, s_wave) + carry;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (base + i < np) partials[base + i] = ex;
      ex += v[i];
    }
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *total = carry;
    if (total_host) *total_host = carry;
  }
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
  uint32_t ex = block_exclusive_scan_t<kScanThreads>(s, &tot, s_wave) + partials[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
}

constexpr int kBinThreads = 256;
// Threads of a counting / placing workgroup: each walks a few of its
// workgroup's Gaussians, so more threads hide more of the memory latency.
constexpr int kPlaceThreads = 1024;

// Tiles one workgroup's LDS histogram covers (64 KB); more tiles per view are
// handled in chunks (grid.z).
constexpr int kBinTileChunk = 16384;

struct Chunk {
  int64_t g0, g1;  // Gaussians of this workgroup
  int t0, nt;      // tiles of this chunk
};

__device__ __forceinline__ Chunk bin_chunk(const Raster& Rr, const BinArgs& a) {
  Chunk c;
  const int64_t per = (a.n + a.n_wg - 1) / a.n_wg;
  c.g0 = (int64_t)blockIdx.x * per;
  c.g1 = c.g0 + per < a.n ? c.g0 + per : a.n;
  c.t0 = (int)blockIdx.z * kBinTileChunk;
  c.nt = min(Rr.n_tiles - c.t0, kBinTileChunk);
  return c;
}

// One workgroup: R[i] = (start, start + T[i]) with start the exclusive scan of
// the tile totals T[0, n) (read at the device-coherent level), T[i] = 0;
// returns the sum.
__device__ uint32_t scan_tile_totals(uint32_t* T, int2* R, int64_t n) {
  __shared__ uint32_t s_wave[kPlaceThreads / 64];
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < n; b0 += (int64_t)kPlaceThreads * kScanItems) {
    const int64_t base = b0 + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      v[i] = base + i < n ? __hip_atomic_load(T + base + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
      sum += v[i];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan_t<kPlaceThreads>(sum, &tot, s_wave) + carry;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (base + i < n) {
        R[base + i] = make_int2((int)ex, (int)(ex + v[i]));
        __hip_atomic_store(T + base + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      ex += v[i];
    }
    carry += tot;
  }
  return carry;
}

// Pairs per (tile, workgroup) in LDS; M[(v n_tiles + t) n_wg + w] = offset of
// workgroup w's pairs inside the range of tile t of view v (reserved with an
// atomic on T, so the order of the workgroups inside a tile is arbitrary).
// The last workgroup writes the ranges R and K.
__global__ __launch_bounds__(kPlaceThreads) void k_bin_count(Raster Rr, BinArgs a) {
  extern __shared__ uint32_t hist[];
  __shared__ bool last;
  const Chunk c = bin_chunk(Rr, a);
  const int64_t view = blockIdx.y;
  for (int i = threadIdx.x; i < c.nt; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  for (int64_t g0 = c.g0 + threadIdx.x; g0 < c.g1; g0 += (int64_t)kRectBatch * blockDim.x) {
    int4 rr[kRectBatch];
    load_rects(a, view, g0, c.g1, rr);
#pragma unroll
    for (int j = 0; j < kRectBatch; ++j) {
      const int4 r = rr[j];
      if (r.w == 0) continue;
      const int tx0 = r.x & 0xffff, tx1 = (int)((uint32_t)r.x >> 16), ty0 = r.y & 0xffff, ty1 = (int)((uint32_t)r.y >> 16);
      for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
          const int t = ty * Rr.ntx + tx - c.t0;
          if ((unsigned)t < (unsigned)c.nt) atomicAdd(&hist[t], 1u);
        }
    }
  }
  __syncthreads();
  const int64_t row = view * Rr.n_tiles + c.t0;
  for (int i = threadIdx.x; i < c.nt; i += blockDim.x) {
    const uint32_t h = hist[i];
    if (h) a.M[(row + i) * a.n_wg + blockIdx.x] = atomicAdd(a.T + row + i, h);
  }
  __syncthreads();  // every reservation of the workgroup has returned
  if (threadIdx.x == 0) {
    const uint32_t n_wg_total = gridDim.x * gridDim.y * gridDim.z;
    const uint32_t t = __hip_atomic_fetch_add(a.ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last = t == n_wg_total - 1;
    if (last) __hip_atomic_store(a.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (!last) return;
  const uint32_t K = scan_tile_totals(a.T, a.R, (int64_t)Rr.n_tiles * a.n_views);
  if (threadIdx.x == 0) {
    *a.K = K;
    if (a.K_host) *a.K_host = K;
  }
}

// Every (Gaussian, tile) pair of the workgroup takes the next position of its
// tile's sub-range (LDS counters seeded with the tile's start + M) and writes
// its key there. Reads R and M only, so it can be repeated with another
// capacity.
__global__ __launch_bounds__(kPlaceThreads) void k_bin_place(Raster Rr, BinArgs a) {
  extern __shared__ uint32_t next[];
  const Chunk c = bin_chunk(Rr, a);
  const int64_t view = blockIdx.y;
  const int64_t row = view * Rr.n_tiles + c.t0;
  // (entries of tiles the workgroup has no pair on are not used)
  for (int i = threadIdx.x; i < c.nt; i += blockDim.x) next[i] = (uint32_t)a.R[row + i].x + a.M[(row + i) * a.n_wg + blockIdx.x];
  // the chunk's tile ranges clipped to the capacity, tiles dealt round-robin
  // over the chunk's workgroups
  for (int i = (int)blockIdx.x + a.n_wg * (int)threadIdx.x; i < c.nt; i += a.n_wg * (int)blockDim.x) {
    const int2 r = a.R[row + i];
    a.ranges[row + i] = make_int2((int)(r.x < a.cap ? r.x : a.cap), (int)(r.y < a.cap ? r.y : a.cap));
  }
  __syncthreads();
  for (int64_t g0 = c.g0 + threadIdx.x; g0 < c.g1; g0 += (int64_t)kRectBatch * blockDim.x) {
    int4 rr[kRectBatch];
    load_rects(a, view, g0, c.g1, rr);
#pragma unroll
    for (int j = 0; j < kRectBatch; ++j) {
      const int4 r = rr[j];
      if (r.w == 0) continue;
      const int64_t o = view * a.n + g0 + (int64_t)j * blockDim.x;
      const uint64_t key = ((uint64_t)(uint32_t)r.z << 32) | (uint64_t)(uint32_t)o;
      const int tx0 = r.x & 0xffff, tx1 = (int)((uint32_t)r.x >> 16), ty0 = r.y & 0xffff, ty1 = (int)((uint32_t)r.y >> 16);
      for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
          const int t = ty * Rr.ntx + tx - c.t0;
          if ((unsigned)t >= (unsigned)c.nt) continue;
          const uint32_t pos = atomicAdd(&next[t], 1u);
          if ((int64_t)pos < a.cap) {
            a.keys[pos] = key;
          } else {
            atomicOr(a.overflow, 1);
          }
        }
    }
  }
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

// Keys a single wave sorts in registers (up to 32 per lane).
constexpr int kWaveSort = 2048;

// The value of lane (lane ^ m) for m in {1, 2, 4, 8, 16, 32}, without LDS:
// DPP quad_perm for 1 and 2, row_half_mirror then quad_perm [3,2,1,0] for 4
// ((i ^ 7) ^ 3 = i ^ 4), row_ror:8 for 8 (a rotation by 8 of a 16-lane row is
// i ^ 8), and v_permlane16_swap / v_permlane32_swap of the value with itself
// for 16 and 32 (the swap leaves the partner row's or half's values in one
// of its two results, picked by the lane's row or half).
__device__ __forceinline__ uint32_t lane_xor32(uint32_t v, int m) {
  const int lane = threadIdx.x & 63;
  switch (m) {
    case 1:
      return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false);
    case 2:
      return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false);
    case 4: {
      const int t = __builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false);
      return (uint32_t)__builtin_amdgcn_update_dpp(0, t, 0x1B, 0xf, 0xf, false);
    }
    case 8:
      return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false);
    case 16: {
      const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
      return ((lane >> 4) & 1) ? p[0] : p[1];
    }
    default: {
      const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
      return (lane & 32) ? p[0] : p[1];
    }
  }
}

__device__ __forceinline__ uint64_t lane_xor64(uint64_t v, int m) {
  const uint32_t lo = lane_xor32((uint32_t)v, m), hi = lane_xor32((uint32_t)(v >> 32), m);
  return ((uint64_t)hi << 32) | lo;
}

// Sorts keys[b, b + len) (0 < len <= 64 E) with one wave: lane l holds
// elements E l .. E l + E - 1 in registers; a bitonic network whose strides
// below E are compare-exchanges inside a lane and whose larger strides
// exchange with lane l ^ (stride / E). Writes the low words (record indices)
// to ids (kKeys false) or the sorted keys to out_keys[b, b + len) (kKeys true).
template <int E, bool kKeys = false>
__device__ void wave_sort(const uint64_t* __restrict__ keys, int64_t b, int len, uint32_t* __restrict__ ids,
                          uint64_t* __restrict__ out_keys = nullptr) {
  const int lane = threadIdx.x & 63;
  uint64_t e[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = E * lane + r;
    e[r] = i < len ? keys[b + i] : ~0ull;  // padding sorts last (keys hold finite depths)
  }
#pragma unroll
  for (int k = 2; k <= 64 * E; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= E) {
        const int m = j / E;
        const bool upper = (lane & m) != 0;  // this lane holds the larger position of each pair
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const bool asc = ((E * lane + r) & k) == 0;
          // (the 512-key network exchanges through DPP / permlane; the larger
          // ones through ds_bpermute, whose code stays smaller)
          const uint64_t p = E == 8 ? lane_xor64(e[r], m) : __shfl_xor(e[r], m, 64);
          // the lower position keeps the minimum of an ascending block, the upper the maximum
          const bool keep_min = asc != upper;
          e[r] = ((e[r] < p) == keep_min) ? e[r] : p;
        }
      } else {
#pragma unroll
        for (int r = 0; r < E; ++r) {
          if ((r & j) == 0) {
            const bool asc = ((E * lane + r) & k) == 0;
            const uint64_t x = e[r], y = e[r | j];
            const bool sw = (x > y) == asc;
            e[r] = sw ? y : x;
            e[r | j] = sw ? x : y;
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = E * lane + r;
    if (i < len) {
      if (kKeys) out_keys[b + i] = e[r];
      else ids[b + i] = (uint32_t)e[r];
    }
  }
}

// Four (view, tile) items per workgroup. Each wave sorts one item of at most
// kWaveSort keys in registers (the smallest of the 512 / 1024 / 2048-key
// networks that holds it). Longer items are cut into runs of kLongRun keys,
// which the workgroup's waves sort side by side into scratch (the 1024-key
// network), and pairwise merges (ping-pong between scratch and keys) join.
__global__ __launch_bounds__(kBinThreads) void k_tile_sort(const int2* __restrict__ ranges, int64_t n_items,
                                                          uint64_t* __restrict__ keys, uint64_t* __restrict__ scratch,
                                                          uint32_t* __restrict__ ids) {
  constexpr int kItems = kBinThreads / 64;
  constexpr int kLongRun = 1024;
  const int64_t item0 = (int64_t)blockIdx.x * kItems;
  const int w = threadIdx.x >> 6;
  if (item0 + w < n_items) {
    const int2 rg = ranges[item0 + w];
    const int len = rg.y - rg.x;
    if (len > 0 && len <= 512) {
      wave_sort<8>(keys, rg.x, len, ids);
    } else if (len > 512 && len <= 1024) {
      wave_sort<16>(keys, rg.x, len, ids);
    } else if (len > 1024 && len <= kWaveSort) {
      wave_sort<32>(keys, rg.x, len, ids);
    }
  }
  // runs of the long items, dealt to the waves in turn
  int n_runs = 0;
  for (int it = 0; it < kItems && item0 + it < n_items; ++it) {
    const int2 rg = ranges[item0 + it];
    const int len = rg.y - rg.x;
    if (len > kWaveSort) n_runs += (len + kLongRun - 1) / kLongRun;
  }
  if (n_runs == 0) return;  // uniform across the workgroup
  for (int j = w; j < n_runs; j += kItems) {
    int r = j;
    for (int it = 0; it < kItems && item0 + it < n_items; ++it) {
      const int2 rg = ranges[item0 + it];
      const int len = rg.y - rg.x;
      const int nr = len > kWaveSort ? (len + kLongRun - 1) / kLongRun : 0;
      if (r < nr) {
        const int c0 = r * kLongRun;
        wave_sort<kLongRun / 64, true>(keys, rg.x + c0, min(kLongRun, len - c0), nullptr, scratch);
        break;
      }
      r -= nr;
    }
  }
  __threadfence_block();
  __syncthreads();
  for (int it = 0; it < kItems && item0 + it < n_items; ++it) {
    const int2 rg = ranges[item0 + it];
    const int64_t b = rg.x;
    const int len = rg.y - rg.x;
    if (len <= kWaveSort) continue;  // uniform across the workgroup
    uint64_t* src = scratch + b;
    uint64_t* dst = keys + b;
    for (int wd = kLongRun; wd < len; wd <<= 1) {
      for (int lo = 0; lo < len; lo += 2 * wd) {
        const int mid = min(lo + wd, len), hi = min(lo + 2 * wd, len);
        merge_runs(src + lo, mid - lo, src + mid, hi - mid, dst + lo);
      }
      __threadfence_block();
      __syncthreads();
      uint64_t* t = src;
      src = dst;
      dst = t;
    }
    for (int i = threadIdx.x; i < len; i += kBinThreads) ids[b + i] = (uint32_t)src[i];
    __syncthreads();
  }
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
                           hipStream_t s, uint32_t* total_host) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, total, 0u, (int64_t)1);
    if (total_host) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, total_host, 0u, (int64_t)1);
    return;
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, temp);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, s, temp, nb, total, total_host);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n, (const uint32_t*)temp);
}

int bin_workgroups(int64_t n) {
  const int64_t w = (n + 1023) / 1024;
  return (int)(w < 1 ? 1 : (w > 128 ? 128 : w));
}

namespace {
dim3 bin_grid(const Raster& R, const BinArgs& a) {
  return dim3((unsigned)a.n_wg, (unsigned)a.n_views, (unsigned)((R.n_tiles + kBinTileChunk - 1) / kBinTileChunk));
}
size_t bin_lds(const Raster& R) { return sizeof(uint32_t) * (size_t)min(R.n_tiles, kBinTileChunk); }
}  // namespace

void launch_bin_count(const Raster& R, const BinArgs& a, hipStream_t s) {
  if (R.n_tiles <= 0 || a.n_views <= 0) {
    launch_fill_u32(a.K, 0u, 1, s);
    if (a.K_host) launch_fill_u32(a.K_host, 0u, 1, s);
    return;
  }
  hipLaunchKernelGGL(k_bin_count, bin_grid(R, a), dim3(kPlaceThreads), bin_lds(R), s, R, a);
}

void launch_tile_bins(const Raster& R, const BinArgs& a, int64_t n_items, int2* ranges, uint64_t* scratch,
                      uint32_t* ids, hipStream_t s) {
  if (n_items <= 0) return;
  BinArgs b = a;
  b.ranges = ranges;
  hipLaunchKernelGGL(k_bin_place, bin_grid(R, b), dim3(kPlaceThreads), bin_lds(R), s, R, b);
  hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)((n_items + kBinThreads / 64 - 1) / (kBinThreads / 64))),
                     dim3(kBinThreads), 0, s, (const int2*)ranges, n_items, a.keys, scratch, ids);
}

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}

void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f32, dim3(fill_blocks(n)), dim3(256), 0, s, p, v, n);
}

// ---- opacity pruning: stable compaction of the Gaussians kept -------------
namespace {
// keep[i] = mask[i] != 0 when a mask is given, else opacity o[i] >= thre (NaN is not kept)
__global__ __launch_bounds__(256) void k_prune_flag(const float* __restrict__ o, const int32_t* __restrict__ mask,
                                                  int64_t n, float thre, uint32_t* __restrict__ keep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keep[i] = (mask ? mask[i] != 0 : o[i] >= thre) ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_prune_scatter(PruneArgs a, int64_t n, const uint32_t* __restrict__ keep,
                                                     const uint32_t* __restrict__ off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !keep[i]) return;
  const int64_t j = off[i];
  constexpr int width[5] = {3, 3, 4, 1, 3};
#pragma unroll
  for (int t = 0; t < 15; ++t) {
    if (!a.in[t]) continue;
    const int w = width[t % 5];
    for (int c = 0; c < w; ++c) a.out[t][w * j + c] = a.in[t][w * i + c];
  }
}
}  // namespace

int64_t prune_temp_words(int64_t n) { return 2 * n + scan_temp_words(n) + 1; }

void launch_prune(const PruneArgs& a, int64_t n, float thre, const int32_t* mask, uint32_t* temp, uint32_t* kept_host,
                  hipStream_t s) {
  uint32_t* keep = temp;
  uint32_t* off = temp + n;
  uint32_t* total = temp + 2 * n;
  uint32_t* scan_tmp = total + 1;
  const unsigned g = (unsigned)((n + 255) / 256);
  if (n > 0) hipLaunchKernelGGL(k_prune_flag, dim3(g), dim3(256), 0, s, a.in[3], mask, n, thre, keep);
  launch_exclusive_scan(keep, off, n, total, scan_tmp, s, kept_host);
  if (n > 0) hipLaunchKernelGGL(k_prune_scatter, dim3(g), dim3(256), 0, s, a, n, keep, off);
}

}  // namespace gsr
