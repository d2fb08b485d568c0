// Seeding (Sec. 3.2): candidate points sampled from a keyframe, and the
// neighbour queries that decide which become new Gaussians.
//
// Candidates: a pixel with positive depth is chosen by Bernoulli thinning with
// caller-supplied random numbers u: for a sub-map's first keyframe iff
// u < p_uniform (+ p_grad where the grey image's central-difference gradient
// exceeds a threshold), afterwards iff the rendered alpha < alpha_n and
// u < p_uniform; chosen pixels are back-projected through the pinhole and the
// inverse of the world-to-camera pose, and compacted in pixel order.
//
// Neighbour queries of the seeding step (Sec. 3.2: a sampled point becomes a
// new Gaussian only if no Gaussian of the active sub-map lies within the
// search radius rho; the supplement sets the new Gaussian's scale from its
// nearest-neighbour distance in the sub-map).
//
// A spatial hash grid over the sub-map's means answers both with one search:
// the cell edge h is r_max (1 + 1e-3), so every mean within r_max of a query
// lies in the 27 cells around the query's cell, whatever the rounding of the
// cell index (cell coordinates below 8192 in magnitude keep that rounding
// under 1e-3 of a cell). The squared distance (dx^2 + dy^2) + dz^2 is evaluated without
// contraction, and the minimum is exact, so results do not depend on the
// order in which the grid is filled.
#include "gsr_internal.h"

namespace gsr {

namespace {

__device__ __forceinline__ int cell_of(float x, float inv_h) {
  return (int)floorf(fminf(fmaxf(x * inv_h, -1.0e9f), 1.0e9f));
}

__device__ __forceinline__ uint32_t bucket_of(int cx, int cy, int cz, uint32_t mask) {
  const uint32_t h = (uint32_t)cx * 73856093u ^ (uint32_t)cy * 19349663u ^ (uint32_t)cz * 83492791u;
  return (h ^ (h >> 15)) & mask;
}

__device__ __forceinline__ float dist2(float ax, float ay, float az, float bx, float by, float bz) {
#pragma clang fp contract(off)
  const float dx = ax - bx, dy = ay - by, dz = az - bz;
  return (dx * dx + dy * dy) + dz * dz;
}

__global__ __launch_bounds__(256) void k_grid_count(const float* __restrict__ p, int64_t n, float inv_h,
                                                  uint32_t mask, uint32_t* __restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t b = bucket_of(cell_of(p[3 * i], inv_h), cell_of(p[3 * i + 1], inv_h), cell_of(p[3 * i + 2], inv_h),
                               mask);
  atomicAdd(&counts[b], 1u);
}

// cursor: zero on entry; pts[offsets[b] + k] = the k-th mean that reached bucket b
__global__ __launch_bounds__(256) void k_grid_fill(const float* __restrict__ p, int64_t n, float inv_h, uint32_t mask,
                                                 const uint32_t* __restrict__ offsets, uint32_t* __restrict__ cursor,
                                                 float4* __restrict__ pts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = p[3 * i], y = p[3 * i + 1], z = p[3 * i + 2];
  const uint32_t b = bucket_of(cell_of(x, inv_h), cell_of(y, inv_h), cell_of(z, inv_h), mask);
  const uint32_t slot = offsets[b] + atomicAdd(&cursor[b], 1u);
  pts[slot] = make_float4(x, y, z, 0.f);
}

// offsets: T + 1 words, bucket b's means are pts[offsets[b], offsets[b + 1]).
// Workgroups are dealt to the 8 XCDs in turn; xcd_tile gives each XCD a
// contiguous run of queries (candidates come in pixel order, so a run covers a
// band of the image and its XCD's L2 holds the part of the grid it needs).
__global__ __launch_bounds__(256) void k_seed_query(const float* __restrict__ q, int64_t m, float inv_h, uint32_t mask,
                                                  const uint32_t* __restrict__ offsets,
                                                  const float4* __restrict__ pts, float r2max, float rho2,
                                                  float* __restrict__ nn_d2, int32_t* __restrict__ keep) {
  const int64_t j = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const float x = q[3 * j], y = q[3 * j + 1], z = q[3 * j + 2];
  const int cx = cell_of(x, inv_h), cy = cell_of(y, inv_h), cz = cell_of(z, inv_h);
  float best = r2max;
  // a 3x3 slice of cells at a time: its nine bucket ranges are loaded
  // together, then each bucket's means four per step, so that several loads
  // are in flight (a step past a bucket's end repeats its first mean of the
  // step; the minimum is exact, so neither that nor the order matters)
  for (int dz = -1; dz <= 1; ++dz) {
    uint32_t s[9], e[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const uint32_t b = bucket_of(cx + t % 3 - 1, cy + t / 3 - 1, cz + dz, mask);
      s[t] = offsets[b];
      e[t] = offsets[b + 1];
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const uint32_t end = e[t];
      for (uint32_t k = s[t]; k < end; k += 4) {
        const float4 p0 = pts[k];
        const float4 p1 = pts[k + 1 < end ? k + 1 : k];
        const float4 p2 = pts[k + 2 < end ? k + 2 : k];
        const float4 p3 = pts[k + 3 < end ? k + 3 : k];
        best = fminf(best, dist2(x, y, z, p0.x, p0.y, p0.z));
        best = fminf(best, dist2(x, y, z, p1.x, p1.y, p1.z));
        best = fminf(best, dist2(x, y, z, p2.x, p2.y, p2.z));
        best = fminf(best, dist2(x, y, z, p3.x, p3.y, p3.z));
      }
    }
  }
  if (nn_d2) nn_d2[j] = best;
  if (keep) keep[j] = best < rho2 ? 0 : 1;
}

__device__ __forceinline__ float grey(const float* C, int64_t P, int64_t i) {
#pragma clang fp contract(off)
  return __fdiv_rn((C[i] + C[P + i]) + C[2 * P + i], 3.f);
}

__device__ __forceinline__ bool seed_pick(const SeedSample& a, int64_t i) {
#pragma clang fp contract(off)
  if (!(a.depth[i] > 0.f)) return false;
  if (a.alpha) return a.alpha[i] < a.alpha_n && a.u[i] < a.p_uniform;
  const int y = (int)(i / a.W), x = (int)(i - (int64_t)y * a.W);
  bool edge = false;
  if (x > 0 && x < a.W - 1 && y > 0 && y < a.H - 1) {
    const int64_t P = (int64_t)a.W * a.H;
    const float gx = grey(a.color, P, i + 1) - grey(a.color, P, i - 1);
    const float gy = grey(a.color, P, i + a.W) - grey(a.color, P, i - a.W);
    edge = gx * gx + gy * gy > a.g2thre;
  }
  return a.u[i] < (edge ? a.p_uniform + a.p_grad : a.p_uniform);
}

__global__ __launch_bounds__(256) void k_seed_flag(SeedSample a, uint32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)a.W * a.H) flag[i] = seed_pick(a, i) ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_seed_emit(SeedSample a, const uint32_t* __restrict__ flag,
                                                 const uint32_t* __restrict__ off, float* __restrict__ points,
                                                 float* __restrict__ colors) {
  const int64_t P = (int64_t)a.W * a.H;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P || !flag[i]) return;
  const int y = (int)(i / a.W), x = (int)(i - (int64_t)y * a.W);
  const float d = a.depth[i];
  const float xc = ((float)x - a.cx) * d / a.fx, yc = ((float)y - a.cy) * d / a.fy;
  // world-to-camera (q, t): X_w = R^T (X_c - t)
  float qw = a.pose7[0], qx = a.pose7[1], qy = a.pose7[2], qz = a.pose7[3];
  const float inv = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= inv; qx *= inv; qy *= inv; qz *= inv;
  const float r00 = 1.f - 2.f * (qy * qy + qz * qz), r01 = 2.f * (qx * qy - qw * qz), r02 = 2.f * (qx * qz + qw * qy);
  const float r10 = 2.f * (qx * qy + qw * qz), r11 = 1.f - 2.f * (qx * qx + qz * qz), r12 = 2.f * (qy * qz - qw * qx);
  const float r20 = 2.f * (qx * qz - qw * qy), r21 = 2.f * (qy * qz + qw * qx), r22 = 1.f - 2.f * (qx * qx + qy * qy);
  const float vx = xc - a.pose7[4], vy = yc - a.pose7[5], vz = d - a.pose7[6];
  const int64_t j = off[i];
  points[3 * j] = r00 * vx + r10 * vy + r20 * vz;
  points[3 * j + 1] = r01 * vx + r11 * vy + r21 * vz;
  points[3 * j + 2] = r02 * vx + r12 * vy + r22 * vz;
  colors[3 * j] = a.color[i];
  colors[3 * j + 1] = a.color[P + i];
  colors[3 * j + 2] = a.color[2 * P + i];
}

__global__ __launch_bounds__(256) void k_seed_keep_flag(const int32_t* __restrict__ keep, int64_t m,
                                                       uint32_t* __restrict__ flag) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) flag[j] = keep[j] != 0 ? 1u : 0u;
}

// Correctly rounded FP32 square root of x: the hardware estimate, then moved
// to the neighbour whose rounding interval holds sqrt(x). The tests are exact
// in FP64 (a midpoint between adjacent floats has 25 significant bits, its
// square at most 50), and sqrt(x) never lies on a midpoint.
__device__ __forceinline__ float sqrt_rn(float x) {
  float s = sqrtf(x);
  if (!(x > 0.f) || !(s < INFINITY)) return s;
  const double dx = (double)x;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const float up = __uint_as_float(__float_as_uint(s) + 1u), dn = __uint_as_float(__float_as_uint(s) - 1u);
    const double mhi = 0.5 * ((double)s + (double)up), mlo = 0.5 * ((double)s + (double)dn);
    if (mhi * mhi < dx) s = up;
    else if (mlo * mlo > dx) s = dn;
  }
  return s;
}

// New Gaussian at row off[j] for every kept point j: mean = the point, colour
// = its pixel colour, scale = the nearest-neighbour distance on all three axes
// (correctly rounded square root of nn_d2), identity rotation, opacity 0.5.
__global__ __launch_bounds__(256) void k_seed_init(SeedInit a, const uint32_t* __restrict__ flag,
                                                 const uint32_t* __restrict__ off) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.m || !flag[j]) return;
  const int64_t r = off[j];
  const float s = sqrt_rn(a.nn_d2[j]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a.means[3 * r + k] = a.points[3 * j + k];
    a.scales[3 * r + k] = s;
    a.colors[3 * r + k] = a.pcolors[3 * j + k];
  }
  reinterpret_cast<float4*>(a.quats)[r] = make_float4(1.f, 0.f, 0.f, 0.f);
  a.opacities[r] = 0.5f;
}

}  // namespace

int64_t seed_init_temp_words(int64_t m) { return 2 * m + 1 + scan_temp_words(m); }

void launch_seed_init(const SeedInit& a, uint32_t* temp, uint32_t* count_host, hipStream_t s) {
  uint32_t* flag = temp;
  uint32_t* off = temp + a.m;
  uint32_t* total = temp + 2 * a.m;
  const unsigned g = (unsigned)((a.m + 255) / 256);
  if (a.m > 0) hipLaunchKernelGGL(k_seed_keep_flag, dim3(g), dim3(256), 0, s, a.keep, a.m, flag);
  launch_exclusive_scan(flag, off, a.m, total, total + 1, s, count_host);
  if (a.m > 0) hipLaunchKernelGGL(k_seed_init, dim3(g), dim3(256), 0, s, a, flag, off);
}

int64_t seed_sample_temp_words(int64_t P) { return 2 * P + 1 + scan_temp_words(P); }

void launch_seed_sample(const SeedSample& a, float* points, float* colors, uint32_t* temp, uint32_t* count_host,
                        hipStream_t s) {
  const int64_t P = (int64_t)a.W * a.H;
  uint32_t* flag = temp;
  uint32_t* off = temp + P;
  uint32_t* total = temp + 2 * P;
  const unsigned g = (unsigned)((P + 255) / 256);
  if (P > 0) hipLaunchKernelGGL(k_seed_flag, dim3(g), dim3(256), 0, s, a, flag);
  launch_exclusive_scan(flag, off, P, total, total + 1, s, count_host);
  if (P > 0) hipLaunchKernelGGL(k_seed_emit, dim3(g), dim3(256), 0, s, a, flag, off, points, colors);
}

uint32_t seed_buckets(int64_t n) {
  uint32_t t = 1024;
  while ((int64_t)t < 2 * n && t < (1u << 30)) t <<= 1;
  return t;
}

// words before the float4 point array, rounded up to 16 bytes
static int64_t seed_pts_offset(int64_t T) { return (3 * T + 1 + scan_temp_words(T) + 3) & ~(int64_t)3; }

int64_t seed_temp_words(int64_t n) { return seed_pts_offset(seed_buckets(n)) + 4 * n; }

// the cell edge h = r_max (1 + 1e-3) as its reciprocal
static float seed_inv_h(float r_max) { return (float)(1.0 / ((double)r_max * 1.001)); }

void launch_seed_grid(const float* means, int64_t n, float r_max, uint32_t* temp, hipStream_t s) {
  const uint32_t T = seed_buckets(n);
  uint32_t* counts = temp;
  uint32_t* cursor = temp + T;
  uint32_t* offsets = temp + 2 * (int64_t)T;
  uint32_t* total = offsets + T;  // offsets[T] = n
  uint32_t* scan_tmp = total + 1;
  float4* pts = reinterpret_cast<float4*>(temp + seed_pts_offset(T));
  const float inv_h = seed_inv_h(r_max);
  const uint32_t mask = T - 1;
  launch_fill_u32(counts, 0u, T, s);
  launch_fill_u32(cursor, 0u, T, s);
  const unsigned gn = (unsigned)((n + 255) / 256);
  if (n > 0) hipLaunchKernelGGL(k_grid_count, dim3(gn), dim3(256), 0, s, means, n, inv_h, mask, counts);
  launch_exclusive_scan(counts, offsets, T, total, scan_tmp, s);
  if (n > 0) hipLaunchKernelGGL(k_grid_fill, dim3(gn), dim3(256), 0, s, means, n, inv_h, mask, offsets, cursor, pts);
}

void launch_seed_query(int64_t n, const float* points, int64_t m, float rho, float r_max, float* nn_d2,
                       int32_t* keep, const uint32_t* temp, hipStream_t s) {
  const uint32_t T = seed_buckets(n);
  const uint32_t* offsets = temp + 2 * (int64_t)T;
  const float4* pts = reinterpret_cast<const float4*>(temp + seed_pts_offset(T));
  const float r2max = r_max * r_max, rho2 = rho * rho;
  const unsigned gm = (unsigned)((m + 255) / 256);
  if (m > 0)
    hipLaunchKernelGGL(k_seed_query, dim3(gm), dim3(256), 0, s, points, m, seed_inv_h(r_max), T - 1, offsets, pts,
                       r2max, rho2, nn_d2, keep);
}

}  // namespace gsr
