// Losses and their upstream gradients (Eq. 9, the L1 part of Eq. 10, and the
// masked tracking loss of Eq. 15), the exact median the inlier mask needs
// (radix select on float bits, all on the device), and Adam.
#include "gsr_internal.h"

namespace gsr {

namespace {

__device__ __forceinline__ float sgnf(float r) { return (float)((r > 0.f) - (r < 0.f)); }

__device__ __forceinline__ void block_add(float v, float* dst) {
  __shared__ float red[4];
  const float s = wave_sum_all(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(dst, red[0] + red[1] + red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_loss_l1(const float* __restrict__ C, const float* __restrict__ D,
                                                const float* __restrict__ Ct, const float* __restrict__ Dt, int64_t P,
                                                float wc3, float wd1, float* __restrict__ loss, float* __restrict__ gC,
                                                float* __restrict__ gD) {
  float acc = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
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
  block_add(acc, loss);
}

// ---- exact lower median of e = |D - D*| over pixels with D* > 0 ----------
// State (uint32 words): [0..255] histogram, [256] prefix, [257] prefix mask,
// [258] remaining rank, [259] number of valid pixels.
constexpr int kSelHist = 0, kSelPrefix = 256, kSelMask = 257, kSelRank = 258, kSelCount = 259;
constexpr int kSelWords = 260;

__global__ void k_select_init(uint32_t* st) {
  for (int i = threadIdx.x; i < kSelWords; i += blockDim.x) st[i] = 0;
}

__global__ __launch_bounds__(256) void k_select_hist(const float* __restrict__ D, const float* __restrict__ Dt, int64_t P,
                                                    int shift, uint32_t* __restrict__ st) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t prefix = st[kSelPrefix], mask = st[kSelMask];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
    if (Dt[i] > 0.f) {
      const uint32_t b = __float_as_uint(fabsf(D[i] - Dt[i]));
      if ((b & mask) == prefix) atomicAdd(&h[(b >> shift) & 0xffu], 1u);
    }
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&st[kSelHist + threadIdx.x], h[threadIdx.x]);
}

// One thread: pick the digit holding the target rank, narrow the prefix.
__global__ void k_select_pick(uint32_t* st, int shift, int first) {
  if (threadIdx.x != 0) return;
  if (first) {
    uint32_t n = 0;
    for (int d = 0; d < 256; ++d) n += st[kSelHist + d];
    st[kSelCount] = n;
    st[kSelRank] = n > 0 ? (n - 1) / 2 : 0;
  }
  uint32_t k = st[kSelRank], c = 0;
  int d = 0;
  for (; d < 256; ++d) {
    const uint32_t h = st[kSelHist + d];
    if (k < c + h) break;
    c += h;
  }
  if (d == 256) d = 255;  // no valid pixel: the median is unused
  st[kSelRank] = k - c;
  st[kSelPrefix] |= (uint32_t)d << shift;
  st[kSelMask] |= 0xffu << shift;
  for (int i = 0; i < 256; ++i) st[kSelHist + i] = 0;
}

__global__ __launch_bounds__(256) void k_loss_track(const float* __restrict__ C, const float* __restrict__ D,
                                                   const float* __restrict__ A, const float* __restrict__ Ct,
                                                   const float* __restrict__ Dt, int64_t P, float lambda_c,
                                                   float inlier_mult, const uint32_t* __restrict__ st,
                                                   float* __restrict__ loss, float* __restrict__ gC,
                                                   float* __restrict__ gD, float* __restrict__ median) {
  const bool any = st[kSelCount] > 0;
  const float med = any ? __uint_as_float(st[kSelPrefix]) : 0.f;
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
  block_add(acc, loss);
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                             const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                                             float eps, float bc1, float bc2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

// Adam over up to kAdamGroups parameter tensors in one launch (each with its
// own step size); the flat index space is the concatenation of the groups.
__global__ __launch_bounds__(256) void k_adam_multi(AdamGroups a, float b1, float b2, float eps, float bc1, float bc2) {
  const int64_t total = a.off[a.n];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    int gi = 0;
    while (gi + 1 < a.n && i >= a.off[gi + 1]) ++gi;
    const int64_t j = i - a.off[gi];
    const float g = a.g[gi][j];
    const float mi = b1 * a.m[gi][j] + (1.f - b1) * g;
    const float vi = b2 * a.v[gi][j] + (1.f - b2) * g * g;
    a.m[gi][j] = mi;
    a.v[gi][j] = vi;
    a.p[gi][j] -= a.lr[gi] * (mi / bc1) / (sqrtf(vi / bc2) + eps);
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
  if (i < 7) {
    const float gi = g[i];
    const float mi = b1 * state[i] + (1.f - b1) * gi;
    const float vi = b2 * state[8 + i] + (1.f - b2) * gi * gi;
    state[i] = mi;
    state[8 + i] = vi;
    const float bc1 = 1.f - powf(b1, t), bc2 = 1.f - powf(b2, t);
    const float lr = i < 4 ? lr_q : lr_t;
    pose[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
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

unsigned grid_for(int64_t n, int64_t cap) {
  int64_t b = (n + 255) / 256;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

void launch_loss_l1(const float* C, const float* D, const float* Ct, const float* Dt, int64_t P, float wc, float wd,
                    float* loss, float* gC, float* gD, hipStream_t s) {
  launch_fill_f32(loss, 0.f, 1, s);
  if (P <= 0) return;
  // a few hundred workgroups: each ends with one atomic on the same address
  hipLaunchKernelGGL(k_loss_l1, dim3(grid_for(P, 512)), dim3(256), 0, s, C, D, Ct, Dt, P, wc / (3.f * (float)P),
                     wd / (float)P, loss, gC, gD);
}

int64_t track_temp_words() { return kSelWords; }

void launch_loss_track(const float* C, const float* D, const float* A, const float* Ct, const float* Dt, int64_t P,
                       float lambda_c, float inlier_mult, float* loss, float* gC, float* gD, float* median,
                       uint32_t* temp, hipStream_t s) {
  launch_fill_f32(loss, 0.f, 1, s);
  hipLaunchKernelGGL(k_select_init, dim3(1), dim3(256), 0, s, temp);
  const unsigned g = grid_for(P, 512);
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    hipLaunchKernelGGL(k_select_hist, dim3(g), dim3(256), 0, s, D, Dt, P, shift, temp);
    hipLaunchKernelGGL(k_select_pick, dim3(1), dim3(64), 0, s, temp, shift, pass == 0 ? 1 : 0);
  }
  hipLaunchKernelGGL(k_loss_track, dim3(grid_for(P, 512)), dim3(256), 0, s, C, D, A, Ct, Dt, P, lambda_c,
                     inlier_mult, (const uint32_t*)temp, loss, gC, gD, median);
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
  hipLaunchKernelGGL(k_adam_multi, dim3(grid_for(a.off[a.n], 4096)), dim3(256), 0, s, a, b1, b2, eps, bc1, bc2);
}
void launch_pose_const_velocity(const float* p0, const float* p1, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pose_const_velocity, dim3(1), dim3(64), 0, s, p0, p1, out);
}
void launch_pose_apply_twist(const float* pose, const float* xi, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pose_apply_twist, dim3(1), dim3(64), 0, s, pose, xi, out);
}
}  // namespace gsr
