// Projection of Gaussians (Eq. 1), EWA 2D covariance (Eq. 2), support box and
// tile rectangle; and the backward of that chain to the 3D parameters and the
// camera pose. One thread per Gaussian; memory bound (56 B in, 60 B out).
#include "gsr_internal.h"

namespace gsr {

namespace {

struct PoseF {
  float qh[4];
  float inv_norm;
  float R[9];
  float t[3];
  bool ok;
};

__device__ __forceinline__ PoseF load_pose(const float* __restrict__ p7) {
  PoseF P;
  const float w = p7[0], x = p7[1], y = p7[2], z = p7[3];
  const float n2 = w * w + x * x + y * y + z * z;
  P.ok = n2 > 0.f && isfinite(n2);
  const float inv = P.ok ? 1.f / sqrtf(n2) : 0.f;
  P.inv_norm = inv;
  P.qh[0] = w * inv;
  P.qh[1] = x * inv;
  P.qh[2] = y * inv;
  P.qh[3] = z * inv;
  quat_rot(P.qh[0], P.qh[1], P.qh[2], P.qh[3], P.R);
  P.t[0] = p7[4];
  P.t[1] = p7[5];
  P.t[2] = p7[6];
  return P;
}

// Everything about one Gaussian that both passes recompute.
struct Geo {
  float qh[4], inv_qn;
  float R[9];
  float s[3];
  float Sig[6];   // Sigma (xx, xy, xz, yy, yz, zz)
  float x[3];     // camera-space mean
  float Sc[6];    // Sigma_c = R_p Sigma R_p^T (xx, xy, xz, yy, yz, zz)
  float J00, J02, J11, J12;
  bool clx, cly;
  float Xc, Yc;
  float Sxx, Sxy, Syy;  // Sigma' with low-pass
  float det;
  float u, v;
};

// Returns false if the Gaussian is culled before the support box.
__device__ __forceinline__ bool project_geo(const Raster& Rr, const PoseF& P, const float* __restrict__ means,
                                            const float* __restrict__ scales, const float* __restrict__ quats,
                                            int64_t k, Geo& g) {
  if (!P.ok) return false;
  const float4 q = reinterpret_cast<const float4*>(quats)[k];
  const float n2 = q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w;
  if (!(n2 > 0.f) || !isfinite(n2)) return false;
  g.inv_qn = 1.f / sqrtf(n2);
  g.qh[0] = q.x * g.inv_qn;
  g.qh[1] = q.y * g.inv_qn;
  g.qh[2] = q.z * g.inv_qn;
  g.qh[3] = q.w * g.inv_qn;
  quat_rot(g.qh[0], g.qh[1], g.qh[2], g.qh[3], g.R);
  g.s[0] = scales[3 * k + 0];
  g.s[1] = scales[3 * k + 1];
  g.s[2] = scales[3 * k + 2];
  // M = R diag(s); Sigma = M M^T
  float M[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[3 * i + j] = g.R[3 * i + j] * g.s[j];
  g.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  g.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  g.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  g.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  g.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  g.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
  const float mx = means[3 * k + 0], my = means[3 * k + 1], mz = means[3 * k + 2];
#pragma unroll
  for (int i = 0; i < 3; ++i) g.x[i] = P.R[3 * i] * mx + P.R[3 * i + 1] * my + P.R[3 * i + 2] * mz + P.t[i];
  if (!isfinite(g.x[0]) || !isfinite(g.x[1]) || !isfinite(g.x[2])) return false;
  const float z = g.x[2];
  if (!(z > Rr.near_z)) return false;
  const float iz = 1.f / z;
  g.u = Rr.fx * g.x[0] * iz + Rr.cx;
  g.v = Rr.fy * g.x[1] * iz + Rr.cy;
  const float X = g.x[0] * iz, Y = g.x[1] * iz;
  g.clx = (X < -Rr.limx) || (X > Rr.limx);
  g.cly = (Y < -Rr.limy) || (Y > Rr.limy);
  g.Xc = fminf(Rr.limx, fmaxf(-Rr.limx, X));
  g.Yc = fminf(Rr.limy, fmaxf(-Rr.limy, Y));
  g.J00 = Rr.fx * iz;
  g.J02 = -Rr.fx * g.Xc * iz;
  g.J11 = Rr.fy * iz;
  g.J12 = -Rr.fy * g.Yc * iz;
  // Sigma_c = R_p Sigma R_p^T
  const float S[9] = {g.Sig[0], g.Sig[1], g.Sig[2], g.Sig[1], g.Sig[3], g.Sig[4], g.Sig[2], g.Sig[4], g.Sig[5]};
  float T[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      T[3 * i + j] = P.R[3 * i] * S[j] + P.R[3 * i + 1] * S[3 + j] + P.R[3 * i + 2] * S[6 + j];
  float Sc[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Sc[3 * i + j] = T[3 * i] * P.R[3 * j] + T[3 * i + 1] * P.R[3 * j + 1] + T[3 * i + 2] * P.R[3 * j + 2];
  g.Sc[0] = Sc[0];
  g.Sc[1] = 0.5f * (Sc[1] + Sc[3]);
  g.Sc[2] = 0.5f * (Sc[2] + Sc[6]);
  g.Sc[3] = Sc[4];
  g.Sc[4] = 0.5f * (Sc[5] + Sc[7]);
  g.Sc[5] = Sc[8];
  // Sigma' = J Sigma_c J^T + h I with J = [[J00, 0, J02], [0, J11, J12]]
  const float a0 = g.J00 * g.Sc[0] + g.J02 * g.Sc[2];  // row 0 of J Sigma_c: (a0, a1, a2)
  const float a1 = g.J00 * g.Sc[1] + g.J02 * g.Sc[4];
  const float a2 = g.J00 * g.Sc[2] + g.J02 * g.Sc[5];
  const float b1 = g.J11 * g.Sc[3] + g.J12 * g.Sc[4];  // row 1: (b0, b1, b2)
  const float b2 = g.J11 * g.Sc[4] + g.J12 * g.Sc[5];
  g.Sxx = a0 * g.J00 + a2 * g.J02 + Rr.lowpass;
  g.Sxy = a1 * g.J11 + a2 * g.J12;
  g.Syy = b1 * g.J11 + b2 * g.J12 + Rr.lowpass;
  g.det = g.Sxx * g.Syy - g.Sxy * g.Sxy;
  if (!(g.det > 0.f) || !isfinite(g.det)) return false;
  return true;
}

// grid.y = view: view v reads pose7 + 7 v and writes entries v * n + k.
__global__ __launch_bounds__(256) void k_project(Raster Rr, ProjectArgs a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n) return;
  const int64_t o = (int64_t)blockIdx.y * a.n + k;
  const PoseF P = load_pose(a.pose7 + 7 * blockIdx.y);
  Geo g;
  uint32_t count = 0;
  int4 rect = make_int4(0, 0, 0, 0);  // packed tile rectangle, depth bits, tile count (0: not binned)
  if (project_geo(Rr, P, a.means, a.scales, a.quats, k, g)) {
    const float op = a.opacities[k];
    if (op >= Rr.amin && isfinite(op)) {
      const float idet = 1.f / g.det;
      const float ca = g.Syy * idet, cb = -g.Sxy * idet, cc = g.Sxx * idet;
      // support: o exp(-sigma) >= alpha_min needs sigma <= ln(o / alpha_min);
      // the box is taken for a slightly larger level, so outside it alpha stays
      // below alpha_min by a factor e^-0.001 and no FP32 rounding of alpha can
      // reach alpha_min there: skipping by box (tiles, blocks, quadrants)
      // never changes a result
      const float smax = logf(op / Rr.amin) * (1.f + kBoxSlack) + kBoxSlack;
      const float rx = sqrtf(2.f * smax * g.Sxx), ry = sqrtf(2.f * smax * g.Syy);
      const float ex0 = g.u - rx, ex1 = g.u + rx, ey0 = g.v - ry, ey1 = g.v + ry;
      if (isfinite(ex0) && isfinite(ex1) && isfinite(ey0) && isfinite(ey1)) {
        const float fx0 = fmaxf(0.f, ceilf(ex0)), fx1 = fminf((float)(Rr.W - 1), floorf(ex1));
        const float fy0 = fmaxf(0.f, ceilf(ey0)), fy1 = fminf((float)(Rr.H - 1), floorf(ey1));
        if (fx0 <= fx1 && fy0 <= fy1) {
          const int px0 = (int)fx0, px1 = (int)fx1, py0 = (int)fy0, py1 = (int)fy1;
          const int tx0 = px0 >> Rr.tw_log2, ty0 = py0 / Rr.th, tx1 = px1 >> Rr.tw_log2, ty1 = py1 / Rr.th;
          count = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
          rect = make_int4((int)((uint32_t)tx0 | ((uint32_t)tx1 << 16)), (int)((uint32_t)ty0 | ((uint32_t)ty1 << 16)),
                           (int)__float_as_uint(g.x[2]), (int)count);
          const float s = -0.5f * kLog2e;
          a.rec_uvab[kRec * o] = make_float4(g.u, g.v, s * ca, -kLog2e * cb);
          a.rec_cob[kRec * o] = make_float4(s * cc, op, __uint_as_float((uint32_t)px0 | ((uint32_t)px1 << 16)),
                                     __uint_as_float((uint32_t)py0 | ((uint32_t)py1 << 16)));
          a.rec_rgbz[kRec * o] = make_float4(a.colors[3 * k], a.colors[3 * k + 1], a.colors[3 * k + 2], g.x[2]);
          // the slot's unused fourth float4 is written too: whole 64-byte lines
          // make the compositing kernels' later gathers of the records faster
          a.rec_rgbz[kRec * o + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
    }
  }
  a.rect[o] = rect;
  a.counts[o] = count;
}

// Backward of the projection for one (Gaussian, view). g2d holds the ten
// per-Gaussian sums of the compositing backward (see below for the first five;
// then dL/d(o, r, g, b) and the direct dL/dz). Adds to
// the parameter gradients and returns the pose partials (dL/dR_p, dL/dt).
__device__ __forceinline__ void chain_one(const Raster& Rr, const PoseF& P, const ProjectBwdArgs& a, int64_t k,
                                          const float* __restrict__ G2, float gm[3], float gs[3], float gq[4],
                                          float& go, float gc[3], float pacc[12]) {
  Geo g;
  if (!project_geo(Rr, P, a.means, a.scales, a.quats, k, g)) return;
  const float idet = 1.f / g.det;
  const float A00 = g.Syy * idet, A01 = -g.Sxy * idet, A11 = g.Sxx * idet;
  // The compositing backward accumulates q = (dL/dalpha) alpha = (dL/dp) / ln 2
  // per pair, with alpha = o 2^p, p = pa dx^2 + pb dx dy + pc dy^2, dx = px - u
  // and the stored (pa, pb, pc) = -log2(e) (a/2, b, c/2) of the conic (a, b, c):
  // G2[0..4] = sum q (dx, dy, dx^2, dx dy, dy^2). As pa, pb, pc are constant per
  // Gaussian, dL/du = -ln2 (2 pa G2[0] + pb G2[1]) = a G2[0] + b G2[1] (likewise
  // for v) and dL/da = -ln2 log2(e) G2[2] / 2 = -G2[2] / 2, dL/db = -G2[3].
  const float g_u = A00 * G2[0] + A01 * G2[1];
  const float g_v = A01 * G2[0] + A11 * G2[1];
  const float g_a = -0.5f * G2[2];
  const float g_b = -G2[3];
  const float g_c = -0.5f * G2[4];
  go += G2[5];
  gc[0] += G2[6];
  gc[1] += G2[7];
  gc[2] += G2[8];
  const float g_zd = G2[9];
  // dL/dSigma' = -A Mg A with Mg = [[g_a, g_b/2], [g_b/2, g_c]]
  const float m01 = 0.5f * g_b;
  const float t00 = A00 * g_a + A01 * m01, t01 = A00 * m01 + A01 * g_c;
  const float t10 = A01 * g_a + A11 * m01, t11 = A01 * m01 + A11 * g_c;
  const float G00 = -(t00 * A00 + t01 * A01);
  const float G01 = -(t00 * A01 + t01 * A11);
  const float G11 = -(t10 * A01 + t11 * A11);
  // Sigma' = J Sc J^T:  dL/dSc = J^T G J,  dL/dJ = 2 G J Sc
  const float J00 = g.J00, J02 = g.J02, J11 = g.J11, J12 = g.J12;
  const float r0[3] = {J00 * g.Sc[0] + J02 * g.Sc[2], J00 * g.Sc[1] + J02 * g.Sc[4], J00 * g.Sc[2] + J02 * g.Sc[5]};
  const float r1[3] = {J11 * g.Sc[1] + J12 * g.Sc[2], J11 * g.Sc[3] + J12 * g.Sc[4], J11 * g.Sc[4] + J12 * g.Sc[5]};
  const float dJ00 = 2.f * (G00 * r0[0] + G01 * r1[0]);
  const float dJ02 = 2.f * (G00 * r0[2] + G01 * r1[2]);
  const float dJ11 = 2.f * (G01 * r0[1] + G11 * r1[1]);
  const float dJ12 = 2.f * (G01 * r0[2] + G11 * r1[2]);
  // J^T G J for J columns c0 = (J00, 0), c1 = (0, J11), c2 = (J02, J12)
  float GSc[9];
  {
    const float c[3][2] = {{J00, 0.f}, {0.f, J11}, {J02, J12}};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        GSc[3 * i + j] = c[i][0] * (G00 * c[j][0] + G01 * c[j][1]) + c[i][1] * (G01 * c[j][0] + G11 * c[j][1]);
  }
  const float z = g.x[2], iz = 1.f / z, iz2 = iz * iz;
  float gx = 0.f, gy = 0.f, gz = 0.f;
  gz += dJ00 * (-Rr.fx * iz2) + dJ11 * (-Rr.fy * iz2);
  if (!g.clx) {
    gx += dJ02 * (-Rr.fx * iz2);
    gz += dJ02 * (2.f * Rr.fx * g.x[0] * iz2 * iz);
  } else {
    gz += dJ02 * (Rr.fx * g.Xc * iz2);
  }
  if (!g.cly) {
    gy += dJ12 * (-Rr.fy * iz2);
    gz += dJ12 * (2.f * Rr.fy * g.x[1] * iz2 * iz);
  } else {
    gz += dJ12 * (Rr.fy * g.Yc * iz2);
  }
  gx += g_u * Rr.fx * iz;
  gz += -g_u * Rr.fx * g.x[0] * iz2;
  gy += g_v * Rr.fy * iz;
  gz += -g_v * Rr.fy * g.x[1] * iz2;
  gz += g_zd;
  // mean: x = R_p mu + t
#pragma unroll
  for (int i = 0; i < 3; ++i) gm[i] += P.R[i] * gx + P.R[3 + i] * gy + P.R[6 + i] * gz;
  // dL/dSigma = R_p^T GSc R_p
  float U[9], GS[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) U[3 * i + j] = P.R[i] * GSc[j] + P.R[3 + i] * GSc[3 + j] + P.R[6 + i] * GSc[6 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) GS[3 * i + j] = U[3 * i] * P.R[j] + U[3 * i + 1] * P.R[3 + j] + U[3 * i + 2] * P.R[6 + j];
  // Sigma = M M^T, M = R diag(s): dL/dM = 2 GS M
  float M[9], GM[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[3 * i + j] = g.R[3 * i + j] * g.s[j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      GM[3 * i + j] = 2.f * (GS[3 * i] * M[j] + GS[3 * i + 1] * M[3 + j] + GS[3 * i + 2] * M[6 + j]);
  float GR[9];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    gs[j] += GM[j] * g.R[j] + GM[3 + j] * g.R[3 + j] + GM[6 + j] * g.R[6 + j];
#pragma unroll
    for (int i = 0; i < 3; ++i) GR[3 * i + j] = GM[3 * i + j] * g.s[j];
  }
  float dq[4];
  quat_rot_vjp(g.qh, g.inv_qn, GR, dq);
#pragma unroll
  for (int i = 0; i < 4; ++i) gq[i] += dq[i];
  if (a.pose_acc) {
    // dL/dR_p = gx mu^T + 2 GSc R_p Sigma ;  dL/dt = gx
    const float mu[3] = {a.means[3 * k], a.means[3 * k + 1], a.means[3 * k + 2]};
    const float S[9] = {g.Sig[0], g.Sig[1], g.Sig[2], g.Sig[1], g.Sig[3], g.Sig[4], g.Sig[2], g.Sig[4], g.Sig[5]};
    float RS[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) RS[3 * i + j] = P.R[3 * i] * S[j] + P.R[3 * i + 1] * S[3 + j] + P.R[3 * i + 2] * S[6 + j];
    const float gxv[3] = {gx, gy, gz};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        pacc[3 * i + j] = gxv[i] * mu[j] + 2.f * (GSc[3 * i] * RS[j] + GSc[3 * i + 1] * RS[3 + j] + GSc[3 * i + 2] * RS[6 + j]);
    pacc[9] = gx;
    pacc[10] = gy;
    pacc[11] = gz;
  }
}

// Adam, by the whole workgroup, on the cnt values of parameter group grp
// starting at base, with their gradients in LDS (g, 16-byte aligned): float4
// accesses when the group's arrays allow, then a scalar tail.
__device__ __forceinline__ void adam_range(const AdamFused& A, int grp, int64_t base, int cnt, const float* g) {
  float* __restrict__ P = A.p[grp] + base;
  float* __restrict__ M = A.m[grp] + base;
  float* __restrict__ V = A.v[grp] + base;
  const float lr = A.lr[grp];
  const bool vec = ((reinterpret_cast<uintptr_t>(P) | reinterpret_cast<uintptr_t>(M) | reinterpret_cast<uintptr_t>(V)) &
                    15u) == 0;
  const int n4 = vec ? cnt / 4 : 0;
  for (int i = threadIdx.x; i < n4; i += blockDim.x) {
    float4 p = reinterpret_cast<float4*>(P)[i], m = reinterpret_cast<float4*>(M)[i];
    float4 v = reinterpret_cast<float4*>(V)[i];
    const float4 gg = reinterpret_cast<const float4*>(g)[i];
    adam_one(p.x, m.x, v.x, gg.x, lr, A.b1, A.b2, A.eps, A.bc1, A.bc2);
    adam_one(p.y, m.y, v.y, gg.y, lr, A.b1, A.b2, A.eps, A.bc1, A.bc2);
    adam_one(p.z, m.z, v.z, gg.z, lr, A.b1, A.b2, A.eps, A.bc1, A.bc2);
    adam_one(p.w, m.w, v.w, gg.w, lr, A.b1, A.b2, A.eps, A.bc1, A.bc2);
    reinterpret_cast<float4*>(P)[i] = p;
    reinterpret_cast<float4*>(M)[i] = m;
    reinterpret_cast<float4*>(V)[i] = v;
  }
  for (int i = 4 * n4 + threadIdx.x; i < cnt; i += blockDim.x) {
    float p = P[i], m = M[i], v = V[i];
    adam_one(p, m, v, g[i], lr, A.b1, A.b2, A.eps, A.bc1, A.bc2);
    P[i] = p;
    M[i] = m;
    V[i] = v;
  }
}

// One thread per Gaussian, looping over the views: parameter gradients are the
// sum over views; pose partials are reduced per view (workgroup sum + one
// atomic per value).
// At most 128 VGPRs (four waves per SIMD; one register spills): the kernel is
// bound by memory latency, so resident waves matter more than the spill.
__global__ __launch_bounds__(256, 4) void k_project_bwd(Raster Rr, ProjectBwdArgs a) {
  __shared__ float red[4][12];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  float gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0.f, gc[3] = {0, 0, 0};
  for (int v = 0; v < a.n_views; ++v) {
    const PoseF P = load_pose(a.pose7 + 7 * v);
    float pacc[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) pacc[i] = 0.f;
    const int64_t o = (int64_t)v * a.n + k;
    if (k < a.n && a.counts[o] > 0) {
      float* g2 = a.g2d + 10 * o;
      chain_one(Rr, P, a, k, g2, gm, gs, gq, go, gc, pacc);
      // leave the sums at zero for the next backward (the compositing backward
      // only adds to Gaussians with tiles, i.e. the ones cleared here)
#pragma unroll
      for (int i = 0; i < 10; ++i) g2[i] = 0.f;
    }
    if (a.pose_acc) {
#pragma unroll
      for (int i = 0; i < 12; ++i) {
        const float s = wave_sum_all(pacc[i]);
        if (lane == 0) red[w][i] = s;
      }
      __syncthreads();
      if (threadIdx.x < 12) {
        const int nw = (blockDim.x + 63) >> 6;
        float s = 0.f;
        for (int i = 0; i < nw; ++i) s += red[i][threadIdx.x];
        a.pose_acc[((int64_t)v * gridDim.x + blockIdx.x) * 12 + threadIdx.x] = s;
      }
      __syncthreads();
    }
  }
  if (a.adam.on && a.adam.reg_w != 0.f && k < a.n) {
    float d[3];
    (void)reg_term(a.scales[3 * k], a.scales[3 * k + 1], a.scales[3 * k + 2], a.adam.reg_w, d);
    gs[0] += d[0];
    gs[1] += d[1];
    gs[2] += d[2];
  }
  if (a.adam.on) {
    // Stage the workgroup's gradients in LDS in parameter order, then run Adam
    // over each group's contiguous range with 16-byte accesses.
    __shared__ __align__(16) float sg[14 * 256];
    const int t = threadIdx.x;
    sg[3 * t] = gm[0];
    sg[3 * t + 1] = gm[1];
    sg[3 * t + 2] = gm[2];
    sg[768 + 3 * t] = gs[0];
    sg[768 + 3 * t + 1] = gs[1];
    sg[768 + 3 * t + 2] = gs[2];
    sg[1536 + 4 * t] = gq[0];
    sg[1536 + 4 * t + 1] = gq[1];
    sg[1536 + 4 * t + 2] = gq[2];
    sg[1536 + 4 * t + 3] = gq[3];
    sg[2560 + t] = go;
    sg[2816 + 3 * t] = gc[0];
    sg[2816 + 3 * t + 1] = gc[1];
    sg[2816 + 3 * t + 2] = gc[2];
    __syncthreads();
    const int64_t k0 = (int64_t)blockIdx.x * blockDim.x;
    const int nk = (int)min((int64_t)blockDim.x, a.n - k0);
    const int width[5] = {3, 3, 4, 1, 3}, soff[5] = {0, 768, 1536, 2560, 2816};
#pragma unroll
    for (int grp = 0; grp < 5; ++grp) adam_range(a.adam, grp, k0 * width[grp], nk * width[grp], sg + soff[grp]);
  }
  if (k < a.n) {
    if (a.g_means) {
      a.g_means[3 * k] = gm[0];
      a.g_means[3 * k + 1] = gm[1];
      a.g_means[3 * k + 2] = gm[2];
    }
    if (a.g_scales) {
      a.g_scales[3 * k] = gs[0];
      a.g_scales[3 * k + 1] = gs[1];
      a.g_scales[3 * k + 2] = gs[2];
    }
    if (a.g_quats) reinterpret_cast<float4*>(a.g_quats)[k] = make_float4(gq[0], gq[1], gq[2], gq[3]);
    if (a.g_opacities) a.g_opacities[k] = go;
    if (a.g_colors) {
      a.g_colors[3 * k] = gc[0];
      a.g_colors[3 * k + 1] = gc[1];
      a.g_colors[3 * k + 2] = gc[2];
    }
  }
}

// From dL/dR_p and dL/dt to the quaternion/translation gradient and the twist
// of the left perturbation (R <- Exp(phi) R, t <- Exp(phi) t + rho):
//   dL/drho = dL/dt,   dL/dphi = sum_j R[:, j] x G[:, j] + t x dL/dt.
// One workgroup per view: the 12 pose partials summed over the projection
// backward's workgroups (fixed order), then dL/d(q, t) and the twist.
__global__ __launch_bounds__(256) void k_pose_finalize(const float* __restrict__ poses7,
                                                      const float* __restrict__ parts, int64_t blocks,
                                                      float* __restrict__ dposes7, float* __restrict__ dtwists6,
                                                      PoseAdam adam) {
  const int v = blockIdx.x;
  __shared__ float red[4][12];
  __shared__ float acc[12];
  __shared__ float g7s[7];
  float s[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) s[i] = 0.f;
  const float* part = parts + (int64_t)v * blocks * 12;
  for (int64_t b = threadIdx.x; b < blocks; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < 12; ++i) s[i] += part[b * 12 + i];
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const float t = wave_sum_all(s[i]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][i] = t;
  }
  __syncthreads();
  if (threadIdx.x < 12) acc[threadIdx.x] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                                           red[3][threadIdx.x];
  __syncthreads();
  const float* pose7 = poses7 + 7 * v;
  if (threadIdx.x == 0) {
    float* dpose7 = dposes7 ? dposes7 + 7 * v : nullptr;
    float* dtwist6 = dtwists6 ? dtwists6 + 6 * v : nullptr;
    const PoseF P = load_pose(pose7);
    float G[9];
    for (int i = 0; i < 9; ++i) G[i] = acc[i];
    const float gt[3] = {acc[9], acc[10], acc[11]};
    if (dpose7 || adam.state) {
      float gq[4] = {0, 0, 0, 0};
      if (P.ok) quat_rot_vjp(P.qh, P.inv_norm, G, gq);
      const float g7[7] = {gq[0], gq[1], gq[2], gq[3], gt[0], gt[1], gt[2]};
      for (int i = 0; i < 7; ++i) {
        g7s[i] = g7[i];
        if (dpose7) dpose7[i] = g7[i];
      }
    }
    if (dtwist6) {
      float phi[3] = {P.t[1] * gt[2] - P.t[2] * gt[1], P.t[2] * gt[0] - P.t[0] * gt[2], P.t[0] * gt[1] - P.t[1] * gt[0]};
      for (int j = 0; j < 3; ++j) {
        const float r0 = P.R[j], r1 = P.R[3 + j], r2 = P.R[6 + j];
        const float g0 = G[j], g1 = G[3 + j], g2 = G[6 + j];
        phi[0] += r1 * g2 - r2 * g1;
        phi[1] += r2 * g0 - r0 * g2;
        phi[2] += r0 * g1 - r1 * g0;
      }
      for (int i = 0; i < 3; ++i) {
        dtwist6[i] = gt[i];
        dtwist6[3 + i] = phi[i];
      }
    }
  }
  if (!adam.state) return;  // uniform: a kernel argument
  // the pose Adam step on the gradient just formed (the pose was read above)
  __syncthreads();
  const float t = adam.state[16] + 1.f;
  __syncthreads();
  if (threadIdx.x < 7)
    pose_adam_elem(const_cast<float*>(pose7), adam.state, threadIdx.x, g7s[threadIdx.x], t, adam.lr_q, adam.lr_t,
                   adam.b1, adam.b2, adam.eps);
  if (threadIdx.x == 0) adam.state[16] = t;
}

}  // namespace

void launch_project(const Raster& R, const ProjectArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  const int64_t blocks = (a.n + 255) / 256;
  hipLaunchKernelGGL(k_project, dim3((unsigned)blocks, (unsigned)a.n_views), dim3(256), 0, s, R, a);
}

int64_t project_bwd_blocks(int64_t n) { return (n + 255) / 256; }

void launch_project_bwd(const Raster& R, const ProjectBwdArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  hipLaunchKernelGGL(k_project_bwd, dim3((unsigned)project_bwd_blocks(a.n)), dim3(256), 0, s, R, a);
}

void launch_pose_finalize(const float* pose7, const float* parts, int64_t blocks, float* dpose7, float* dtwist6,
                          int n_views, hipStream_t s, const PoseAdam* adam) {
  if (n_views <= 0) return;
  PoseAdam pa{};
  if (adam && n_views == 1) pa = *adam;
  hipLaunchKernelGGL(k_pose_finalize, dim3((unsigned)n_views), dim3(256), 0, s, pose7, parts, blocks, dpose7,
                     dtwist6, pa);
}

}  // namespace gsr
