// Tracking-initialisation network: a small CNN that proposes a pose
// correction from the render at the current pose and the observed RGB-D
// frame (both downsampled to 160 x 120, 8 channels: the render and the
// observed-minus-rendered residual). Four 3x3 stride-2 convolutions (64
// channels, ReLU), moment pooling (mean and first spatial moments) and a
// linear head to a 6-vector twist. Convolutions are implicit GEMMs on the gfx950 matrix
// cores (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 accumulation);
// activations and weights are BF16, master weights and the head FP32.
//
// Layouts: activations NHWC BF16 [B, H, W, C]; packed weights [64][KP] with
// K ordered (tap = 3 ky + kx, channel) and zero-padded to KP = 32 ceil(9 C / 32);
// transposed weights [C][9][64] for the data gradient.
//
// MFMA 16x16x32 operand layout (64 lanes): A[i][k] in lane i + 16 (k / 8),
// element k % 8; B[k][j] in lane j + 16 (k / 8), element k % 8; D[i][j] in
// lane j + 16 (i / 4), element i % 4.
#include <hip/hip_bf16.h>

#include "gsr_internal.h"

namespace gsr {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kHeadIn = 3 * 64;     // pooled features: three moments of 64 channels
constexpr float kDiffGain = 4.f;    // scale of the observed-minus-rendered channels

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// float -> bf16 with round-to-nearest-even
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  const u16x8 v = *reinterpret_cast<const u16x8*>(p);
  return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x8 zero8() {
  const u16x8 z = {0, 0, 0, 0, 0, 0, 0, 0};
  return __builtin_bit_cast(bf16x8, z);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

struct ConvShape {
  int B, H, W, C;   // input
  int OH, OW;       // output (stride 2, pad 1, 3x3)
  int KP;           // padded 9 * C
};

// ---- forward: out = relu(conv(in) + bias), 64 output pixels x 64 channels per workgroup
__global__ __launch_bounds__(256) void k_conv_fwd(ConvShape s, const uint16_t* __restrict__ in,
                                                 const uint16_t* __restrict__ wk, const float* __restrict__ bias,
                                                 uint16_t* __restrict__ out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t M = (int64_t)s.B * s.OH * s.OW;
  const int64_t m = (int64_t)blockIdx.x * 64 + wv * 16 + (lane & 15);
  int b = 0, oy = 0, ox = 0;
  if (m < M) {
    b = (int)(m / ((int64_t)s.OH * s.OW));
    const int r = (int)(m - (int64_t)b * s.OH * s.OW);
    oy = r / s.OW;
    ox = r - oy * s.OW;
  }
  f32x4 acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < s.KP; k0 += 32) {
    const int kk = k0 + (lane >> 4) * 8;
    const int tap = kk / s.C, ci = kk - tap * s.C;
    bf16x8 a = zero8();
    if (m < M && tap < 9) {
      const int iy = 2 * oy + tap / 3 - 1, ix = 2 * ox + tap % 3 - 1;
      if (iy >= 0 && iy < s.H && ix >= 0 && ix < s.W)
        a = load8(in + (((int64_t)b * s.H + iy) * s.W + ix) * s.C + ci);
    }
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const bf16x8 bw = load8(wk + (int64_t)(nb * 16 + (lane & 15)) * s.KP + kk);
      acc[nb] = mfma(a, bw, acc[nb]);
    }
  }
  // D[i][j]: pixel row i = 4 (lane / 16) + e of this wave's 16, channel j = lane % 16 (+16 nb)
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int co = nb * 16 + (lane & 15);
    const float bs = bias[co];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t mo = (int64_t)blockIdx.x * 64 + wv * 16 + 4 * (lane >> 4) + e;
      if (mo < M) out[mo * 64 + co] = f2bf(fmaxf(acc[nb][e] + bs, 0.f));
    }
  }
}

// ---- data gradient: din = (conv^T dout) * [in > 0] (the ReLU mask of the
// previous layer, whose output is this layer's input). GEMM over K = 9 x 64.
__global__ __launch_bounds__(256) void k_conv_bwd_data(ConvShape s, const uint16_t* __restrict__ dout,
                                                      const uint16_t* __restrict__ wt, const uint16_t* __restrict__ in,
                                                      uint16_t* __restrict__ din) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t M = (int64_t)s.B * s.H * s.W;  // input pixels
  const int64_t m = (int64_t)blockIdx.x * 64 + wv * 16 + (lane & 15);
  int b = 0, iy = 0, ix = 0;
  if (m < M) {
    b = (int)(m / ((int64_t)s.H * s.W));
    const int r = (int)(m - (int64_t)b * s.H * s.W);
    iy = r / s.W;
    ix = r - iy * s.W;
  }
  f32x4 acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < 9 * 64; k0 += 32) {
    const int kk = k0 + (lane >> 4) * 8;
    const int tap = kk >> 6, co = kk & 63;
    const int ty = iy + 1 - tap / 3, tx = ix + 1 - tap % 3;  // = 2 oy, 2 ox
    bf16x8 a = zero8();
    if (m < M && ty >= 0 && tx >= 0 && !(ty & 1) && !(tx & 1) && (ty >> 1) < s.OH && (tx >> 1) < s.OW)
      a = load8(dout + (((int64_t)b * s.OH + (ty >> 1)) * s.OW + (tx >> 1)) * 64 + co);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int c = nb * 16 + (lane & 15);
      const bf16x8 bw = c < s.C ? load8(wt + ((int64_t)c * 9 + tap) * 64 + co) : zero8();
      acc[nb] = mfma(a, bw, acc[nb]);
    }
  }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int c = nb * 16 + (lane & 15);
    if (c >= s.C) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t mo = (int64_t)blockIdx.x * 64 + wv * 16 + 4 * (lane >> 4) + e;
      if (mo < M) {
        const int64_t o = mo * s.C + c;
        din[o] = bf2f(in[o]) > 0.f ? f2bf(acc[nb][e]) : (uint16_t)0;
      }
    }
  }
}

// ---- weight gradient: dW[co][kk] += sum_m dy[m][co] im2col(in)[m][kk]. A
// workgroup owns 64 columns kk and walks pixel chunks of 64 (grid-stride over
// grid.y); chunks are staged transposed in LDS so both MFMA operands are
// contiguous 8-element runs; one atomic add per output element at the end.
constexpr int kWPix = 64;
__global__ __launch_bounds__(256) void k_conv_bwd_weight(ConvShape s, const uint16_t* __restrict__ dy,
                                                        const uint16_t* __restrict__ in, float* __restrict__ dw) {
  __shared__ uint16_t sd[64][kWPix + 8];  // [co][pixel]
  __shared__ uint16_t sa[64][kWPix + 8];  // [kk - kk0][pixel]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, tid = threadIdx.x;
  const int kk0 = blockIdx.x * 64;
  const int64_t M = (int64_t)s.B * s.OH * s.OW;
  f32x4 acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t p0 = (int64_t)blockIdx.y * kWPix; p0 < M; p0 += (int64_t)gridDim.y * kWPix) {
    __syncthreads();
    // stage: 64 pixels x 64 values each, 16 per thread
    for (int t = tid; t < kWPix * 64; t += 256) {
      const int px = t >> 6, col = t & 63;
      const int64_t m = p0 + px;
      uint16_t dv = 0, av = 0;
      if (m < M) {
        dv = dy[m * 64 + col];
        const int kk = kk0 + col;
        const int tap = kk / s.C, ci = kk - tap * s.C;
        if (tap < 9) {
          const int b = (int)(m / ((int64_t)s.OH * s.OW));
          const int r = (int)(m - (int64_t)b * s.OH * s.OW);
          const int oy = r / s.OW, ox = r - oy * s.OW;
          const int iy = 2 * oy + tap / 3 - 1, ix = 2 * ox + tap % 3 - 1;
          if (iy >= 0 && iy < s.H && ix >= 0 && ix < s.W) av = in[(((int64_t)b * s.H + iy) * s.W + ix) * s.C + ci];
        }
      }
      sd[col][px] = dv;
      sa[col][px] = av;
    }
    __syncthreads();
    // wave wv: output rows co = 16 wv + i, columns kk = kk0 + 16 nb + j; K = 64 pixels
#pragma unroll
    for (int k0 = 0; k0 < kWPix; k0 += 32) {
      const int pk = k0 + (lane >> 4) * 8;
      u16x8 av8, bv8;
#pragma unroll
      for (int e = 0; e < 8; ++e) av8[e] = sd[wv * 16 + (lane & 15)][pk + e];
      const bf16x8 a = __builtin_bit_cast(bf16x8, av8);
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
#pragma unroll
        for (int e = 0; e < 8; ++e) bv8[e] = sa[nb * 16 + (lane & 15)][pk + e];
        acc[nb] = mfma(a, __builtin_bit_cast(bf16x8, bv8), acc[nb]);
      }
    }
  }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int kk = kk0 + nb * 16 + (lane & 15);
    if (kk >= s.KP) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int co = wv * 16 + 4 * (lane >> 4) + e;
      atomicAdd(&dw[(int64_t)co * s.KP + kk], acc[nb][e]);
    }
  }
}

// Bias gradient: sum over pixels of dy[m][co] (one workgroup per 64 channels x pixel stripe).
__global__ __launch_bounds__(256) void k_bias_grad(const uint16_t* __restrict__ dy, int64_t M, float* __restrict__ db) {
  const int co = threadIdx.x & 63, r = threadIdx.x >> 6;
  float s = 0.f;
  for (int64_t m = (int64_t)blockIdx.x * 4 + r; m < M; m += (int64_t)gridDim.x * 4) s += bf2f(dy[m * 64 + co]);
  atomicAdd(&db[co], s);
}

// Head. Moment pooling over the last feature map (OH x OW pixels): for each
// channel c, pool[b][k][c] = (1/npix) sum_p m_k(p) act[b][p][c] with m_0 = 1,
// m_1 = x^(p), m_2 = y^(p), x^ = (2 x + 1) / OW - 1 and y^ = (2 y + 1) / OH - 1
// (pixel centres mapped to (-1, 1)); out[b] = Wfc pool[b] + bfc over the 192
// pooled values (k major). The first moments keep where features sit, which a
// plain average cancels (a forward motion or a roll moves image content
// radially or around the centre, with zero mean displacement).
// One workgroup per sample, one lane per channel.
__device__ __forceinline__ float moment_x(int p, int OW) { return (2.f * (float)(p % OW) + 1.f) / (float)OW - 1.f; }
__device__ __forceinline__ float moment_y(int p, int OW, int OH) {
  return (2.f * (float)(p / OW) + 1.f) / (float)OH - 1.f;
}

__global__ __launch_bounds__(64) void k_head_fwd(const uint16_t* __restrict__ act, int OH, int OW,
                                                const float* __restrict__ wfc, const float* __restrict__ bfc,
                                                float* __restrict__ pool, float* __restrict__ out) {
  const int b = blockIdx.x, c = threadIdx.x;
  const int npix = OH * OW;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f;
  for (int p = 0; p < npix; ++p) {
    const float v = bf2f(act[((int64_t)b * npix + p) * 64 + c]);
    s0 += v;
    s1 += v * moment_x(p, OW);
    s2 += v * moment_y(p, OW, OH);
  }
  const float inv = 1.f / (float)npix;
  __shared__ float sp[kHeadIn];
  sp[c] = s0 * inv;
  sp[64 + c] = s1 * inv;
  sp[128 + c] = s2 * inv;
  for (int k = 0; k < 3; ++k) pool[b * kHeadIn + 64 * k + c] = sp[64 * k + c];
  __syncthreads();
  if (c < 6) {
    float o = bfc[c];
    for (int i = 0; i < kHeadIn; ++i) o += wfc[c * kHeadIn + i] * sp[i];
    out[b * 6 + c] = o;
  }
}

// Loss L = 1/(2B) sum ((out - label) / scale)^2, its gradient, the head's
// gradients (atomic over samples), and dL/dact4[p][c] = (1/npix)
// sum_k m_k(p) dpool[k][c] * [act > 0] with dpool = Wfc^T dout.
__global__ __launch_bounds__(64) void k_head_bwd(const float* __restrict__ out, const float* __restrict__ label,
                                                const float* __restrict__ scale, int B, const float* __restrict__ pool,
                                                const float* __restrict__ wfc, const uint16_t* __restrict__ act,
                                                int OH, int OW, const float* __restrict__ dout_in,
                                                float* __restrict__ dwfc, float* __restrict__ dbfc,
                                                uint16_t* __restrict__ dact, float* __restrict__ loss) {
  const int b = blockIdx.x, c = threadIdx.x;
  const int npix = OH * OW;
  __shared__ float g[6];
  if (c < 6) {
    float d;
    if (dout_in) {
      d = dout_in[b * 6 + c];
    } else {
      const float r = (out[b * 6 + c] - label[b * 6 + c]) / scale[c];
      d = r / scale[c] / (float)B;
      atomicAdd(loss, 0.5f * r * r / (float)B);
    }
    g[c] = d;
    atomicAdd(&dbfc[c], d);
  }
  __syncthreads();
  float dp[3] = {0.f, 0.f, 0.f};
  for (int k = 0; k < 3; ++k) {
    const int i = 64 * k + c;
    for (int j = 0; j < 6; ++j) {
      dp[k] += wfc[j * kHeadIn + i] * g[j];
      atomicAdd(&dwfc[j * kHeadIn + i], g[j] * pool[b * kHeadIn + i]);
    }
  }
  const float inv = 1.f / (float)npix;
  for (int p = 0; p < npix; ++p) {
    const int64_t o = ((int64_t)b * npix + p) * 64 + c;
    const float d = (dp[0] + moment_x(p, OW) * dp[1] + moment_y(p, OW, OH) * dp[2]) * inv;
    dact[o] = bf2f(act[o]) > 0.f ? f2bf(d) : (uint16_t)0;
  }
}

// Master FP32 packed weights [64][KP] -> BF16 packed copy and BF16 transposed
// copy [C][9][64] for the data gradient.
__global__ void k_cast_weights(const float* __restrict__ w, int C, int KP, uint16_t* __restrict__ wk,
                               uint16_t* __restrict__ wt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 64 * KP) return;
  const int co = i / KP, kk = i - co * KP;
  const uint16_t v = f2bf(w[i]);
  wk[i] = v;
  if (kk < 9 * C && wt) {
    const int tap = kk / C, ci = kk - tap * C;
    wt[((int64_t)ci * 9 + tap) * 64 + co] = v;
  }
}

// Input packing: f x f average pooling of the rendered and observed RGB-D
// frames into 8 BF16 channels: the render (r, g, b, depth * depth_scale) and
// the observation minus the render, times kDiffGain (the residual, formed in
// FP32 before rounding to BF16, where a few-millimetre depth residual would
// otherwise fall below the precision of depths of metres).
__global__ void k_pack_input(const float* __restrict__ rc, const float* __restrict__ rd, const float* __restrict__ oc,
                             const float* __restrict__ od, int H, int W, int f, float depth_scale,
                             uint16_t* __restrict__ out) {
  const int OW = W / f, OH = H / f;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= OW * OH) return;
  const int y = i / OW, x = i - y * OW;
  float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t P = (int64_t)H * W;
  for (int dy = 0; dy < f; ++dy)
    for (int dx = 0; dx < f; ++dx) {
      const int64_t p = (int64_t)(y * f + dy) * W + (x * f + dx);
      acc[0] += rc[p];
      acc[1] += rc[P + p];
      acc[2] += rc[2 * P + p];
      acc[3] += rd[p] * depth_scale;
      acc[4] += oc[p] - rc[p];
      acc[5] += oc[P + p] - rc[P + p];
      acc[6] += oc[2 * P + p] - rc[2 * P + p];
      acc[7] += (od[p] - rd[p]) * depth_scale;
    }
  const float inv = 1.f / (float)(f * f);
  for (int c = 0; c < 8; ++c) out[(int64_t)i * 8 + c] = f2bf(acc[c] * inv * (c < 4 ? 1.f : kDiffGain));
}

ConvShape shape_of(int B, int H, int W, int C) {
  ConvShape s;
  s.B = B;
  s.H = H;
  s.W = W;
  s.C = C;
  s.OH = (H + 1) / 2;
  s.OW = (W + 1) / 2;
  s.KP = ((9 * C + 31) / 32) * 32;
  return s;
}

}  // namespace

int conv_kp(int C) { return ((9 * C + 31) / 32) * 32; }

void launch_conv_fwd(int B, int H, int W, int C, const uint16_t* in, const uint16_t* wk, const float* bias,
                     uint16_t* out, hipStream_t st) {
  const ConvShape s = shape_of(B, H, W, C);
  const int64_t M = (int64_t)B * s.OH * s.OW;
  hipLaunchKernelGGL(k_conv_fwd, dim3((unsigned)((M + 63) / 64)), dim3(256), 0, st, s, in, wk, bias, out);
}

void launch_conv_bwd_data(int B, int H, int W, int C, const uint16_t* dout, const uint16_t* wt, const uint16_t* in,
                          uint16_t* din, hipStream_t st) {
  const ConvShape s = shape_of(B, H, W, C);
  const int64_t M = (int64_t)B * H * W;
  hipLaunchKernelGGL(k_conv_bwd_data, dim3((unsigned)((M + 63) / 64)), dim3(256), 0, st, s, dout, wt, in, din);
}

void launch_conv_bwd_weight(int B, int H, int W, int C, const uint16_t* dy, const uint16_t* in, float* dw, float* db,
                            hipStream_t st) {
  const ConvShape s = shape_of(B, H, W, C);
  const int64_t M = (int64_t)B * s.OH * s.OW;
  int64_t gy = (M + kWPix - 1) / kWPix;
  if (gy > 64) gy = 64;
  hipLaunchKernelGGL(k_conv_bwd_weight, dim3((unsigned)(s.KP / 64 + (s.KP % 64 ? 1 : 0)), (unsigned)gy), dim3(256), 0,
                     st, s, dy, in, dw);
  int64_t gb = (M + 1023) / 1024;
  if (gb > 256) gb = 256;
  if (gb < 1) gb = 1;
  hipLaunchKernelGGL(k_bias_grad, dim3((unsigned)gb), dim3(256), 0, st, dy, M, db);
}

void launch_head_fwd(int B, int OH, int OW, const uint16_t* act, const float* wfc, const float* bfc, float* pool,
                     float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_head_fwd, dim3((unsigned)B), dim3(64), 0, st, act, OH, OW, wfc, bfc, pool, out);
}

void launch_head_bwd(int B, int OH, int OW, const float* out, const float* label, const float* scale,
                     const float* pool, const float* wfc, const uint16_t* act, const float* dout, float* dwfc,
                     float* dbfc, uint16_t* dact, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_head_bwd, dim3((unsigned)B), dim3(64), 0, st, out, label, scale, B, pool, wfc, act, OH, OW,
                     dout, dwfc, dbfc, dact, loss);
}

void launch_cast_weights(const float* w, int C, uint16_t* wk, uint16_t* wt, hipStream_t st) {
  const int KP = conv_kp(C);
  hipLaunchKernelGGL(k_cast_weights, dim3((unsigned)((64 * KP + 255) / 256)), dim3(256), 0, st, w, C, KP, wk, wt);
}

void launch_pack_input(const float* rc, const float* rd, const float* oc, const float* od, int H, int W, int f,
                       float depth_scale, uint16_t* out, hipStream_t st) {
  const int n = (W / f) * (H / f);
  hipLaunchKernelGGL(k_pack_input, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rc, rd, oc, od, H, W, f,
                     depth_scale, out);
}

}  // namespace gsr
