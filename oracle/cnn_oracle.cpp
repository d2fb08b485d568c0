// FP64 CPU oracle for the tracking-initialisation CNN (TEST INFRASTRUCTURE
// ONLY; shares nothing with the HIP library).
//
// A 3x3 convolution with zero padding, in NCHW layout, written as its
// definition:
//   out[b, o, y, x] = bias[o] + sum_{c, ky, kx} in[b, c, s y + ky - p, s x + kx - p] w[o, c, ky, kx]
// and its exact adjoints with respect to the input, the weights and the bias.

#include <cstdint>
#include <vector>

extern "C" {

static inline int64_t idx4(int64_t a, int64_t b, int64_t c, int64_t d, int64_t B, int64_t C, int64_t D) {
  return ((a * B + b) * C + c) * D + d;
}

int orc_conv2d_fwd(int batch, int cin, int h, int w, int cout, int stride, int pad, int k, const double* in,
                   const double* wt, const double* bias, double* out) {
  const int oh = (h + 2 * pad - k) / stride + 1, ow = (w + 2 * pad - k) / stride + 1;
  for (int b = 0; b < batch; ++b)
    for (int o = 0; o < cout; ++o)
      for (int y = 0; y < oh; ++y)
        for (int x = 0; x < ow; ++x) {
          double s = bias ? bias[o] : 0.0;
          for (int c = 0; c < cin; ++c)
            for (int ky = 0; ky < k; ++ky)
              for (int kx = 0; kx < k; ++kx) {
                const int iy = stride * y + ky - pad, ix = stride * x + kx - pad;
                if (iy < 0 || iy >= h || ix < 0 || ix >= w) continue;
                s += in[idx4(b, c, iy, ix, cin, h, w)] * wt[idx4(o, c, ky, kx, cin, k, k)];
              }
          out[idx4(b, o, y, x, cout, oh, ow)] = s;
        }
  return 0;
}

// Adjoint: given dL/dout, accumulate dL/din (may be NULL), dL/dw, dL/dbias (may be NULL).
int orc_conv2d_bwd(int batch, int cin, int h, int w, int cout, int stride, int pad, int k, const double* in,
                   const double* wt, const double* dout, double* din, double* dw, double* dbias) {
  const int oh = (h + 2 * pad - k) / stride + 1, ow = (w + 2 * pad - k) / stride + 1;
  if (din)
    for (int64_t i = 0; i < (int64_t)batch * cin * h * w; ++i) din[i] = 0.0;
  for (int64_t i = 0; i < (int64_t)cout * cin * k * k; ++i) dw[i] = 0.0;
  if (dbias)
    for (int o = 0; o < cout; ++o) dbias[o] = 0.0;
  for (int b = 0; b < batch; ++b)
    for (int o = 0; o < cout; ++o)
      for (int y = 0; y < oh; ++y)
        for (int x = 0; x < ow; ++x) {
          const double g = dout[idx4(b, o, y, x, cout, oh, ow)];
          if (dbias) dbias[o] += g;
          for (int c = 0; c < cin; ++c)
            for (int ky = 0; ky < k; ++ky)
              for (int kx = 0; kx < k; ++kx) {
                const int iy = stride * y + ky - pad, ix = stride * x + kx - pad;
                if (iy < 0 || iy >= h || ix < 0 || ix >= w) continue;
                dw[idx4(o, c, ky, kx, cin, k, k)] += g * in[idx4(b, c, iy, ix, cin, h, w)];
                if (din) din[idx4(b, c, iy, ix, cin, h, w)] += g * wt[idx4(o, c, ky, kx, cin, k, k)];
              }
        }
  return 0;
}

}  // extern "C"
