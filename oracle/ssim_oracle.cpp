// FP64 CPU oracle for the structural-similarity term of the mapping colour
// loss (Gaussian-SLAM Eq. 10: L_color = (1 - lambda) |I^ - I|_1 +
// lambda (1 - SSIM(I^, I)), with SSIM as defined by Wang et al. 2004).
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call
// this file; only the tests and the benchmark's CPU-baseline leg do. It shares
// no code, header, table or helper with the HIP library.
//
// Definition used (the paper names SSIM and its source without parameters;
// these are the source's standard settings):
//   * per channel and per pixel p, a local window of 11 x 11 positions centred
//     on p with circular-symmetric Gaussian weights w (sigma = 1.5), normalised
//     so that the 121 weights sum to one;
//   * window positions outside the image hold the value 0 (zero padding);
//   * weighted local statistics over the window:
//       mu_x = sum w x,  sigma_x^2 = sum w (x - mu_x)^2,
//       sigma_xy = sum w (x - mu_x)(y - mu_y), and likewise for y;
//   * SSIM(p) = (2 mu_x mu_y + C1)(2 sigma_xy + C2) /
//               ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)),
//     C1 = (0.01 L)^2, C2 = (0.03 L)^2 with dynamic range L = 1;
//   * SSIM(I^, I) is the mean of SSIM(p) over all channels and pixels.
// The gradient of that mean with respect to x = I^ follows the chain rule
// through the statistics: with sum w = 1 over the full window,
//   d mu_x / d x_q = w_q,  d sigma_x^2 / d x_q = 2 w_q (x_q - mu_x),
//   d sigma_xy / d x_q = w_q (y_q - mu_y)
// for every in-image position q of p's window, and the partials of SSIM(p)
// with respect to (mu_x, sigma_x^2, sigma_xy) are taken from the quotient
// above as written.

#include <cmath>
#include <cstdint>
#include <vector>

extern "C" {

// X, Y: [C, H, W] row-major. map: [C, H, W] SSIM(p) or NULL. mean: SSIM(X, Y).
// dmean_dX: [C, H, W] gradient of the mean with respect to X, or NULL.
int orc_ssim(int C, int H, int W, const double* X, const double* Y, double* map, double* mean, double* dmean_dX) {
  if (C < 0 || H < 0 || W < 0 || !mean) return -1;
  const int R = 5;  // window half-width: 11 x 11 positions
  const double sigma = 1.5, c1 = 0.01 * 0.01, c2 = 0.03 * 0.03;
  double w[11][11], wsum = 0.0;
  for (int i = 0; i < 11; ++i)
    for (int j = 0; j < 11; ++j) {
      const double di = i - R, dj = j - R;
      w[i][j] = std::exp(-(di * di + dj * dj) / (2.0 * sigma * sigma));
      wsum += w[i][j];
    }
  for (int i = 0; i < 11; ++i)
    for (int j = 0; j < 11; ++j) w[i][j] /= wsum;

  const int64_t plane = (int64_t)H * W, n = (int64_t)C * plane;
  if (dmean_dX)
    for (int64_t i = 0; i < n; ++i) dmean_dX[i] = 0.0;
  double total = 0.0;
  for (int c = 0; c < C; ++c) {
    const double* x = X + c * plane;
    const double* y = Y + c * plane;
    // value at window position (py + i - R, px + j - R), 0 outside the image
    auto at = [&](const double* a, int py, int px) -> double {
      return (py < 0 || py >= H || px < 0 || px >= W) ? 0.0 : a[(int64_t)py * W + px];
    };
    for (int py = 0; py < H; ++py)
      for (int px = 0; px < W; ++px) {
        double mx = 0, my = 0;
        for (int i = 0; i < 11; ++i)
          for (int j = 0; j < 11; ++j) {
            mx += w[i][j] * at(x, py + i - R, px + j - R);
            my += w[i][j] * at(y, py + i - R, px + j - R);
          }
        double vx = 0, vy = 0, cxy = 0;
        for (int i = 0; i < 11; ++i)
          for (int j = 0; j < 11; ++j) {
            const double dx = at(x, py + i - R, px + j - R) - mx;
            const double dy = at(y, py + i - R, px + j - R) - my;
            vx += w[i][j] * dx * dx;
            vy += w[i][j] * dy * dy;
            cxy += w[i][j] * dx * dy;
          }
        const double a1 = 2.0 * mx * my + c1, a2 = 2.0 * cxy + c2;
        const double b1 = mx * mx + my * my + c1, b2 = vx + vy + c2;
        const double s = (a1 * a2) / (b1 * b2);
        if (map) map[c * plane + (int64_t)py * W + px] = s;
        total += s;
        if (!dmean_dX) continue;
        // partials of s with respect to mu_x, sigma_x^2 and sigma_xy
        const double ds_dmx = s * (2.0 * my / a1 - 2.0 * mx / b1);
        const double ds_dvx = -s / b2;
        const double ds_dcxy = 2.0 * s / a2;
        for (int i = 0; i < 11; ++i)
          for (int j = 0; j < 11; ++j) {
            const int qy = py + i - R, qx = px + j - R;
            if (qy < 0 || qy >= H || qx < 0 || qx >= W) continue;
            const int64_t q = (int64_t)qy * W + qx;
            const double g = ds_dmx * w[i][j] + ds_dvx * 2.0 * w[i][j] * (x[q] - mx) +
                             ds_dcxy * w[i][j] * (y[q] - my);
            dmean_dX[c * plane + q] += g / (double)n;
          }
      }
  }
  *mean = n > 0 ? total / (double)n : 1.0;
  return 0;
}

}  // extern "C"
