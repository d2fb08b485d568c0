// FP64 CPU oracle for differentiable Gaussian rasterization (Gaussian-SLAM,
// arXiv 2312.10070, Sec. 3.1 "Gaussian Splatting" and Sec. 3.3 "Geometry and
// Color Encoding", Sec. 3.4 "Tracking").
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call
// this file; only the tests, the smoke check and the CPU-baseline leg of the
// benchmark do. It shares no code, header, table or helper with the HIP
// library: every formula here is written out from the paper's definitions in
// plain double precision, with no blocking, fusion or reordering.
//
// What it computes (per the paper; where the paper is silent, the reading taken
// is stated beside the code that applies it):
//   * projection of each Gaussian: camera-space mean (Eq. 1, world-to-camera
//     pose), EWA 2D covariance Sigma' = J R Sigma R^T J^T + h I (Eq. 2) with
//     Sigma = R S S^T R^T (Sec. 3.1), its inverse (the conic) and a support box
//     outside which alpha < alpha_min exactly;
//   * per pixel, brute-force front-to-back compositing of ALL depth-ordered
//     Gaussians: colour (Eq. 3), alpha (Eq. 4), depth (Eq. 6) and the
//     accumulated alpha 1 - T_final;
//   * the analytic backward of those outputs (Eq. 7, Eq. 8 and the colour,
//     alpha and direct-depth analogues) chained to means, scales, quaternions,
//     opacities, colours and the camera pose (quaternion + translation, and a
//     left-perturbation twist);
//   * the L1 mapping loss (Eq. 9, L1 part of Eq. 10), the isotropic scale
//     regulariser (Eq. 11) and the masked tracking loss (Eq. 15, with the
//     inlier and alpha^3 masks of the supplement);
//   * one Adam step (Kingma & Ba), the optimiser both loops use.
//
// "Several results are correct" handling: a discrete decision whose FP64
// margin is within a relative band `amb_rel` (alpha vs alpha_min, T' vs T_min,
// raw alpha vs alpha_max), or the order of two consecutive candidates whose
// depths agree within `amb_z`, is an ambiguity event. In the forward, a pixel
// with exactly one event also gets the result with that decision flipped (the
// pair swapped, for an order event) as "alt"; two or more events mark its
// image values unverifiable. In the backward, every decision path of a pixel
// with events is enumerated (each branch flips a subset of the events met on
// its own path) and the per-element maximum of |branch - primary| over the
// branches feeds a slack; only a pixel with more than kMaxEventBits events is
// unverifiable there.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

struct Cam {
  int W, H;
  double fx, fy, cx, cy, near_z;
  double bg[3];
};

struct Opt {
  double lowpass, amin, amax, tmin, guard;
  int tw, th;
  double amb_rel, amb_z;
};

Cam read_cam(const double* c) {
  Cam k;
  k.W = (int)c[0];
  k.H = (int)c[1];
  k.fx = c[2];
  k.fy = c[3];
  k.cx = c[4];
  k.cy = c[5];
  k.near_z = c[6];
  k.bg[0] = c[7];
  k.bg[1] = c[8];
  k.bg[2] = c[9];
  return k;
}

Opt read_opt(const double* o) {
  Opt k;
  k.lowpass = o[0];
  k.amin = o[1];
  k.amax = o[2];
  k.tmin = o[3];
  k.guard = o[4];
  k.tw = (int)o[5];
  k.th = (int)o[6];
  k.amb_rel = o[7];
  k.amb_z = o[8];
  return k;
}

// Rotation matrix of a unit quaternion (w, x, y, z), row-major.
void quat_to_R(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

// d/dq of sum_ij G_ij R_ij(q) for the formula above (q treated as free).
void quat_to_R_vjp(const double q[4], const double G[9], double gq[4]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  // Partial derivatives of each R entry, written out entry by entry.
  const double dRdw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
  const double dRdx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
  const double dRdy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
  const double dRdz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
  gq[0] = gq[1] = gq[2] = gq[3] = 0;
  for (int i = 0; i < 9; ++i) {
    gq[0] += G[i] * dRdw[i];
    gq[1] += G[i] * dRdx[i];
    gq[2] += G[i] * dRdy[i];
    gq[3] += G[i] * dRdz[i];
  }
}

// Gradient through q_hat = q / |q|.
void normalize_vjp(const double q[4], const double g_hat[4], double gq[4]) {
  const double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double qh[4], d = 0;
  for (int i = 0; i < 4; ++i) {
    qh[i] = q[i] / n;
    d += qh[i] * g_hat[i];
  }
  for (int i = 0; i < 4; ++i) gq[i] = (g_hat[i] - qh[i] * d) / n;
}

// C = A * B for 3x3 row-major.
void mm3(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
      C[i * 3 + j] = s;
    }
}
void transpose3(const double* A, double* T) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T[j * 3 + i] = A[i * 3 + j];
}

struct Pose {
  double q[4];   // as given
  double qh[4];  // normalised
  double R[9];
  double t[3];
  bool ok;
};

Pose read_pose(const double* p7) {
  Pose P;
  for (int i = 0; i < 4; ++i) P.q[i] = p7[i];
  for (int i = 0; i < 3; ++i) P.t[i] = p7[4 + i];
  const double n = std::sqrt(P.q[0] * P.q[0] + P.q[1] * P.q[1] + P.q[2] * P.q[2] + P.q[3] * P.q[3]);
  P.ok = n > 0 && std::isfinite(n);
  for (int i = 0; i < 4; ++i) P.qh[i] = P.ok ? P.q[i] / n : 0;
  quat_to_R(P.qh, P.R);
  return P;
}

// Everything the forward and backward need about one Gaussian.
struct Proj {
  bool valid;
  double x[3];  // camera-space mean
  double u, v;
  double Sp[3];  // Sigma' (xx, xy, yy) including the low-pass term
  double a, b, c;  // conic = inverse of Sigma' (xx, xy, yy)
  double o, col[3];
  double smax;  // support level: alpha >= alpha_min only where sigma <= smax
  int px0, px1, py0, py1;  // pixel support box (inclusive)
  int tx0, tx1, ty0, ty1;  // tile rectangle (inclusive)
  double margin;           // distance of the box edges to the nearest integer
  // intermediates kept for the backward
  double qh[4], q[4], s[3], R[9], Sig[9], Sigc[9], J[6];
  bool clx, cly;
  double Xc, Yc;  // clamped x/z and y/z used inside J
};

double frac_dist(double t) { return std::fabs(t - std::nearbyint(t)); }

Proj project_one(int64_t k, const double* means, const double* scales, const double* quats,
                 const double* opac, const double* colors, const Pose& P, const Cam& cam,
                 const Opt& opt) {
  Proj g;
  std::memset(&g, 0, sizeof(g));
  g.valid = false;
  if (!P.ok) return g;
  const double* q = quats + 4 * k;
  const double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!(n > 0) || !std::isfinite(n)) return g;
  for (int i = 0; i < 4; ++i) {
    g.q[i] = q[i];
    g.qh[i] = q[i] / n;
  }
  quat_to_R(g.qh, g.R);
  for (int i = 0; i < 3; ++i) g.s[i] = scales[3 * k + i];
  // Sigma = R diag(s^2) R^T (Sec. 3.1, covariance decomposition)
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int m = 0; m < 3; ++m) acc += g.R[i * 3 + m] * g.s[m] * g.s[m] * g.R[j * 3 + m];
      g.Sig[i * 3 + j] = acc;
    }
  // Camera-space mean x = R_p mu + t_p (Eq. 1, world-to-camera)
  const double* mu = means + 3 * k;
  for (int i = 0; i < 3; ++i)
    g.x[i] = P.R[i * 3 + 0] * mu[0] + P.R[i * 3 + 1] * mu[1] + P.R[i * 3 + 2] * mu[2] + P.t[i];
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(g.x[i])) return g;
  const double z = g.x[2];
  if (!(z > cam.near_z)) return g;
  g.u = cam.fx * g.x[0] / z + cam.cx;
  g.v = cam.fy * g.x[1] / z + cam.cy;
  // Local affine Jacobian of the perspective projection (Eq. 2), with the
  // lateral coordinate clamped to a guard band beyond the image.
  const double limx = opt.guard * std::max(cam.cx, cam.W - cam.cx) / cam.fx;
  const double limy = opt.guard * std::max(cam.cy, cam.H - cam.cy) / cam.fy;
  const double X = g.x[0] / z, Y = g.x[1] / z;
  g.clx = (X < -limx) || (X > limx);
  g.cly = (Y < -limy) || (Y > limy);
  g.Xc = std::min(limx, std::max(-limx, X));
  g.Yc = std::min(limy, std::max(-limy, Y));
  g.J[0] = cam.fx / z;
  g.J[1] = 0;
  g.J[2] = -cam.fx * g.Xc / z;
  g.J[3] = 0;
  g.J[4] = cam.fy / z;
  g.J[5] = -cam.fy * g.Yc / z;
  // Sigma_c = R_p Sigma R_p^T
  double Rt[9], tmp[9];
  transpose3(P.R, Rt);
  mm3(P.R, g.Sig, tmp);
  mm3(tmp, Rt, g.Sigc);
  // Sigma' = J Sigma_c J^T + h I
  double JS[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int m = 0; m < 3; ++m) acc += g.J[i * 3 + m] * g.Sigc[m * 3 + j];
      JS[i * 3 + j] = acc;
    }
  double S2[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double acc = 0;
      for (int m = 0; m < 3; ++m) acc += JS[i * 3 + m] * g.J[j * 3 + m];
      S2[i * 2 + j] = acc;
    }
  g.Sp[0] = S2[0] + opt.lowpass;
  g.Sp[1] = 0.5 * (S2[1] + S2[2]);
  g.Sp[2] = S2[3] + opt.lowpass;
  const double det = g.Sp[0] * g.Sp[2] - g.Sp[1] * g.Sp[1];
  if (!(det > 0) || !std::isfinite(det)) return g;
  g.a = g.Sp[2] / det;
  g.b = -g.Sp[1] / det;
  g.c = g.Sp[0] / det;
  g.o = opac[k];
  for (int i = 0; i < 3; ++i) g.col[i] = colors[3 * k + i];
  // Support: o exp(-sigma) >= alpha_min needs sigma <= ln(o / alpha_min);
  // for |dx| > sqrt(2 s Sigma'_xx) the minimum of sigma over dy already
  // exceeds s, so a box of half-widths sqrt(2 s Sigma'_xx), sqrt(2 s Sigma'_yy)
  // with s >= smax is conservative. The box only selects work (which pixels
  // and tiles a Gaussian is evaluated on), so any conservative s gives the
  // same image; s = (1 + 1e-3) smax + 1e-3 keeps alpha below alpha_min by a
  // factor e^-0.001 outside the box, so binary32 evaluation cannot reach
  // alpha_min there either.
  if (!(g.o >= opt.amin) || !std::isfinite(g.o)) return g;
  g.smax = std::log(g.o / opt.amin);
  const double sbox = (1.0 + 1e-3) * g.smax + 1e-3;
  const double rx = std::sqrt(2.0 * sbox * g.Sp[0]);
  const double ry = std::sqrt(2.0 * sbox * g.Sp[2]);
  const double ex0 = g.u - rx, ex1 = g.u + rx, ey0 = g.v - ry, ey1 = g.v + ry;
  if (!std::isfinite(ex0) || !std::isfinite(ex1) || !std::isfinite(ey0) || !std::isfinite(ey1)) return g;
  const double fx0 = std::max(0.0, std::ceil(ex0));
  const double fx1 = std::min((double)(cam.W - 1), std::floor(ex1));
  const double fy0 = std::max(0.0, std::ceil(ey0));
  const double fy1 = std::min((double)(cam.H - 1), std::floor(ey1));
  g.margin = std::min(std::min(frac_dist(ex0), frac_dist(ex1)), std::min(frac_dist(ey0), frac_dist(ey1)));
  if (fx0 > fx1 || fy0 > fy1) return g;
  g.px0 = (int)fx0;
  g.px1 = (int)fx1;
  g.py0 = (int)fy0;
  g.py1 = (int)fy1;
  g.tx0 = g.px0 / opt.tw;
  g.tx1 = g.px1 / opt.tw;
  g.ty0 = g.py0 / opt.th;
  g.ty1 = g.py1 / opt.th;
  g.valid = true;
  return g;
}

struct Scene {
  int64_t n;
  const double *means, *scales, *quats, *opac, *colors;
  Pose P;
  Cam cam;
  Opt opt;
  std::vector<Proj> proj;
  std::vector<int64_t> order;  // valid Gaussians by (z ascending, index ascending)
};

void build_scene(Scene& S, int nthreads) {
  S.proj.resize(S.n);
  auto work = [&](int64_t b, int64_t e) {
    for (int64_t k = b; k < e; ++k)
      S.proj[k] = project_one(k, S.means, S.scales, S.quats, S.opac, S.colors, S.P, S.cam, S.opt);
  };
  if (nthreads <= 1 || S.n < 4096) {
    work(0, S.n);
  } else {
    std::vector<std::thread> th;
    const int64_t chunk = (S.n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
      const int64_t b = t * chunk, e = std::min(S.n, b + chunk);
      if (b < e) th.emplace_back(work, b, e);
    }
    for (auto& x : th) x.join();
  }
  S.order.clear();
  for (int64_t k = 0; k < S.n; ++k)
    if (S.proj[k].valid) S.order.push_back(k);
  std::stable_sort(S.order.begin(), S.order.end(), [&](int64_t i, int64_t j) {
    if (S.proj[i].x[2] != S.proj[j].x[2]) return S.proj[i].x[2] < S.proj[j].x[2];
    return i < j;
  });
}

// One composited pair of a pixel (what the backward needs).
struct Pair {
  int64_t id;
  double alpha, T, e, dx, dy;
  bool clamped;
};

struct PixResult {
  double C[3], D, A, T;
  int ncomp;
  int events;       // ambiguity events met on this branch
  uint64_t hash;    // fingerprint of every discrete decision
  std::vector<Pair> pairs;
  std::vector<int64_t> cand;  // Gaussians that may be composited on some branch (keep_pairs only)
  bool tie3;        // three or more consecutive candidates chained by depth ties
};

// Branches are enumerated over at most this many events per pixel.
constexpr int kMaxEventBits = 10;

// Front-to-back compositing of one pixel (Eq. 3, Eq. 4, Eq. 6). Bit e of
// `flips` inverts the decision of ambiguity event e (counted from 0, in
// processing order along this branch); 0 = the primary branch. Events: alpha within amb_rel of alpha_max (clamp) or of
// alpha_min (skip), T' within amb_rel of T_min (stop), and two consecutive
// candidates that both may be composited and whose depths agree within amb_z
// (their order; the flipped branch composites them swapped).
void composite_pixel(const Scene& S, int px, int py, bool pruned, uint64_t flips, bool keep_pairs,
                     PixResult& r) {
  auto flipped = [flips](int ev) { return ev < 64 && ((flips >> ev) & 1ull); };
  const Opt& opt = S.opt;
  // candidates in depth order
  std::vector<int64_t> cand;
  std::vector<double> raw_alpha;
  for (int64_t k : S.order) {
    const Proj& g = S.proj[k];
    if (pruned && (px < g.px0 || px > g.px1 || py < g.py0 || py > g.py1)) continue;
    const double dx = px - g.u, dy = py - g.v;
    const double sigma = 0.5 * (g.a * dx * dx + g.c * dy * dy) + g.b * dx * dy;
    const double a = std::min(opt.amax, g.o * std::exp(-sigma));
    if (a < opt.amin * (1.0 - opt.amb_rel)) continue;  // certainly skipped
    cand.push_back(k);
    raw_alpha.push_back(a);
  }
  double T = 1.0, C[3] = {0, 0, 0}, D = 0;
  int ev = 0, nc = 0;
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
  };
  r.pairs.clear();
  if (keep_pairs) r.cand = cand;
  // Adjacent swaps reach both orders of a tied pair but not every order of a
  // longer tie chain; such a pixel is flagged (its backward is unverifiable).
  r.tie3 = false;
  for (size_t i = 0; i + 2 < cand.size(); ++i) {
    const double z0 = S.proj[cand[i]].x[2], z1 = S.proj[cand[i + 1]].x[2], z2 = S.proj[cand[i + 2]].x[2];
    if (std::fabs(z1 - z0) <= opt.amb_z * z1 && std::fabs(z2 - z1) <= opt.amb_z * z2) r.tie3 = true;
  }
  for (size_t i = 0; i < cand.size(); ++i) {
    // an order event with the next candidate
    if (i + 1 < cand.size()) {
      const double za = S.proj[cand[i]].x[2], zb = S.proj[cand[i + 1]].x[2];
      if (std::fabs(zb - za) <= opt.amb_z * zb) {
        if (flipped(ev)) {
          std::swap(cand[i], cand[i + 1]);
          std::swap(raw_alpha[i], raw_alpha[i + 1]);
        }
        ++ev;
      }
    }
    const int64_t k = cand[i];
    const Proj& g = S.proj[k];
    const double dx = px - g.u, dy = py - g.v;
    const double sigma = 0.5 * (g.a * dx * dx + g.c * dy * dy) + g.b * dx * dy;
    const double e = std::exp(-sigma);
    const double raw = g.o * e;
    bool clamped = raw > opt.amax;
    if (std::fabs(raw - opt.amax) <= opt.amb_rel * opt.amax) {
      if (flipped(ev)) clamped = !clamped;
      ++ev;
    }
    const double alpha = std::min(opt.amax, raw);
    bool skip = alpha < opt.amin;
    if (std::fabs(alpha - opt.amin) <= opt.amb_rel * opt.amin) {
      if (flipped(ev)) skip = !skip;
      ++ev;
    }
    if (skip) continue;
    const double Tn = T * (1.0 - alpha);
    bool stop = Tn < opt.tmin;
    if (std::fabs(Tn - opt.tmin) <= opt.amb_rel * opt.tmin) {
      if (flipped(ev)) stop = !stop;
      ++ev;
    }
    mix((uint64_t)k * 4 + (stop ? 1 : 0) + (clamped ? 2 : 0));
    if (stop) break;
    for (int ch = 0; ch < 3; ++ch) C[ch] += g.col[ch] * alpha * T;
    D += g.x[2] * alpha * T;
    if (keep_pairs) r.pairs.push_back(Pair{k, alpha, T, e, dx, dy, clamped});
    T = Tn;
    ++nc;
  }
  for (int ch = 0; ch < 3; ++ch) r.C[ch] = C[ch] + T * S.cam.bg[ch];
  r.D = D;
  r.A = 1.0 - T;
  r.T = T;
  r.ncomp = nc;
  r.events = ev;
  r.hash = h;
}

// Per-pair partial derivatives of the three outputs, reduced with the upstream
// gradients, accumulated into per-Gaussian 2D gradients
//   g2d = (u, v, conic_a, conic_b, conic_c, opacity, r, g, b, z_direct).
// Derivatives (for the composited list j = 1..m, T_j = prod_{k<j}(1 - alpha_k)):
//   dC/dc_j = alpha_j T_j, dD/dz_j (direct) = alpha_j T_j,
//   dC/dalpha_j = c_j T_j - (sum_{u>j} c_u alpha_u T_u + T_fin bg) / (1 - alpha_j),
//   dD/dalpha_j = z_j T_j - (sum_{u>j} z_u alpha_u T_u) / (1 - alpha_j)   (Eq. 8),
//   dA/dalpha_j = T_fin / (1 - alpha_j).
struct G2 {
  int64_t id;
  double g[10];
};

// Rounding error bound of an FP32 evaluation of the screen position (Eq. 1):
// each coordinate of the camera-space mean x = R mu + t carries a few ulps of
// |R||mu| + |t|, and u = fx x / z + cx a few ulps of |u| more (eight and four
// ulps are taken).
void screen_delta(const Scene& S, const Proj& g, double& du, double& dv) {
  const double ulp = std::ldexp(1.0, -24);
  // |R mu| = |mu| <= |x| + |t| (R is a rotation), so |R||mu| + |t| <= |x| + 2 |t|
  const double tn = std::sqrt(S.P.t[0] * S.P.t[0] + S.P.t[1] * S.P.t[1] + S.P.t[2] * S.P.t[2]);
  const double xn = std::sqrt(g.x[0] * g.x[0] + g.x[1] * g.x[1] + g.x[2] * g.x[2]);
  const double dcam = 8 * ulp * (xn + 2 * tn);
  const double z = g.x[2];
  du = 4 * ulp * std::fabs(g.u) + S.cam.fx / z * (dcam + std::fabs(g.x[0] / z) * dcam);
  dv = 4 * ulp * std::fabs(g.v) + S.cam.fy / z * (dcam + std::fabs(g.x[1] / z) * dcam);
}

// With `mag` non-NULL it also receives, per pair, the same ten terms with every
// factor replaced by its magnitude and every sum (in particular the two terms
// of dC/dalpha and Eq. 8, which nearly cancel where a Gaussian matches what
// lies behind it) by the sum of magnitudes: the scale FP32 rounding acts on.
// *kappa_out receives the pixel's transmittance condition number
// kappa = 1 + sum_k alpha_k / (1 - alpha_k): a relative error e in every
// alpha_k moves every T_j = prod_{k<j} (1 - alpha_k) by at most kappa e, since
// d(1 - alpha_k) / (1 - alpha_k) = -alpha_k e / (1 - alpha_k).
//
// With `pos` non-NULL it receives, per pair, a first-order bound of how much
// the ten terms move when the Gaussian's screen position (u, v) carries the
// rounding error of its FP32 evaluation, delta_u and delta_v (screen_delta):
// next to a Gaussian's centre, dx = px - u is small and that rounding is a
// large part of it.
void pixel_backward(const Scene& S, const PixResult& r, const double gC[3], double gD, double gA,
                    std::vector<G2>& out, std::vector<G2>* mag = nullptr, std::vector<G2>* pos = nullptr,
                    double* kappa_out = nullptr) {
  out.clear();
  if (mag) mag->clear();
  if (pos) pos->clear();
  double SC[3], SD = 0, MC[3], MD = 0;
  for (int ch = 0; ch < 3; ++ch) {
    SC[ch] = r.T * S.cam.bg[ch];
    MC[ch] = std::fabs(SC[ch]);
  }
  const double Tfin = r.T;
  if (kappa_out) {
    double kappa = 1.0;
    for (const Pair& p : r.pairs) kappa += p.alpha / (1.0 - p.alpha);
    *kappa_out = kappa;
  }
  for (int j = (int)r.pairs.size() - 1; j >= 0; --j) {
    const Pair& p = r.pairs[j];
    const Proj& g = S.proj[p.id];
    G2 c, m;
    c.id = m.id = p.id;
    for (int f = 0; f < 10; ++f) c.g[f] = m.g[f] = 0;
    const double w = p.alpha * p.T;
    for (int ch = 0; ch < 3; ++ch) c.g[6 + ch] = w * gC[ch];
    c.g[9] = w * gD;
    const double inv = 1.0 / (1.0 - p.alpha);
    double dA = 0, mA = 0;
    for (int ch = 0; ch < 3; ++ch) {
      dA += gC[ch] * (g.col[ch] * p.T - SC[ch] * inv);
      mA += std::fabs(gC[ch]) * (std::fabs(g.col[ch]) * p.T + MC[ch] * inv);
    }
    dA += gD * (g.x[2] * p.T - SD * inv);
    mA += std::fabs(gD) * (std::fabs(g.x[2]) * p.T + MD * inv);
    dA += gA * Tfin * inv;
    mA += std::fabs(gA) * Tfin * inv;
    for (int ch = 0; ch < 3; ++ch) {
      SC[ch] += g.col[ch] * w;
      MC[ch] += std::fabs(g.col[ch]) * w;
    }
    SD += g.x[2] * w;
    MD += std::fabs(g.x[2]) * w;
    if (!p.clamped) {
      c.g[5] = dA * p.e;  // d alpha / d o = exp(-sigma)
      const double gs = -dA * p.alpha;  // d alpha / d sigma = -alpha
      c.g[2] = gs * 0.5 * p.dx * p.dx;
      c.g[3] = gs * p.dx * p.dy;
      c.g[4] = gs * 0.5 * p.dy * p.dy;
      c.g[0] = gs * -(g.a * p.dx + g.b * p.dy);
      c.g[1] = gs * -(g.b * p.dx + g.c * p.dy);
      if (mag) {
        const double ms = mA * p.alpha;
        m.g[5] = mA * p.e;
        m.g[2] = ms * 0.5 * p.dx * p.dx;
        m.g[3] = ms * std::fabs(p.dx * p.dy);
        m.g[4] = ms * 0.5 * p.dy * p.dy;
        m.g[0] = ms * (std::fabs(g.a * p.dx) + std::fabs(g.b * p.dy));
        m.g[1] = ms * (std::fabs(g.b * p.dx) + std::fabs(g.c * p.dy));
      }
    }
    out.push_back(c);
    if (mag) {
      for (int f = 6; f < 10; ++f) m.g[f] = std::fabs(c.g[f]);
      mag->push_back(m);
    }
    if (pos) {
      double du, dv;
      screen_delta(S, g, du, dv);
      G2 d;
      d.id = p.id;
      // alpha moves by alpha |d sigma / d(u, v)| (delta_u, delta_v); every term is linear in alpha
      const double ea = std::fabs(g.a * p.dx + g.b * p.dy) * du + std::fabs(g.b * p.dx + g.c * p.dy) * dv;
      for (int f = 0; f < 10; ++f) d.g[f] = std::fabs(c.g[f]) * ea;
      if (!p.clamped) {
        const double as = std::fabs(dA * p.alpha);
        d.g[0] += as * (std::fabs(g.a) * du + std::fabs(g.b) * dv);
        d.g[1] += as * (std::fabs(g.b) * du + std::fabs(g.c) * dv);
        d.g[2] += as * std::fabs(p.dx) * du;
        d.g[3] += as * (std::fabs(p.dy) * du + std::fabs(p.dx) * dv);
        d.g[4] += as * std::fabs(p.dy) * dv;
      }
      pos->push_back(d);
    }
  }
}

// Chain the 2D gradient of one Gaussian to its 3D parameters and to the pose.
// out3d: means(3) scales(3) quats(4) opacity(1) colors(3) = 14 values.
// pose7: d/d(qw,qx,qy,qz,tx,ty,tz); tw6: left-perturbation twist (rho, phi).
void chain_3d(const Scene& S, int64_t k, const double g2[10], double out3d[14], double pose7[7],
              double tw6[6]) {
  const Proj& g = S.proj[k];
  const Cam& cam = S.cam;
  const Pose& P = S.P;
  const double z = g.x[2];
  // conic -> Sigma': with A = Sigma'^{-1}, dL/dSigma' = -A M A where M is the
  // symmetric matrix gradient w.r.t. A (off-diagonal entries carry half of the
  // gradient of the single conic_b parameter).
  const double A[4] = {g.a, g.b, g.b, g.c};
  const double M[4] = {g2[2], 0.5 * g2[3], 0.5 * g2[3], g2[4]};
  double AM[4], GS[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) AM[i * 2 + j] = A[i * 2 + 0] * M[0 * 2 + j] + A[i * 2 + 1] * M[1 * 2 + j];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) GS[i * 2 + j] = -(AM[i * 2 + 0] * A[0 * 2 + j] + AM[i * 2 + 1] * A[1 * 2 + j]);
  // Sigma' = J Sigma_c J^T + h I:  dL/dJ = 2 GS J Sigma_c,  dL/dSigma_c = J^T GS J
  double JSc[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int m = 0; m < 3; ++m) acc += g.J[i * 3 + m] * g.Sigc[m * 3 + j];
      JSc[i * 3 + j] = acc;
    }
  double GJ[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) GJ[i * 3 + j] = 2.0 * (GS[i * 2 + 0] * JSc[0 * 3 + j] + GS[i * 2 + 1] * JSc[1 * 3 + j]);
  double GSc[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) acc += g.J[p * 3 + i] * GS[p * 2 + q] * g.J[q * 3 + j];
      GSc[i * 3 + j] = acc;
    }
  // J -> camera coordinates
  double gx[3] = {0, 0, 0};
  gx[2] += GJ[0] * (-cam.fx / (z * z));
  gx[2] += GJ[4] * (-cam.fy / (z * z));
  if (!g.clx) {
    gx[0] += GJ[2] * (-cam.fx / (z * z));
    gx[2] += GJ[2] * (2.0 * cam.fx * g.x[0] / (z * z * z));
  } else {
    gx[2] += GJ[2] * (cam.fx * g.Xc / (z * z));
  }
  if (!g.cly) {
    gx[1] += GJ[5] * (-cam.fy / (z * z));
    gx[2] += GJ[5] * (2.0 * cam.fy * g.x[1] / (z * z * z));
  } else {
    gx[2] += GJ[5] * (cam.fy * g.Yc / (z * z));
  }
  // (u, v) -> camera coordinates
  gx[0] += g2[0] * cam.fx / z;
  gx[2] += g2[0] * (-cam.fx * g.x[0] / (z * z));
  gx[1] += g2[1] * cam.fy / z;
  gx[2] += g2[1] * (-cam.fy * g.x[1] / (z * z));
  // direct depth term of Eq. 6
  gx[2] += g2[9];
  // x = R_p mu + t:  dL/dmu = R_p^T gx
  for (int i = 0; i < 3; ++i) out3d[i] = P.R[0 * 3 + i] * gx[0] + P.R[1 * 3 + i] * gx[1] + P.R[2 * 3 + i] * gx[2];
  // Sigma_c = R_p Sigma R_p^T:  dL/dSigma = R_p^T GSc R_p
  double Rt[9], tmp[9], GSig[9];
  transpose3(P.R, Rt);
  mm3(Rt, GSc, tmp);
  mm3(tmp, P.R, GSig);
  // Sigma = (R diag s)(R diag s)^T:  dL/d(R diag s) = 2 GSig (R diag s)
  double Ms[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Ms[i * 3 + j] = g.R[i * 3 + j] * g.s[j];
  double GM[9];
  mm3(GSig, Ms, GM);
  for (int i = 0; i < 9; ++i) GM[i] *= 2.0;
  double GR[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) GR[i * 3 + j] = GM[i * 3 + j] * g.s[j];
  for (int j = 0; j < 3; ++j) {
    double acc = 0;
    for (int i = 0; i < 3; ++i) acc += GM[i * 3 + j] * g.R[i * 3 + j];
    out3d[3 + j] = acc;
  }
  double gqh[4], gq[4];
  quat_to_R_vjp(g.qh, GR, gqh);
  normalize_vjp(g.q, gqh, gq);
  for (int i = 0; i < 4; ++i) out3d[6 + i] = gq[i];
  out3d[10] = g2[5];
  for (int i = 0; i < 3; ++i) out3d[11 + i] = g2[6 + i];
  // Pose: dL/dR_p = gx mu^T + 2 GSc R_p Sigma ; dL/dt = gx
  const double* mu = S.means + 3 * k;
  double GRp[9];
  double RS[9], GRS[9];
  mm3(P.R, g.Sig, RS);
  mm3(GSc, RS, GRS);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) GRp[i * 3 + j] = gx[i] * mu[j] + 2.0 * GRS[i * 3 + j];
  double gqph[4], gqp[4];
  quat_to_R_vjp(P.qh, GRp, gqph);
  normalize_vjp(P.q, gqph, gqp);
  for (int i = 0; i < 4; ++i) pose7[i] = gqp[i];
  for (int i = 0; i < 3; ++i) pose7[4 + i] = gx[i];
  // Twist of the left perturbation T <- exp(xi^) T, xi = (rho, phi):
  //   dx = rho + phi x x  => dL/drho = gx, dL/dphi += x cross gx
  //   dSigma_c = [phi]x Sigma_c - Sigma_c [phi]x => <GSc, E_k Sigma_c - Sigma_c E_k>
  for (int i = 0; i < 3; ++i) tw6[i] = gx[i];
  tw6[3] = g.x[1] * gx[2] - g.x[2] * gx[1];
  tw6[4] = g.x[2] * gx[0] - g.x[0] * gx[2];
  tw6[5] = g.x[0] * gx[1] - g.x[1] * gx[0];
  for (int k = 0; k < 3; ++k) {
    double E[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    // E = [e_k]x
    if (k == 0) { E[5] = -1; E[7] = 1; }
    if (k == 1) { E[2] = 1; E[6] = -1; }
    if (k == 2) { E[1] = -1; E[3] = 1; }
    double ES[9], SE[9];
    mm3(E, g.Sigc, ES);
    mm3(g.Sigc, E, SE);
    double acc = 0;
    for (int i = 0; i < 9; ++i) acc += GSc[i] * (ES[i] - SE[i]);
    tw6[3 + k] += acc;
  }
}

void scene_from_args(Scene& S, int64_t n, const double* means, const double* scales, const double* quats,
                     const double* opac, const double* colors, const double* pose7, const double* cam,
                     const double* opt) {
  S.n = n;
  S.means = means;
  S.scales = scales;
  S.quats = quats;
  S.opac = opac;
  S.colors = colors;
  S.P = read_pose(pose7);
  S.cam = read_cam(cam);
  S.opt = read_opt(opt);
}

template <class F>
void parallel_for(int64_t n, int nthreads, F f) {
  if (nthreads <= 1 || n < 2) {
    f(0, 0, n);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    const int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b < e) th.emplace_back(f, t, b, e);
  }
  for (auto& x : th) x.join();
}

}  // namespace

extern "C" {

// Record layout of orc_project (double[ORC_REC] per Gaussian).
enum { ORC_REC = 24 };

int orc_project(int64_t n, const double* means, const double* scales, const double* quats,
                const double* opac, const double* colors, const double* pose7, const double* cam,
                const double* opt, double* out) {
  Scene S;
  scene_from_args(S, n, means, scales, quats, opac, colors, pose7, cam, opt);
  for (int64_t k = 0; k < n; ++k) {
    const Proj g = project_one(k, means, scales, quats, opac, colors, S.P, S.cam, S.opt);
    double* r = out + ORC_REC * k;
    r[0] = g.valid ? 1 : 0;
    r[1] = g.x[0];
    r[2] = g.x[1];
    r[3] = g.x[2];
    r[4] = g.u;
    r[5] = g.v;
    r[6] = g.Sp[0];
    r[7] = g.Sp[1];
    r[8] = g.Sp[2];
    r[9] = g.a;
    r[10] = g.b;
    r[11] = g.c;
    r[12] = g.x[2];
    r[13] = g.o;
    r[14] = g.px0;
    r[15] = g.px1;
    r[16] = g.py0;
    r[17] = g.py1;
    r[18] = g.tx0;
    r[19] = g.tx1;
    r[20] = g.ty0;
    r[21] = g.ty1;
    r[22] = g.margin;
    r[23] = g.smax;
  }
  return 0;
}

// Forward render. mode 0 = pure brute force over all Gaussians, 1 = skip
// Gaussians whose support box misses the pixel (identical by construction).
// pix = NULL renders every pixel, else only the npix listed linear indices.
// Outputs are full-size planar arrays; unlisted pixels are left untouched.
// amb: 0 = no ambiguity, 1 = one event (alt_* hold the flipped branch),
//      2 = unverifiable image values (two or more events).
int orc_render(int64_t n, const double* means, const double* scales, const double* quats,
               const double* opac, const double* colors, const double* pose7, const double* cam,
               const double* opt, int mode, int64_t npix, const int64_t* pix, int nthreads,
               double* color, double* depth, double* alpha, double* Tfin, int32_t* ncomp, int32_t* amb,
               double* alt_color, double* alt_depth, double* alt_alpha, uint64_t* dec_hash) {
  Scene S;
  scene_from_args(S, n, means, scales, quats, opac, colors, pose7, cam, opt);
  build_scene(S, nthreads);
  const int W = S.cam.W, H = S.cam.H;
  const int64_t P = (int64_t)W * H;
  const int64_t cnt = pix ? npix : P;
  parallel_for(cnt, nthreads, [&](int, int64_t b, int64_t e) {
    PixResult r, ra;
    for (int64_t i = b; i < e; ++i) {
      const int64_t p = pix ? pix[i] : i;
      const int px = (int)(p % W), py = (int)(p / W);
      composite_pixel(S, px, py, mode == 1, 0, false, r);
      for (int ch = 0; ch < 3; ++ch) color[ch * P + p] = r.C[ch];
      depth[p] = r.D;
      alpha[p] = r.A;
      if (Tfin) Tfin[p] = r.T;
      if (ncomp) ncomp[p] = r.ncomp;
      if (dec_hash) dec_hash[p] = r.hash;
      int a = r.events == 0 ? 0 : r.events == 1 ? 1 : 2;
      if (amb) amb[p] = a;
      if (a == 1) {
        composite_pixel(S, px, py, mode == 1, 1, false, ra);
        if (ra.events != 1) a = 2;
        if (amb) amb[p] = a;
      }
      if (alt_color) {
        const PixResult& src = (a == 1) ? ra : r;
        for (int ch = 0; ch < 3; ++ch) alt_color[ch * P + p] = src.C[ch];
        alt_depth[p] = src.D;
        alt_alpha[p] = src.A;
      }
    }
  });
  return 0;
}

// Analytic backward (FP64) of the render for upstream gradients gC [3,H,W],
// gD [H,W], gA [H,W] (NULL = 0) over the listed pixels (NULL = all).
// gflat / aref / slack / g2d use the flat layout
//   means 3n | scales 3n | quats 4n | opacities n | colors 3n | pose7 | twist6
// (g2d: [n,10]). aref = sum over pixels of the per-pixel term magnitudes of
// pixel_backward (sums of magnitudes before any cancellation) times the
// pixel's transmittance condition number kappa, chained with absolute
// Jacobians: the scale of FP32 rounding, used as a tolerance floor;
// aref_plain (may be NULL) is the same without kappa. slack =
// sum over pixels of the per-element maximum |branch - primary| over every
// decision path of the pixel, plus the FP32 screen-position bound of
// pixel_backward (absolute Jacobians again).
// Returns the number of unverifiable pixels (more than kMaxEventBits events, or
// a chain of three or more depth ties)
// among those with nonzero upstream gradient: their contributions are included
// on the primary branch and every candidate Gaussian of theirs gets slack 1e30.
int64_t orc_backward(int64_t n, const double* means, const double* scales, const double* quats,
                     const double* opac, const double* colors, const double* pose7, const double* cam,
                     const double* opt, int mode, int64_t npix, const int64_t* pix, int nthreads,
                     const double* gC, const double* gD, const double* gA, double* gflat, double* aref,
                     double* slack, double* g2d_out, double* aref_plain) {
  Scene S;
  scene_from_args(S, n, means, scales, quats, opac, colors, pose7, cam, opt);
  build_scene(S, nthreads);
  const int W = S.cam.W, H = S.cam.H;
  const int64_t P = (int64_t)W * H;
  const int64_t cnt = pix ? npix : P;
  if (nthreads < 1) nthreads = 1;
  std::vector<std::vector<double>> acc(nthreads), aabs(nthreads), aplain(nthreads), aslk(nthreads);
  std::vector<int64_t> unver(nthreads, 0);
  for (int t = 0; t < nthreads; ++t) {
    acc[t].assign(10 * n, 0.0);
    aabs[t].assign(10 * n, 0.0);
    aplain[t].assign(10 * n, 0.0);
    aslk[t].assign(10 * n, 0.0);
  }
  parallel_for(cnt, nthreads, [&](int t, int64_t b, int64_t e) {
    PixResult r, ra;
    std::vector<G2> c1, c2, cm, cpos, maxd;
    for (int64_t i = b; i < e; ++i) {
      const int64_t p = pix ? pix[i] : i;
      const int px = (int)(p % W), py = (int)(p / W);
      const double g3[3] = {gC[p], gC[P + p], gC[2 * P + p]};
      const double gd = gD[p], ga = gA ? gA[p] : 0.0;
      if (g3[0] == 0 && g3[1] == 0 && g3[2] == 0 && gd == 0 && ga == 0) continue;
      composite_pixel(S, px, py, mode == 1, 0, true, r);
      double kappa = 1.0;
      pixel_backward(S, r, g3, gd, ga, c1, &cm, &cpos, &kappa);
      for (size_t q = 0; q < c1.size(); ++q)
        for (int f = 0; f < 10; ++f) {
          acc[t][10 * c1[q].id + f] += c1[q].g[f];
          aabs[t][10 * c1[q].id + f] += kappa * cm[q].g[f];
          aplain[t][10 * c1[q].id + f] += cm[q].g[f];
          aslk[t][10 * c1[q].id + f] += cpos[q].g[f];
        }
      if (r.events == 0) continue;
      // every other decision path of this pixel: per-element max |branch - primary|
      maxd.clear();
      auto merge = [&](int64_t id, const double* d) {
        for (G2& m : maxd)
          if (m.id == id) {
            for (int f = 0; f < 10; ++f) m.g[f] = std::max(m.g[f], std::fabs(d[f]));
            return;
          }
        G2 m{id, {}};
        for (int f = 0; f < 10; ++f) m.g[f] = std::fabs(d[f]);
        maxd.push_back(m);
      };
      int width = r.events;
      uint64_t next = 1;
      bool complete = width <= kMaxEventBits && !r.tie3;
      while (complete) {
        const uint64_t lim = 1ull << width;
        int widest = width;
        for (uint64_t m = next; m < lim; ++m) {
          composite_pixel(S, px, py, mode == 1, m, true, ra);
          widest = std::max(widest, ra.events);
          pixel_backward(S, ra, g3, gd, ga, c2);
          for (const G2& c : c2) {
            double d[10];
            for (int f = 0; f < 10; ++f) d[f] = c.g[f];
            for (const G2& b : c1)
              if (b.id == c.id) {
                for (int f = 0; f < 10; ++f) d[f] -= b.g[f];
                break;
              }
            merge(c.id, d);
          }
          for (const G2& b : c1) {
            bool in2 = false;
            for (const G2& c : c2) in2 = in2 || c.id == b.id;
            if (!in2) merge(b.id, b.g);
          }
        }
        next = lim;
        if (widest <= width) break;
        if (widest > kMaxEventBits) complete = false;
        width = widest;
      }
      if (complete) {
        for (const G2& m : maxd)
          for (int f = 0; f < 10; ++f) aslk[t][10 * m.id + f] += m.g[f];
      } else {
        // too many events to enumerate: exclude every candidate of this pixel
        unver[t]++;
        for (int64_t id : r.cand)
          for (int f = 0; f < 10; ++f) aslk[t][10 * id + f] = 1e30;
      }
    }
  });
  std::vector<double> g2(10 * n, 0.0), ab2(10 * n, 0.0), ap2(10 * n, 0.0), sl2(10 * n, 0.0);
  for (int t = 0; t < nthreads; ++t)
    for (int64_t i = 0; i < 10 * n; ++i) {
      g2[i] += acc[t][i];
      ab2[i] += aabs[t][i];
      ap2[i] += aplain[t][i];
      sl2[i] += aslk[t][i];
    }
  if (g2d_out)
    for (int64_t i = 0; i < 10 * n; ++i) g2d_out[i] = g2[i];
  const int64_t off_s = 3 * n, off_q = 6 * n, off_o = 10 * n, off_c = 11 * n, off_p = 14 * n;
  const int64_t total = 14 * n + 13;
  for (int64_t i = 0; i < total; ++i) {
    gflat[i] = 0;
    if (aref) aref[i] = 0;
    if (aref_plain) aref_plain[i] = 0;
    if (slack) slack[i] = 0;
  }
  for (int64_t k = 0; k < n; ++k) {
    const Proj& g = S.proj[k];
    if (!g.valid) continue;
    double o3[14], p7[7], t6[6];
    chain_3d(S, k, &g2[10 * k], o3, p7, t6);
    auto scatter = [&](double* dst, const double* v3, const double* vp, const double* vt, bool absval,
                       double scale) {
      for (int i = 0; i < 3; ++i) dst[3 * k + i] += scale * (absval ? std::fabs(v3[i]) : v3[i]);
      for (int i = 0; i < 3; ++i) dst[off_s + 3 * k + i] += scale * (absval ? std::fabs(v3[3 + i]) : v3[3 + i]);
      for (int i = 0; i < 4; ++i) dst[off_q + 4 * k + i] += scale * (absval ? std::fabs(v3[6 + i]) : v3[6 + i]);
      dst[off_o + k] += scale * (absval ? std::fabs(v3[10]) : v3[10]);
      for (int i = 0; i < 3; ++i) dst[off_c + 3 * k + i] += scale * (absval ? std::fabs(v3[11 + i]) : v3[11 + i]);
      for (int i = 0; i < 7; ++i) dst[off_p + i] += scale * (absval ? std::fabs(vp[i]) : vp[i]);
      for (int i = 0; i < 6; ++i) dst[off_p + 7 + i] += scale * (absval ? std::fabs(vt[i]) : vt[i]);
    };
    scatter(gflat, o3, p7, t6, false, 1.0);
    if (aref || aref_plain || slack) {
      // absolute-Jacobian propagation, one unit 2D direction at a time
      for (int f = 0; f < 10; ++f) {
        if (ab2[10 * k + f] == 0 && sl2[10 * k + f] == 0) continue;
        double unit[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        unit[f] = 1.0;
        double u3[14], up[7], ut[6];
        chain_3d(S, k, unit, u3, up, ut);
        if (aref) scatter(aref, u3, up, ut, true, ab2[10 * k + f]);
        if (aref_plain) scatter(aref_plain, u3, up, ut, true, ap2[10 * k + f]);
        if (slack) scatter(slack, u3, up, ut, true, sl2[10 * k + f]);
      }
    }
  }
  int64_t nu = 0;
  for (int t = 0; t < nthreads; ++t) nu += unver[t];
  return nu;
}

// Tile lists (O6): for every tile (row-major ids, tile_w x tile_h tiles) the
// valid Gaussians whose tile rectangle contains it, in (z, index) order.
// Call with ids = NULL to get K; counts[n] = tiles per Gaussian; ranges[2*n_tiles].
int orc_tile_lists(int64_t n, const double* means, const double* scales, const double* quats,
                   const double* opac, const double* colors, const double* pose7, const double* cam,
                   const double* opt, int64_t* K_out, int64_t* counts, int64_t* ranges, int32_t* ids,
                   int64_t cap) {
  Scene S;
  scene_from_args(S, n, means, scales, quats, opac, colors, pose7, cam, opt);
  build_scene(S, 1);
  const int ntx = (S.cam.W + S.opt.tw - 1) / S.opt.tw;
  const int nty = (S.cam.H + S.opt.th - 1) / S.opt.th;
  const int64_t nt = (int64_t)ntx * nty;
  std::vector<int64_t> per_tile(nt, 0);
  int64_t K = 0;
  for (int64_t k = 0; k < n; ++k) {
    const Proj& g = S.proj[k];
    int64_t c = 0;
    if (g.valid) c = (int64_t)(g.tx1 - g.tx0 + 1) * (g.ty1 - g.ty0 + 1);
    if (counts) counts[k] = c;
    K += c;
    if (g.valid)
      for (int ty = g.ty0; ty <= g.ty1; ++ty)
        for (int tx = g.tx0; tx <= g.tx1; ++tx) per_tile[(int64_t)ty * ntx + tx]++;
  }
  *K_out = K;
  if (ranges) {
    int64_t s = 0;
    for (int64_t t = 0; t < nt; ++t) {
      ranges[2 * t] = s;
      s += per_tile[t];
      ranges[2 * t + 1] = s;
    }
  }
  if (!ids) return 0;
  if (cap < K) return -1;
  std::vector<int64_t> fill(nt, 0);
  int64_t s = 0;
  for (int64_t t = 0; t < nt; ++t) {
    fill[t] = s;
    s += per_tile[t];
  }
  for (int64_t k : S.order) {
    const Proj& g = S.proj[k];
    for (int ty = g.ty0; ty <= g.ty1; ++ty)
      for (int tx = g.tx0; tx <= g.tx1; ++tx) {
        const int64_t t = (int64_t)ty * ntx + tx;
        ids[fill[t]++] = (int32_t)k;
      }
  }
  return 0;
}

// Mapping loss (Eq. 9 and the L1 part of Eq. 10, weights w_c and w_d):
//   L = w_c mean_{3P} |C - C*| + w_d mean_P |D - D*|,  sign(0) = 0.
int orc_loss_l1(int64_t P, const float* C, const float* D, const float* Ct, const float* Dt, double wc,
                double wd, double* loss, double* gC, double* gD) {
  double lc = 0, ld = 0;
  for (int64_t i = 0; i < 3 * P; ++i) {
    const double r = (double)C[i] - (double)Ct[i];
    lc += std::fabs(r);
    gC[i] = wc * ((r > 0) - (r < 0)) / (3.0 * P);
  }
  for (int64_t i = 0; i < P; ++i) {
    const double r = (double)D[i] - (double)Dt[i];
    ld += std::fabs(r);
    gD[i] = wd * ((r > 0) - (r < 0)) / (double)P;
  }
  *loss = wc * lc / (3.0 * P) + wd * ld / (double)P;
  return 0;
}

// Isotropic regularisation of the scales (Eq. 11):
//   L_reg = (1/N) sum_k |s_k - sbar_k 1|_1, sbar_k = (s_k,x + s_k,y + s_k,z) / 3,
// the mean of Gaussian k's own three scales (the reading of "mean scale" that
// makes the term isotropic). With sign(0) = 0, its gradient is
//   dL/ds_k,j = (1/N) (sign(r_j) - (1/3) sum_i sign(r_i)),  r_i = s_k,i - sbar_k.
// scales: [N,3]; grad: [N,3] (overwritten) or NULL; *loss = L_reg (0 if N = 0).
int orc_loss_reg(int64_t N, const double* scales, double* loss, double* grad) {
  double total = 0.0;
  for (int64_t k = 0; k < N; ++k) {
    const double* s = scales + 3 * k;
    const double sbar = (s[0] + s[1] + s[2]) / 3.0;
    double sg[3], sgsum = 0.0;
    for (int i = 0; i < 3; ++i) {
      const double r = s[i] - sbar;
      total += std::fabs(r);
      sg[i] = (double)((r > 0) - (r < 0));
      sgsum += sg[i];
    }
    if (grad)
      for (int j = 0; j < 3; ++j) grad[3 * k + j] = (sg[j] - sgsum / 3.0) / (double)N;
  }
  *loss = N > 0 ? total / (double)N : 0.0;
  return 0;
}

// Tracking loss (Eq. 15 with the supplement's masks):
//   valid = observed depth > 0; e = |D - D*|; m = lower median of e over valid
//   pixels; inlier = valid and e <= inlier_mult * m; w = inlier * alpha^3
//   (detached); L = sum_p w (lambda_c sum_ch |C - C*| + (1 - lambda_c) |D - D*|).
// The discrete decisions (median element, inlier test) are taken in binary32,
// the precision the rendered inputs carry; everything else is FP64.
int orc_loss_track(int64_t P, const float* C, const float* D, const float* A, const float* Ct,
                   const float* Dt, double lambda_c, float inlier_mult, double* loss, double* gC,
                   double* gD, float* median_out, int64_t* n_inlier) {
  std::vector<float> ev;
  ev.reserve(P);
  for (int64_t i = 0; i < P; ++i)
    if (Dt[i] > 0.0f) ev.push_back(std::fabs(D[i] - Dt[i]));
  float med = 0.0f;
  const bool any = !ev.empty();
  if (any) {
    std::sort(ev.begin(), ev.end());
    med = ev[(ev.size() - 1) / 2];
  }
  const float thr = inlier_mult * med;
  double L = 0;
  int64_t ni = 0;
  for (int64_t i = 0; i < P; ++i) {
    const bool valid = Dt[i] > 0.0f;
    const float e32 = std::fabs(D[i] - Dt[i]);
    const bool inl = any && valid && (e32 <= thr);
    const double a = A[i];
    const double w = inl ? a * a * a : 0.0;
    ni += inl ? 1 : 0;
    double lc = 0;
    for (int ch = 0; ch < 3; ++ch) {
      const double r = (double)C[ch * P + i] - (double)Ct[ch * P + i];
      lc += std::fabs(r);
      gC[ch * P + i] = w * lambda_c * ((r > 0) - (r < 0));
    }
    const double rd = (double)D[i] - (double)Dt[i];
    gD[i] = w * (1.0 - lambda_c) * ((rd > 0) - (rd < 0));
    L += w * (lambda_c * lc + (1.0 - lambda_c) * std::fabs(rd));
  }
  *loss = L;
  *median_out = med;
  *n_inlier = ni;
  return 0;
}

// One bias-corrected Adam step (Kingma & Ba 2015) on n parameters; step >= 1.
int orc_adam(int64_t n, double* param, double* m, double* v, const double* g, int64_t step, double lr,
             double b1, double b2, double eps) {
  const double c1 = 1.0 - std::pow(b1, (double)step);
  const double c2 = 1.0 - std::pow(b2, (double)step);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    const double mh = m[i] / c1, vh = v[i] / c2;
    param[i] -= lr * mh / (std::sqrt(vh) + eps);
  }
  return 0;
}

// Left perturbation exp(xi^) T of pose7 by the twist xi = (rho, phi):
// R' = Exp(phi) R (Rodrigues' formula), t' = Exp(phi) t + rho. The output
// quaternion is R' as a unit quaternion with w >= 0 (Shepperd's method).
int orc_pose_apply_twist(const double* p7, const double* xi, double* out) {
  const Pose P = read_pose(p7);
  const double th = std::sqrt(xi[3] * xi[3] + xi[4] * xi[4] + xi[5] * xi[5]);
  double K[9] = {0, -xi[5], xi[4], xi[5], 0, -xi[3], -xi[4], xi[3], 0};
  double E[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  if (th > 0) {
    double K2[9];
    mm3(K, K, K2);
    const double a = std::sin(th) / th, b = (1 - std::cos(th)) / (th * th);
    for (int i = 0; i < 9; ++i) E[i] += a * K[i] + b * K2[i];
  }
  double R[9];
  mm3(E, P.R, R);
  for (int i = 0; i < 3; ++i) out[4 + i] = E[3 * i] * P.t[0] + E[3 * i + 1] * P.t[1] + E[3 * i + 2] * P.t[2] + xi[i];
  const double tr = R[0] + R[4] + R[8];
  double q[4];
  if (tr > 0) {
    const double s = std::sqrt(tr + 1.0) * 2;
    q[0] = 0.25 * s; q[1] = (R[7] - R[5]) / s; q[2] = (R[2] - R[6]) / s; q[3] = (R[3] - R[1]) / s;
  } else if (R[0] > R[4] && R[0] > R[8]) {
    const double s = std::sqrt(1.0 + R[0] - R[4] - R[8]) * 2;
    q[0] = (R[7] - R[5]) / s; q[1] = 0.25 * s; q[2] = (R[1] + R[3]) / s; q[3] = (R[2] + R[6]) / s;
  } else if (R[4] > R[8]) {
    const double s = std::sqrt(1.0 + R[4] - R[0] - R[8]) * 2;
    q[0] = (R[2] - R[6]) / s; q[1] = (R[1] + R[3]) / s; q[2] = 0.25 * s; q[3] = (R[5] + R[7]) / s;
  } else {
    const double s = std::sqrt(1.0 + R[8] - R[0] - R[4]) * 2;
    q[0] = (R[3] - R[1]) / s; q[1] = (R[2] + R[6]) / s; q[2] = (R[5] + R[7]) / s; q[3] = 0.25 * s;
  }
  const double sg = q[0] < 0 ? -1.0 : 1.0;
  const double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int i = 0; i < 4; ++i) out[i] = sg * q[i] / n;
  return 0;
}

// Constant-speed pose initialisation (Eq. 13) applied to pose7 = (q, t):
// t = t1 + (t1 - t0); q = normalise(q1 + (q1 - q0')) where q0' is q0 or -q0,
// whichever lies in q1's hemisphere (q and -q are the same rotation).
int orc_pose_const_velocity(const double* p0, const double* p1, double* out) {
  double d = 0;
  for (int i = 0; i < 4; ++i) d += p0[i] * p1[i];
  const double s = d < 0 ? -1.0 : 1.0;
  double q[4], n = 0;
  for (int i = 0; i < 4; ++i) {
    q[i] = p1[i] + (p1[i] - s * p0[i]);
    n += q[i] * q[i];
  }
  n = std::sqrt(n);
  for (int i = 0; i < 4; ++i) out[i] = n > 0 ? q[i] / n : p1[i];
  for (int i = 0; i < 3; ++i) out[4 + i] = p1[4 + i] + (p1[4 + i] - p0[4 + i]);
  return 0;
}

}  // extern "C"
