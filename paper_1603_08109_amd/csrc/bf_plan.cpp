// Host-side planning and the single-image entry points of the C ABI.
//
// Planning follows Sec. 2-3 of the paper:
//   * support W: given (box) or ceil(3 sigma_s) (Gaussian, Sec. 1);
//   * w(0) of the kernel normalised to sum 1 over Omega (Prop. accuracy);
//   * eps = w(0) delta / (2T + delta)                         (Cor. eps);
//   * N = ceil(q / W0(q e^{-p})), p = 1 + log lambda, q = -lambda - log eps,
//     lambda = T^2 / sigma_r^2                                 (Prop. LambW),
//     or Algorithm 1 as printed, or the exact Poisson tail of Prop. upperBound.
// The float64 tables of the range-safe recursion (see gpa_tables) are built
// here and uploaded once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "bf_internal.h"

namespace bfgpa {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// Principal branch of the Lambert W function on [-1/e, inf): the inverse of
// w -> w e^w, by Halley iterations from a branch-point / asymptotic start.
double lambert_w0(double z) {
  const double em1 = 1.0 / M_E;
  if (!(z >= -em1)) return std::numeric_limits<double>::quiet_NaN();
  if (z == 0.0) return 0.0;
  double w;
  if (z < -0.25) {
    double p = std::sqrt(2.0 * (M_E * z + 1.0));
    w = -1.0 + p - p * p / 3.0 + 11.0 / 72.0 * p * p * p;
  } else if (z < 3.0) {
    w = std::log1p(z) * (1.0 - 0.25 * std::log1p(z) / (1.0 + std::log1p(z)));
  } else {
    double l1 = std::log(z), l2 = std::log(l1);
    w = l1 - l2 + l2 / l1;
  }
  for (int it = 0; it < 64; ++it) {
    double ew = std::exp(w);
    double f = w * ew - z;
    double wp1 = w + 1.0;
    if (wp1 == 0.0) break;
    double den = ew * wp1 - (w + 2.0) * f / (2.0 * wp1);
    double dw = f / den;
    w -= dw;
    if (std::fabs(dw) <= 1e-15 * (1.0 + std::fabs(w))) break;
  }
  return w;
}

// sum_{n >= N} e^{-lam} lam^n / n!  (Prop. upperBound).  Summed directly
// from the tail side when N > lam (terms then decrease), else as one minus
// the head (the tail is then at least about one half, so no cancellation).
double poisson_tail(int N, double lam) {
  if (N <= 0) return 1.0;
  if (lam <= 0.0) return 0.0;
  auto logpmf = [lam](double n) { return -lam + n * std::log(lam) - std::lgamma(n + 1.0); };
  if ((double)N > lam) {
    double s = 0.0;
    for (int n = N; n < N + 100000; ++n) {
      double t = std::exp(logpmf(n));
      s += t;
      if (t <= 1e-18 * s || (t == 0.0 && n > lam)) break;
    }
    return s;
  }
  double head = 0.0;
  for (int n = 0; n < N; ++n) head += std::exp(logpmf(n));
  return std::max(0.0, 1.0 - head);
}

// p = 1 + log lambda and q = -lambda - log eps of Prop. (LambW).
struct ChernoffPQ {
  double p, q;
};
static ChernoffPQ chernoff_pq(double lam, double eps) { return {1.0 + std::log(lam), -lam - std::log(eps)}; }

// theta = q / W0(q e^{-p}), the root above lambda of nu(x) = x log x - p x - q
// (Prop. LambW); the order is its ceiling.
static int chernoff_order(double lam, double eps) {
  const ChernoffPQ c = chernoff_pq(lam, eps);
  return (int)std::ceil(c.q / lambert_w0(c.q * std::exp(-c.p)) - 1e-12);
}

// The four-term Lambert-W series of eq. (series), W0(t) ~ t - t^2 + 3t^3/2 - 8t^4/3.
static double lambert_w0_series(double t) { return t * (1.0 - t * (1.0 - t * (1.5 - t * (8.0 / 3.0)))); }

// One Newton step on nu(x) = x log x - p x - q, eq. (Newton_method).
static double nu_newton_step(double x, const ChernoffPQ& c) {
  return x - (x * std::log(x) - c.p * x - c.q) / (std::log(x) + 1.0 - c.p);
}

// The order rule of Algorithm 1: the root of Prop. (LambW) with W0 taken from
// the series (note q e^{-p} = q / (e lambda)), refined by three Newton steps
// when sigma_r < 30, and the fixed order 10 for sigma_r >= 70 (which carries
// no guarantee).  Returns -1 when the series gives no finite root.
static int alg1_order(double sigma_r, double eps, double T) {
  if (sigma_r >= 70.0) return 10;
  const double lam = (T / sigma_r) * (T / sigma_r);
  const ChernoffPQ c = chernoff_pq(lam, eps);
  double x = c.q / lambert_w0_series(c.q / (M_E * lam));
  const int newton_steps = sigma_r < 30.0 ? 3 : 0;
  for (int k = 0; k < newton_steps; ++k) x = nu_newton_step(x, c);
  if (!std::isfinite(x)) return -1;
  return (int)std::ceil(x - 1e-12);
}

static int poisson_order(double lam, double eps) {
  int N = 1;
  while (poisson_tail(N, lam) > eps && N < 1000000) ++N;
  return N;
}

// 1-D kernel factor w1(a), a = -W..W, unnormalised.
std::vector<double> taps1d(int kind, double sigma_s, int W) {
  std::vector<double> t(2 * W + 1);
  for (int a = -W; a <= W; ++a)
    t[a + W] = (kind == BF_BOX) ? 1.0 : std::exp(-(double)a * a / (2.0 * sigma_s * sigma_s));
  return t;
}

// Fill defaults and check ranges.  Returns BF_OK or a negative code.
static int normalise(const bf_params* in, bf_params* p) {
  if (!in) return fail(BF_EINVAL, "params is NULL");
  *p = *in;
  if (p->kernel != BF_BOX && p->kernel != BF_GAUSS && p->kernel != BF_GAUSS_REC)
    return fail(BF_EINVAL, "kernel must be BF_BOX, BF_GAUSS or BF_GAUSS_REC");
  constexpr int kKnownFlags = BF_FLAG_FP32_ACCUM | BF_FLAG_GRAD | BF_FLAG_STREAMED | BF_FLAG_JOINT |
                              BF_FLAG_MIRROR | BF_FLAG_TILE_VALU | BF_FLAG_MFMA_FP32;
  if (p->flags & ~kKnownFlags) return fail(BF_EINVAL, "unknown flag bits");
  if (p->kernel == BF_GAUSS) {
    if (!(p->sigma_s > 0.0) || !std::isfinite(p->sigma_s)) return fail(BF_EINVAL, "sigma_s must be > 0");
    if (p->W <= 0) p->W = (int)std::ceil(3.0 * p->sigma_s - 1e-12);
  }
  if (p->kernel == BF_GAUSS_REC) {
    // the fit's recursions stay well conditioned in float32 over this range
    if (!(p->sigma_s >= 0.5 && p->sigma_s <= 100.0)) return fail(BF_EINVAL, "recursive Gaussian: sigma_s in [0.5, 100]");
    p->W = 0;  // unbounded support
  }
  if (p->W < 0) return fail(BF_EINVAL, "W must be >= 0");
  if (!(p->sigma_r > 0.0) || !std::isfinite(p->sigma_r)) return fail(BF_EINVAL, "sigma_r must be > 0");
  if (p->T == 0.0) p->T = 127.5;
  if (!(p->T > 0.0) || !std::isfinite(p->T)) return fail(BF_EINVAL, "T must be > 0");
  if (std::isnan(p->center)) p->center = p->T;
  if (p->delta == 0.0) p->delta = 1e-3;
  if (!(p->delta > 0.0)) return fail(BF_EINVAL, "delta must be > 0");
  if (p->N < 0) return fail(BF_EINVAL, "N must be >= 0");
  if (p->n_rule < BF_NRULE_LAMBERTW || p->n_rule > BF_NRULE_POISSON) return fail(BF_EINVAL, "unknown n_rule");
  if (p->height < 0 || p->width < 0) return fail(BF_EINVAL, "height/width must be >= 0");
  return BF_OK;
}

// Order and bounds for normalised parameters.
// dims: 2 for images, 3 for volumes (the centre weight of w1 x w1 x w1).
static int plan_order(const bf_params* p, bf_plan_info* info, int dims = 2) {
  std::memset(info, 0, sizeof(*info));
  std::vector<double> t = taps1d(p->kernel, p->sigma_s, p->W);
  double s = 0.0;
  for (double v : t) s += v;
  info->W = p->W;
  info->w0 = p->kernel == BF_GAUSS_REC ? rg_w0(p->sigma_s) : std::pow(t[p->W] / s, (double)dims);
  info->eps = info->w0 * p->delta / (2.0 * p->T + p->delta);
  info->lambda = (p->T / p->sigma_r) * (p->T / p->sigma_r);
  // exp(-x^2/2) must stay a normal float64 for |x| <= T/sigma_r (float32 up to
  // lambda = 170; beyond, only the wide-range streamed Gaussian runs)
  if (info->lambda > kLambdaF64)
    return fail(BF_EUNSUPPORTED, "sigma_r too small: need T/sigma_r <= 37 (exp(-x^2/2) underflows float64)");
  int need = chernoff_order(info->lambda, info->eps);
  int status = BF_OK;
  int N;
  if (p->N > 0) {
    N = p->N;
    if (N < need) status = BF_WNOGUARANTEE;
  } else if (p->n_rule == BF_NRULE_ALG1) {
    N = alg1_order(p->sigma_r, info->eps, p->T);
    if (N <= 0) return fail(BF_EUNSUPPORTED, "Algorithm 1 series gives a non-positive order at this eps");
    if (p->sigma_r >= 70.0 || poisson_tail(N, info->lambda) > info->eps) status = BF_WNOGUARANTEE;
  } else if (p->n_rule == BF_NRULE_POISSON) {
    N = poisson_order(info->lambda, info->eps);
  } else {
    N = need;
  }
  if (N < 1) N = 1;
  if (N > 4096) return fail(BF_EUNSUPPORTED, "order N above 4096");
  info->N = N;
  info->kernel_bound = poisson_tail(N, info->lambda);
  info->guaranteed_delta = (info->kernel_bound < info->w0)
      ? 2.0 * p->T * info->kernel_bound / (info->w0 - info->kernel_bound)
      : std::numeric_limits<double>::infinity();
  if (p->kernel == BF_GAUSS_REC) {
    // Prop. (accuracy) assumes w >= 0; the recursive fit has small negative
    // lobes, so N is chosen by the same rule but no +-delta bound is claimed
    info->guaranteed_delta = std::numeric_limits<double>::infinity();
    status = BF_WNOGUARANTEE;
    set_error("recursive Gaussian: the kernel has negative lobes, Prop. (accuracy) gives no +-delta bound");
    return status;
  }
  if (status == BF_WNOGUARANTEE) set_error("order below the bound: no +-delta guarantee");
  return status;
}

// Tables of the range-safe form of Algorithm 2 (float64, stored float32).
// With X = T / sigma_r, M_n = max_{|x| <= X} e^{-x^2/2} |x|^n, i.e.
// (n/e)^{n/2} for n <= X^2 and e^{-X^2/2} X^n beyond; r_n = M_n / M_{n-1}.
// The kernels keep F~_n = F_n / M_n (|F~_n| <= 1) and the coefficient
// a_n = e^{-x_i^2/2} x_i^n M_n / n! (|a_n| <= 1); their products equal the
// terms of eqs. (P), (Q) times e^{-x_i^2/2}, which cancels in P/Q.
void gpa_tables(double lam, int N, std::vector<double>& s, std::vector<double>& r,
                std::vector<double>& inv) {
  const double X = std::sqrt(lam);
  auto logM = [&](int n) -> double {
    if (n == 0) return 0.0;
    if ((double)n <= lam) return 0.5 * n * (std::log((double)n) - 1.0);
    return -0.5 * lam + n * std::log(X);
  };
  s.assign(N + 2, 0.0);
  r.assign(N + 2, 0.0);
  inv.assign(N + 2, 0.0);
  for (int n = 1; n <= N + 1; ++n) {
    r[n] = std::exp(logM(n) - logM(n - 1));
    s[n] = 1.0 / r[n];
    inv[n] = 1.0 / n;
  }
}

// Deriche's fit of the sampled Gaussian exp(-x^2/2), x = n / sigma_s, by two
// damped oscillations (a, a', b, omega):
// h(n) = sum_j (a_j cos(omega_j x) + a'_j sin(omega_j x)) e^{-b_j x}, x = |n| / sigma_s.
static const double kDericheFit[2][4] = {{1.680, 3.735, 1.783, 0.6318}, {-0.6803, -0.2598, 1.723, 1.997}};

// Normalised centre weight (h(0) / sum_n h(|n|))^2 of the 2-D kernel; with
// q = rho e^{i theta} per oscillation, sum_{m >= 1} h_j(m) = Re[(a - i a') q / (1 - q)].
double rg_w0(double sigma_s) {
  double h0 = 0.0, tail = 0.0;
  for (const auto& f : kDericheFit) {
    const std::complex<double> q = std::polar(std::exp(-f[2] / sigma_s), f[3] / sigma_s);
    h0 += f[0];
    tail += std::real(std::complex<double>(f[0], -f[1]) * q / (1.0 - q));
  }
  const double S = h0 + 2.0 * tail;
  return (h0 / S) * (h0 / S);
}

// Per oscillation, the pole q = rho e^{i theta}, rho = e^{-b/sigma_s},
// theta = omega/sigma_s: h_j(n) = Re[(a - i a') q^n], so the causal part is
// Re[(a - i a') w] with w[i] = q w[i-1] + x[i] and the anticausal part the
// same with w'[i] = q (w'[i+1] + x[i+1]).  The scans over chunks of 16 or 8
// samples move states by q^16 or q^8 per chunk: the table holds q^(8 m),
// m = 1 .. 128.
void rg_table(double sigma_s, float* out) {
  for (int j = 0; j < 2; ++j) {
    const std::complex<double> q = std::polar(std::exp(-kDericheFit[j][2] / sigma_s), kDericheFit[j][3] / sigma_s);
    out[8 * j + 0] = (float)kDericheFit[j][0];
    out[8 * j + 1] = (float)kDericheFit[j][1];
    out[8 * j + 2] = (float)q.real();
    out[8 * j + 3] = (float)q.imag();
    std::complex<double> q8 = q;
    for (int i = 0; i < 3; ++i) q8 *= q8;  // q^8
    std::complex<double> z = q8;
    for (int m = 1; m <= kRgPow; ++m) {
      out[16 + 2 * (kRgPow * j + m - 1)] = (float)z.real();
      out[17 + 2 * (kRgPow * j + m - 1)] = (float)z.imag();
      z *= q8;
    }
  }
}

// Device constant tables of one image, as one float array: s_n, r_n, 1/n
// (n = 0 .. N+1, rows of *stride floats); 1/sqrt(n) and sqrt(n) as float64
// (two rows of *stride doubles, the wide-range path); the taps and the d^2
// taps (kTapPad zeros on each side, rows of *ntapr floats); the recursive-
// Gaussian table.  Every offset is even, so the doubles stay aligned.
std::vector<float> const_tables(const bf_params& p, const bf_plan_info& info, int64_t* stride,
                                int64_t* ntapr) {
  std::vector<double> s, r, inv;
  // the range-safe tables serve lambda <= 170 (the wide-range path reads none of them)
  gpa_tables(std::min(info.lambda, kLambdaF32), info.N, s, r, inv);
  const int N = info.N, W = p.W;
  *stride = ((N + 2 + 63) / 64) * 64;
  *ntapr = ((2 * W + 1 + 2 * kTapPad + 63) / 64) * 64;
  const int64_t nrg = p.kernel == BF_GAUSS_REC ? kRgTabFloats : 0;
  const int64_t taps0 = 7 * *stride;
  std::vector<float> h(taps0 + 2 * *ntapr + nrg, 0.0f);
  if (nrg) rg_table(p.sigma_s, h.data() + taps0 + 2 * *ntapr);
  std::vector<double> isq(*stride, 0.0), sq(*stride, 0.0);
  for (int n = 0; n <= N + 1; ++n) {
    h[n] = (float)s[n];
    h[*stride + n] = (float)r[n];
    h[2 * *stride + n] = (float)inv[n];
    sq[n] = std::sqrt((double)n);
    isq[n] = n > 0 ? 1.0 / sq[n] : 0.0;
  }
  std::memcpy(h.data() + 3 * *stride, isq.data(), *stride * sizeof(double));
  std::memcpy(h.data() + 5 * *stride, sq.data(), *stride * sizeof(double));
  std::vector<double> t = taps1d(p.kernel, p.sigma_s, W);
  for (int a = -W; a <= W; ++a) {
    h[taps0 + kTapPad + a + W] = (float)t[a + W];
    h[taps0 + *ntapr + kTapPad + a + W] = (float)((double)a * a * t[a + W]);
  }
  return h;
}

void bind_tables(TileParams& tp, const float* d, int64_t stride, int64_t ntapr) {
  tp.s_tab = d;
  tp.r_tab = d + stride;
  tp.inv_tab = d + 2 * stride;
  tp.isq = (const double*)(d + 3 * stride);
  tp.sq = (const double*)(d + 5 * stride);
  tp.taps = d + 7 * stride;
  tp.taps2 = d + 7 * stride + ntapr;
}

// Rough per-output cost of a tile shape (VALU instructions per order n),
// scaled up when the register footprint limits waves per SIMD.
static double tile_cost(int kernel, int W, int opt, int mreg) {
  const int TY = 4 * opt;
  const double area = (double)TY * kTileCols;
  const double L = 2.0 * W + 1.0;
  const double rows = (double)(TY + 2 * W);
  const double npx = (double)region_floats(TY, W);
  double row, col;
  if (kernel == BF_BOX) {
    row = rows * kTileCols * (2.0 + L / kRowSegBoxHost);
    col = area * (2.0 + L / opt);
  } else {
    row = rows * kTileCols * (L + 4.0);
    col = area * (L + 4.0);
  }
  const double upd = 2.0 * npx;
  const double acc = 5.0 * area;
  const double regs = 2.0 * mreg + 9.0 * opt + 40.0;
  const double occ = regs <= 128 ? 1.0 : regs <= 168 ? 1.1 : regs <= 256 ? 1.3 : 1.8;
  return (row + col + upd + acc) / area * occ;
}

// Same units for the streamed path: rows staged 256 wide, exact column pass,
// plus about 20 bytes of device-memory traffic per pixel and order (~100
// instruction slots at the chip's VALU : HBM balance).
static double streamed_cost(int kernel, int W) {
  const double L = 2.0 * W + 1.0;
  if (kernel == BF_BOX) return (256.0 + 2 * W) / 256.0 * (2.0 + L / 16.0) + 2.0 + 5.0 + 100.0;
  return (256.0 + 2 * W) / 256.0 * (L + 4.0) + (L + 4.0) + 5.0 + 100.0;
}

static int choose_forward_tile(int kernel, int W, int H, int Wd, int N, bool allow_streamed, int* variant,
                               int* TY, double* cost = nullptr) {
  const int nv = forward_variant_count();
  int best = -1;
  double bestc = 0.0;
  for (int v = 0; v < nv; ++v) {
    Variant vv = forward_variant(v);
    const int ty = 4 * vv.opt;
    if (region_floats(ty, W) > (int64_t)kThreads * vv.mreg) continue;
    if (forward_lds_bytes(ty, W) > max_lds_bytes()) continue;
    double c = tile_cost(kernel, W, vv.opt, vv.mreg);
    // small images: prefer shapes that give every CU at least one tile
    const int64_t tiles = (int64_t)((H + ty - 1) / ty) * ((Wd + kTileCols - 1) / kTileCols);
    if (tiles < 256) c *= 1.0 + (256.0 - tiles) / 256.0;
    if (best < 0 || c < bestc) {
      best = v;
      bestc = c;
    }
  }
  if (best < 0) return fail(BF_EUNSUPPORTED, "support W too large for the fused tile kernels");
  // The streamed engines pay a fixed cost per call and per block of orders
  // (the lift, the final ratio, launch ramps, the box strips' warm-up rows)
  // for a lower cost per order at wide supports, so the crossover falls with
  // the order N.  Measured on 4096^2 (ms, fused / streamed, sigma_r = 10 / 30
  // / 50, N = 250 / 50 / 30): box W = 13 5.11 / 4.44, 1.15 / 1.28; W = 16
  // 5.25 / 4.52, 1.17 / 1.30, 0.72 / 0.76; W = 20 8.38 / 4.71, 1.84 / 1.35,
  // 1.11 / 0.79.  Gaussian W = 14 11.5 / 13.0, 2.46 / 3.00; W = 15 13.6 /
  // 13.1, 2.90 / 3.00, 1.71 / 1.90; W = 16 13.1 / 13.1, 2.84 / 3.00; W = 18
  // 18.6 / 13.4, 3.93 / 3.04, 2.31 / 1.92.  Box strips therefore from W = 18,
  // and from W = 13 with 150 orders or more, on images of 2^20 pixels and
  // more; the Gaussian from W = 17, and from W = 15 with 150 orders or more,
  // on images of 2^22 pixels and more (64 orders per block).  Below 2^22
  // pixels (16 orders per block) the Gaussian's split passes win from about
  // W = 14 at every size measured, 64 x 64 to 2048^2 (on 256 images of
  // 64..1024 x 64..768 with sigma_s in [2, 15]: 166.6 ms fused, 75.7 ms taking
  // the faster engine per image, 76.1 ms from W = 16 on); W = 15 on 512^2 is
  // still faster fused (0.21 vs 0.23 ms), hence W >= 16.
  const int64_t npx = (int64_t)H * Wd;
  if (allow_streamed && ls_supported(W)) {
    const bool gauss_wide = npx >= (1 << 22) ? (W >= 17 || (W >= 15 && N >= 150))
                                             : (W >= 16 || (npx >= (1 << 20) && bestc > streamed_cost(kernel, W)));
    const bool box_wide = npx >= (1 << 20) && ls_box_strip_supported(W) && (W >= 18 || (W >= 13 && N >= 150));
    if (kernel == BF_BOX ? box_wide : gauss_wide) return fail(BF_EUNSUPPORTED, "streamed path is cheaper at this support");
  }
  *variant = best;
  *TY = 4 * forward_variant(best).opt;
  if (cost) *cost = bestc;
  return BF_OK;
}

// Cross filter: the fused tile variants with room for two region images.
static int choose_joint_tile(int kernel, int W, int H, int Wd, int* variant, int* TY) {
  int best = -1;
  double bestc = 0.0;
  for (int v = 0; v < joint_variant_count(); ++v) {
    const Variant vv = joint_variant(v);
    const int ty = 4 * vv.opt;
    if (region_floats(ty, W) > (int64_t)kThreads * vv.mreg) continue;
    if (joint_lds_bytes(ty, W) > max_lds_bytes()) continue;
    double c = tile_cost(kernel, W, vv.opt, vv.mreg);
    const int64_t tiles = (int64_t)((H + ty - 1) / ty) * ((Wd + kTileCols - 1) / kTileCols);
    if (tiles < 256) c *= 1.0 + (256.0 - tiles) / 256.0;
    if (best < 0 || c < bestc) {
      best = v;
      bestc = c;
    }
  }
  if (best < 0) return fail(BF_EUNSUPPORTED, "support W too large for the cross-filter tiles");
  *variant = best;
  *TY = 4 * joint_variant(best).opt;
  return BF_OK;
}

// The forward engine of a plan: the fused VALU tile (variant, TY), the
// fused matrix-core tile (Gaussian only), or the streamed sequence.
struct ForwardPath {
  int engine;   // BF_PATH_*
  int variant;  // VALU tile variant, or -1
  int TY;       // tile rows (0 on the streamed path)
};

// N: the order the plan takes (the engines' crossover depends on it).
static int choose_forward_path(const bf_params& p, int N, ForwardPath* fp) {
  if ((p.flags & BF_FLAG_STREAMED) && (p.flags & BF_FLAG_TILE_VALU))
    return fail(BF_EINVAL, "at most one of the STREAMED / TILE_VALU flags");
  const bool mirror = (p.flags & BF_FLAG_MIRROR) != 0;
  fp->variant = -1;
  fp->TY = 0;
  if ((p.T / p.sigma_r) * (p.T / p.sigma_r) > kLambdaF32) {
    // float32 exp(-x^2/2) underflows: the streamed Gaussian with float64 states
    if (p.kernel != BF_GAUSS ||
        (p.flags & (BF_FLAG_JOINT | BF_FLAG_GRAD | BF_FLAG_TILE_VALU | BF_FLAG_MFMA_FP32)))
      return fail(BF_EUNSUPPORTED,
                  "sigma_r too small for float32: T/sigma_r above 13 runs only the plain forward Gaussian "
                  "(no adjoint or cross filter, split-bfloat16 streamed passes)");
    if (!ls_wide_supported(p.W)) return fail(BF_EUNSUPPORTED, "T/sigma_r above 13: Gaussian W <= 120");
    fp->engine = BF_PATH_WIDE;
    return BF_OK;
  }
  if (p.kernel == BF_GAUSS_REC) {
    if (p.flags & (BF_FLAG_JOINT | BF_FLAG_MIRROR | BF_FLAG_TILE_VALU))
      return fail(BF_EUNSUPPORTED, "the recursive Gaussian runs the plain filter, zero border, own engine");
    if (p.height > 0 && p.width > 0 && !rg_supported(p.height, p.width))
      return fail(BF_EUNSUPPORTED, "recursive Gaussian: width and height <= 8192");
    fp->engine = BF_PATH_RECURSIVE;
    return BF_OK;
  }
  if (p.flags & BF_FLAG_JOINT) {
    if (p.flags & (BF_FLAG_GRAD | BF_FLAG_STREAMED))
      return fail(BF_EUNSUPPORTED, "the cross filter has no adjoint or streamed path");
    fp->engine = BF_PATH_TILE;
    return choose_joint_tile(p.kernel, p.W, p.height, p.width, &fp->variant, &fp->TY);
  }
  if (p.flags & BF_FLAG_TILE_VALU) {
    fp->engine = BF_PATH_TILE;
    return choose_forward_tile(p.kernel, p.W, p.height, p.width, N, false, &fp->variant, &fp->TY);
  }
  if (!(p.flags & BF_FLAG_STREAMED)) {
    double c = 0.0;
    if (choose_forward_tile(p.kernel, p.W, p.height, p.width, N, true, &fp->variant, &fp->TY, &c) == BF_OK) {
      fp->engine = BF_PATH_TILE;
      return BF_OK;
    }
  }
  if (!ls_supported(p.W)) return fail(BF_EUNSUPPORTED, "support W too large");
  if (mirror && !ls_mirror_supported(p.kernel, p.W))
    return fail(BF_EUNSUPPORTED, "support W too large for the mirror border");
  fp->engine = BF_PATH_STREAMED;
  fp->variant = -1;
  fp->TY = 0;
  return BF_OK;
}

static int choose_backward_tile(int W, bool sigs, int* variant, int* TY) {
  const int nv = backward_variant_count();
  for (int v = 0; v < nv; ++v) {
    Variant vv = backward_variant(v);
    const int ty = 4 * vv.opt;
    if (region_floats_bwd(ty, W) > (int64_t)kThreads * vv.mreg) continue;
    if (backward_lds_bytes(ty, W, sigs) + 2 * kThreads * 8 > max_lds_bytes()) continue;
    *variant = v;
    *TY = ty;
    return BF_OK;
  }
  return fail(BF_EUNSUPPORTED, "support W too large for the adjoint tile kernels");
}

static int hip_fail(hipError_t e, const char* what) {
  return fail(BF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace bfgpa

using namespace bfgpa;

extern "C" {

const char* bf_version(void) { return "bf_gpa 0.1 (gfx950)"; }

const char* bf_status_string(int status) {
  switch (status) {
    case BF_OK: return "ok";
    case BF_EINVAL: return "invalid argument";
    case BF_ENOMEM: return "out of memory";
    case BF_EHIP: return "HIP runtime error";
    case BF_EUNSUPPORTED: return "unsupported";
    case BF_WNOGUARANTEE: return "warning: order below the accuracy guarantee";
    default: return "unknown status";
  }
}

const char* bf_last_error_message(void) { return g_err.c_str(); }

int bf_order(const bf_params* in, bf_plan_info* out) {
  if (!out) return fail(BF_EINVAL, "info is NULL");
  bf_params p;
  int st = normalise(in, &p);
  if (st < 0) return st;
  st = plan_order(&p, out);
  if (st < 0) return st;
  // the engine needs the image size, except that lambda above 170 admits one engine whatever the size
  if ((p.height > 0 && p.width > 0) || out->lambda > kLambdaF32) {
    ForwardPath fp;
    const int pst = choose_forward_path(p, out->N, &fp);
    if (pst < 0) return pst;
    out->path = fp.engine;
    out->tile_rows = fp.TY;
    out->tile_cols = (fp.engine == BF_PATH_STREAMED || fp.engine == BF_PATH_RECURSIVE || fp.engine == BF_PATH_WIDE) ? 0
                                                                                                                : kTileCols;
  }
  return st;
}

// Reflecting border with BF_FLAG_GRAD: the forward plan of the image (reflecting border, no
// adjoint workspace of its own) holds a zero-border adjoint plan of the image extended by W on
// each side, plus the three extended planes bf_backward pads into and folds back from.
static int plan_mirror_adjoint(const bf_params& p, bf_plan_t** out) {
  bf_params q = p;
  q.flags &= ~BF_FLAG_GRAD;
  bf_plan_t* pl = nullptr;
  const int wst = bf_plan(&q, &pl);
  if (wst < 0) return wst;
  bf_params r = p;
  r.flags &= ~BF_FLAG_MIRROR;
  r.height = p.height + 2 * p.W;
  r.width = p.width + 2 * p.W;
  bf_plan_t* adj = nullptr;
  int st = bf_plan(&r, &adj);
  if (st < 0) {
    const std::string msg = g_err;
    bf_destroy(pl);
    return fail(st, "reflecting-border adjoint: " + msg);
  }
  if (adj->info.N != pl->info.N || adj->info.W != pl->info.W) {
    bf_destroy(adj);
    bf_destroy(pl);
    return fail(BF_EINVAL, "reflecting-border adjoint: order or support differs on the extended image");
  }
  const int64_t plane = (((int64_t)r.height * r.width + 63) / 64) * 64;  // 256-byte aligned planes
  hipError_t e = hipMalloc(&pl->d_mpad, 3 * plane * sizeof(float));
  if (e != hipSuccess) {
    pl->d_mpad = nullptr;
    bf_destroy(adj);
    bf_destroy(pl);
    return fail(BF_ENOMEM, "hipMalloc reflecting-border adjoint planes failed");
  }
  pl->mirror_adj = adj;
  pl->mpad_plane = plane;
  pl->p.flags |= BF_FLAG_GRAD;
  pl->info.workspace_bytes += adj->info.workspace_bytes + 3 * plane * (int64_t)sizeof(float);
  *out = pl;
  if (wst == BF_WNOGUARANTEE) set_error("order below the bound: no +-delta guarantee");
  return wst;
}

int bf_plan(const bf_params* in, bf_plan_t** out) {
  if (!out) return fail(BF_EINVAL, "out is NULL");
  *out = nullptr;
  bf_params p;
  int st = normalise(in, &p);
  if (st < 0) return st;
  if (p.height <= 0 || p.width <= 0) return fail(BF_EINVAL, "height and width must be > 0");
  bf_plan_info info;
  int ost = plan_order(&p, &info);
  if (ost < 0) return ost;
  if (p.kernel == BF_GAUSS_REC && (p.flags & BF_FLAG_GRAD))
    return fail(BF_EUNSUPPORTED, "the recursive Gaussian has no adjoint");
  if ((p.flags & BF_FLAG_MIRROR) && (p.flags & BF_FLAG_GRAD)) return plan_mirror_adjoint(p, out);
  ForwardPath fpath;
  st = choose_forward_path(p, info.N, &fpath);
  if (st < 0) return st;
  const bool wide = fpath.engine == BF_PATH_WIDE;
  const bool ls = fpath.engine == BF_PATH_STREAMED || wide;  // streamed orders through device memory
  const int variant = fpath.variant, TY = fpath.TY;
  const bool grad = (p.flags & BF_FLAG_GRAD) != 0;
  const bool sigs = p.kernel == BF_GAUSS;
  int bvariant = -1, bTY = 0;
  bool bls = false;
  if (grad) {
    st = (p.flags & BF_FLAG_STREAMED) ? BF_EUNSUPPORTED : choose_backward_tile(p.W, sigs, &bvariant, &bTY);
    if (st < 0) {
      if (!bls_supported(p.W, sigs)) return fail(BF_EUNSUPPORTED, "support W too large for the adjoint");
      bls = true;  // streamed adjoint
      bvariant = -1;
      bTY = 0;
    }
  }

  bf_plan_t* pl = new (std::nothrow) bf_plan_t();
  if (!pl) return fail(BF_ENOMEM, "host allocation failed");
  pl->p = p;
  pl->info = info;
  pl->info.path = fpath.engine;
  pl->info.tile_rows = TY;
  pl->info.tile_cols = (ls || fpath.engine == BF_PATH_RECURSIVE) ? 0 : kTileCols;
  if (ls && !wide && p.kernel == BF_BOX && ls_box_strip_supported(p.W)) {
    const StripShape sh = ls_box_strip_shape(p.height, p.width, p.W, false);
    pl->info.tile_rows = sh.seg_rows;
    pl->info.tile_cols = sh.oc;
  }
  pl->rec = fpath.engine == BF_PATH_RECURSIVE;
  pl->wide = wide;
  pl->variant = variant;
  pl->TY = TY;
  pl->bvariant = bvariant;
  pl->bTY = bTY;
  pl->ls = ls;
  pl->d_ls = nullptr;
  pl->bls = bls;
  pl->d_bls = nullptr;
  std::memset(&pl->bls_state, 0, sizeof(pl->bls_state));
  std::memset(&pl->ls_state, 0, sizeof(pl->ls_state));
  hipGetDevice(&pl->device);

  // constant tables: s, r, inv (N+2 each), taps and d^2 taps (padded)
  int64_t stride = 0, ntapr = 0;
  std::vector<float> h = const_tables(p, info, &stride, &ntapr);
  pl->tab_stride = stride;
  size_t bytes = h.size() * sizeof(float);
  hipError_t e = hipMalloc(&pl->d_const, bytes);
  if (e != hipSuccess) { delete pl; return fail(BF_ENOMEM, "hipMalloc tables failed"); }
  e = hipMemcpy(pl->d_const, h.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) { hipFree(pl->d_const); delete pl; return hip_fail(e, "hipMemcpy tables"); }
  int64_t ws = (int64_t)bytes;
  pl->d_work = nullptr;
  pl->d_partials = nullptr;
  pl->ntiles_b = 0;
  if (grad) {
    int64_t plane = (int64_t)p.height * p.width;
    e = hipMalloc(&pl->d_work, 3 * plane * sizeof(float));
    if (e != hipSuccess) { hipFree(pl->d_const); delete pl; return fail(BF_ENOMEM, "hipMalloc adjoint workspace failed"); }
    ws += 3 * plane * sizeof(float);
    pl->ntiles_b = bls ? kBlsPartials : ((p.height + bTY - 1) / bTY) * ((p.width + kTileCols - 1) / kTileCols);
    e = hipMalloc(&pl->d_partials, 2 * (size_t)pl->ntiles_b * sizeof(double));
    if (e != hipSuccess) {
      hipFree(pl->d_work); hipFree(pl->d_const); delete pl;
      return fail(BF_ENOMEM, "hipMalloc partials failed");
    }
    ws += 2 * (int64_t)pl->ntiles_b * sizeof(double);
  }
  if (ls) {
    // the plain Gaussian forward (no adjoint state, zero border, split passes)
    // keeps its row-filtered images pre-split
    const int nblock = ls_block_orders(p.height, p.width, p.kernel, p.W);
    const bool split = !wide && !grad && p.kernel == BF_GAUSS && !(p.flags & (BF_FLAG_MIRROR | BF_FLAG_MFMA_FP32)) &&
                       ls_split_supported(p.W, nblock);
    const int64_t lb = ls_state_bytes(p.height, p.width, p.W, grad, wide, split, nblock);
    e = hipMalloc(&pl->d_ls, lb);
    if (e != hipSuccess) {
      if (pl->d_work) hipFree(pl->d_work);
      if (pl->d_partials) hipFree(pl->d_partials);
      hipFree(pl->d_const);
      delete pl;
      return fail(BF_ENOMEM, "hipMalloc large-support state failed");
    }
    e = hipMemset(pl->d_ls, 0, lb);  // zero rows around the row-filtered images
    if (e != hipSuccess) {
      hipFree(pl->d_ls);
      hipFree(pl->d_const);
      delete pl;
      return hip_fail(e, "hipMemset large-support state");
    }
    pl->ls_state = ls_layout(pl->d_ls, p.height, p.width, p.W, grad, wide, split, nblock);
    ws += lb;
  }
  if (pl->rec) {
    const int64_t rb = rg_state_bytes(p.height, p.width);
    e = hipMalloc(&pl->d_ls, rb);
    if (e != hipSuccess) {
      hipFree(pl->d_const);
      delete pl;
      return fail(BF_ENOMEM, "hipMalloc recursive-Gaussian state failed");
    }
    pl->ls_state = rg_layout(pl->d_ls, p.height, p.width);
    ws += rb;
  }
  if (bls) {
    const int bblock = bls_block_orders(p.height, p.width);
    const int64_t bb = bls_state_bytes(p.height, p.width, p.W, sigs, bblock);
    e = hipMalloc(&pl->d_bls, bb);
    if (e == hipSuccess) {
      e = hipMemset(pl->d_bls, 0, bb);  // zero rows around the row-filtered images
      if (e != hipSuccess) hipFree(pl->d_bls);
    }
    if (e != hipSuccess) {
      if (pl->d_ls) hipFree(pl->d_ls);
      hipFree(pl->d_work);
      hipFree(pl->d_partials);
      hipFree(pl->d_const);
      delete pl;
      return e == hipErrorOutOfMemory ? fail(BF_ENOMEM, "hipMalloc streamed adjoint state failed")
                                      : hip_fail(e, "streamed adjoint state");
    }
    pl->bls_state = bls_layout(pl->d_bls, p.height, p.width, p.W, sigs, bblock);
    ws += bb;
  }
  pl->info.workspace_bytes = ws;
  *out = pl;
  if (ost == BF_WNOGUARANTEE) set_error("order below the bound: no +-delta guarantee");
  return ost;
}

int bf_plan_clone_workspace(const bf_plan_t* plan, bf_plan_t** out) {
  if (!plan || !out) return fail(BF_EINVAL, "NULL argument");
  *out = nullptr;
  bf_params p = plan->p;  // normalised parameters: the same N, W and tables
  return plan->depth > 0 ? bf_plan_volume(&p, plan->depth, out) : bf_plan(&p, out);
}


int bf_plan_get_info(const bf_plan_t* plan, bf_plan_info* out) {
  if (!plan || !out) return fail(BF_EINVAL, "NULL argument");
  *out = plan->info;
  return BF_OK;
}

int bf_destroy(bf_plan_t* plan) {
  if (!plan) return BF_OK;
  int dev = 0;
  hipGetDevice(&dev);
  hipSetDevice(plan->device);
  if (plan->d_const) hipFree(plan->d_const);
  if (plan->d_work) hipFree(plan->d_work);
  if (plan->d_partials) hipFree(plan->d_partials);
  if (plan->d_ls) hipFree(plan->d_ls);
  if (plan->d_bls) hipFree(plan->d_bls);
  if (plan->d_mpad) hipFree(plan->d_mpad);
  hipSetDevice(dev);
  if (plan->mirror_adj) bf_destroy(plan->mirror_adj);
  delete plan;
  return BF_OK;
}

}  // extern "C"

namespace bfgpa {
static void fill_common_tables(const bf_params& p, const bf_plan_info& info, const float* d_const,
                               int64_t tab_stride, bool wide, TileParams& tp) {
  tp.H = p.height;
  tp.Wd = p.width;
  tp.W = p.W;
  tp.N = info.N;
  tp.kt = p.kernel;
  tp.sigma_r = (float)p.sigma_r;
  tp.inv_sigma_r = (float)(1.0 / p.sigma_r);
  tp.center = (float)p.center;
  tp.inv_T = (float)(1.0 / p.T);
  tp.X = (float)(p.T / p.sigma_r);
  tp.inv_sigma_s3 = p.kernel == BF_GAUSS ? (float)(1.0 / (p.sigma_s * p.sigma_s * p.sigma_s)) : 0.0f;
  const int64_t ntapr = ((2 * p.W + 1 + 2 * kTapPad + 63) / 64) * 64;
  bind_tables(tp, d_const, tab_stride, ntapr);
  tp.rg_tab = p.kernel == BF_GAUSS_REC ? d_const + 7 * tab_stride + 2 * ntapr : nullptr;
  tp.saved_plane = (int64_t)p.height * p.width;
  tp.mirror = (p.flags & BF_FLAG_MIRROR) ? 1 : 0;
  tp.mfma_x3 = (p.flags & BF_FLAG_MFMA_FP32) ? 0 : 1;
  tp.wide = wide ? 1 : 0;
}

static void fill_common(const bf_plan_t* pl, TileParams& tp) {
  fill_common_tables(pl->p, pl->info, pl->d_const, pl->tab_stride, pl->wide, tp);
}

// The streamed forward of a plan, reading the image pointers (and, with
// save, the saved-state pointer) from the device copy `dyn` of the call's
// parameters when the kernels run: the batch captures these launches once
// into its graph and replays them for every call.
hipError_t plan_forward_streamed_dyn(const bf_plan_t* pl, const TileParams* dyn, bool save, hipStream_t s) {
  if (!pl || !dyn || !pl->ls || pl->wide || (save && !pl->ls_state.DP)) return hipErrorInvalidValue;
  TileParams tp;
  std::memset(&tp, 0, sizeof(tp));
  fill_common(pl, tp);
  tp.dyn = dyn;
  tp.dyn_save = save ? 1 : 0;
  tp.TY = pl->TY;
  tp.tiles_x = (pl->p.width + kTileCols - 1) / kTileCols;
  return launch_forward_ls(tp, pl->ls_state, save, s);
}

// The adjoint of bf_backward for a streamed plan, every pointer read from
// device parameters when the kernels run (the batch records it once into its
// adjoint graph): the recompute writes the forward state to fdyn->saved, and
// the adjoint reads in, gout and saved from adyn and writes adyn->out and
// adyn->gsig where they are set.
hipError_t plan_backward_streamed_dyn(const bf_plan_t* pl, const TileParams* fdyn, const TileParams* adyn,
                                      bool recompute, bool sigs, hipStream_t s) {
  if (!pl || !fdyn || !adyn || !pl->ls || pl->wide || pl->mirror_adj || !(pl->p.flags & BF_FLAG_GRAD) ||
      (pl->bvariant < 0 && !pl->bls) || !pl->ls_state.DP)
    return hipErrorInvalidValue;
  TileParams tp;
  std::memset(&tp, 0, sizeof(tp));
  fill_common(pl, tp);
  tp.tiles_x = (pl->p.width + kTileCols - 1) / kTileCols;
  if (recompute) {
    TileParams fp = tp;
    fp.dyn = fdyn;
    fp.dyn_save = 1;
    fp.TY = pl->TY;
    const hipError_t e = launch_forward_ls(fp, pl->ls_state, true, s);
    if (e != hipSuccess) return e;
  }
  tp.dyn = adyn;
  tp.TY = pl->bTY;
  sigs = sigs && pl->p.kernel == BF_GAUSS;
  return pl->bls ? launch_backward_ls(tp, pl->bls_state, sigs, pl->d_partials, nullptr, s)
                 : launch_backward(tp, pl->bvariant, sigs, pl->d_partials, nullptr, s);
}
}  // namespace bfgpa

extern "C" {

int bf_forward(const bf_plan_t* pl, const float* in, int64_t in_pitch, float* out,
               int64_t out_pitch, float* saved, void* stream) {
  if (!pl || !in || !out) return fail(BF_EINVAL, "NULL plan or image pointer");
  if (in_pitch < pl->p.width || out_pitch < pl->p.width) return fail(BF_EINVAL, "pitch smaller than width");
  if ((const void*)in == (const void*)out) return fail(BF_EINVAL, "in and out must not alias");
  if (pl->p.flags & BF_FLAG_JOINT) return fail(BF_EINVAL, "a cross-filter plan runs with bf_forward_joint");
  if (pl->depth > 0) return fail(BF_EINVAL, "a volume plan runs with bf_forward_volume");
  if (saved && (pl->p.flags & BF_FLAG_MIRROR))
    return fail(BF_EUNSUPPORTED, "the reflecting border keeps no adjoint state (its adjoint recomputes)");
  TileParams tp;
  std::memset(&tp, 0, sizeof(tp));
  fill_common(pl, tp);
  tp.in = in;
  tp.in_pitch = in_pitch;
  tp.out = out;
  tp.out_pitch = out_pitch;
  tp.saved = saved;
  tp.TY = pl->TY;
  tp.tiles_x = (pl->p.width + kTileCols - 1) / kTileCols;
  const bool acc64 = (pl->p.flags & BF_FLAG_FP32_ACCUM) == 0;
  hipError_t e;
  if (pl->ls) {
    if (saved && !pl->ls_state.DP)
      return fail(BF_EINVAL, "saved state needs a plan built with BF_FLAG_GRAD");
    e = pl->wide ? launch_forward_wide(tp, pl->ls_state, (hipStream_t)stream)
                 : launch_forward_ls(tp, pl->ls_state, saved != nullptr, (hipStream_t)stream);
  } else if (pl->rec) {
    if (saved) return fail(BF_EINVAL, "the recursive Gaussian keeps no adjoint state");
    e = launch_forward_rg(tp, pl->ls_state, (hipStream_t)stream);
  } else {
    e = launch_forward(tp, pl->variant, acc64, saved != nullptr, (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(e, "forward launch");
  return BF_OK;
}

int bf_forward_noalloc(const bf_params* in_p, const float* in, int64_t in_pitch, float* out,
                       int64_t out_pitch, void* stream) {
  if (!in_p || !in || !out) return fail(BF_EINVAL, "NULL parameter or image pointer");
  bf_params p;
  int st = normalise(in_p, &p);
  if (st < 0) return st;
  if (p.height <= 0 || p.width <= 0) return fail(BF_EINVAL, "height and width must be > 0");
  if (in_pitch < p.width || out_pitch < p.width) return fail(BF_EINVAL, "pitch smaller than width");
  if ((const void*)in == (const void*)out) return fail(BF_EINVAL, "in and out must not alias");
  if (p.flags & (BF_FLAG_GRAD | BF_FLAG_JOINT | BF_FLAG_STREAMED))
    return fail(BF_EUNSUPPORTED, "the allocation-free forward is the plain fused-tile forward "
                                 "(no adjoint, cross filter or streamed engine)");
  bf_plan_info info;
  const int ost = plan_order(&p, &info);
  if (ost < 0) return ost;
  ForwardPath fpath;
  st = choose_forward_path(p, info.N, &fpath);
  if (st < 0) return st;
  if (fpath.engine != BF_PATH_TILE)
    return fail(BF_EUNSUPPORTED, "the allocation-free forward serves the fused-tile engine only; this image "
                                 "size and support take an engine whose per-pixel state needs bf_plan's workspace");
  int64_t stride = 0, ntapr = 0;
  const std::vector<float> h = const_tables(p, info, &stride, &ntapr);
  if ((int64_t)h.size() > noalloc_capacity_floats())
    return fail(BF_EINVAL, "constant tables of " + std::to_string(h.size()) + " floats exceed the static buffer of " +
                               std::to_string(noalloc_capacity_floats()) + " (order N too large)");
  float* d = nullptr;
  hipError_t e = noalloc_scratch(&d);
  if (e != hipSuccess) return hip_fail(e, "static table buffer address");
  const hipStream_t s = (hipStream_t)stream;
  e = noalloc_fill(d, h.data(), (int64_t)h.size(), s);
  if (e != hipSuccess) return hip_fail(e, "static table fill");
  TileParams tp;
  std::memset(&tp, 0, sizeof(tp));
  fill_common_tables(p, info, d, stride, false, tp);
  tp.in = in;
  tp.in_pitch = in_pitch;
  tp.out = out;
  tp.out_pitch = out_pitch;
  tp.TY = fpath.TY;
  tp.tiles_x = (p.width + kTileCols - 1) / kTileCols;
  const bool acc64 = (p.flags & BF_FLAG_FP32_ACCUM) == 0;
  e = launch_forward(tp, fpath.variant, acc64, false, s);
  if (e != hipSuccess) return hip_fail(e, "forward launch");
  if (ost == BF_WNOGUARANTEE) set_error("order below the bound: no +-delta guarantee");
  return ost;
}

int bf_plan_volume(const bf_params* in, int32_t depth, bf_plan_t** out) {
  if (!out) return fail(BF_EINVAL, "out is NULL");
  *out = nullptr;
  if (depth <= 0) return fail(BF_EINVAL, "depth must be > 0");
  bf_params p;
  int st = normalise(in, &p);
  if (st < 0) return st;
  if (p.height <= 0 || p.width <= 0) return fail(BF_EINVAL, "height and width must be > 0");
  if (p.kernel == BF_GAUSS_REC) return fail(BF_EUNSUPPORTED, "volumes take the box or the truncated Gaussian");
  if (p.flags & (BF_FLAG_GRAD | BF_FLAG_JOINT | BF_FLAG_TILE_VALU))
    return fail(BF_EUNSUPPORTED, "volumes: forward filter (zero or mirror border), streamed engine only");
  if (p.W > kVolMaxW) return fail(BF_EUNSUPPORTED, "volumes: W <= 32");
  if ((int64_t)depth * p.height > (1 << 30) / std::max(1, p.width))
    return fail(BF_EUNSUPPORTED, "volume too large");
  bf_plan_info info;
  const int ost = plan_order(&p, &info, 3);
  if (ost < 0) return ost;
  // T/sigma_r above 13: the Gaussian's float64-state (wide-range) passes
  const bool wide = info.lambda > kLambdaF32;
  if (wide && (p.kernel != BF_GAUSS || (p.flags & BF_FLAG_MFMA_FP32)))
    return fail(BF_EUNSUPPORTED, "sigma_r too small for float32 volumes: T/sigma_r above 13 takes the Gaussian "
                                 "on its split-bfloat16 passes only");
  bf_plan_t* pl = new (std::nothrow) bf_plan_t();
  if (!pl) return fail(BF_ENOMEM, "host allocation failed");
  pl->p = p;
  pl->info = info;
  pl->info.path = BF_PATH_VOLUME;
  pl->wide = wide;
  pl->variant = -1;
  pl->bvariant = -1;
  pl->depth = depth;
  hipGetDevice(&pl->device);
  int64_t stride = 0, ntapr = 0;
  std::vector<float> h = const_tables(p, info, &stride, &ntapr);
  pl->tab_stride = stride;
  const size_t bytes = h.size() * sizeof(float);
  hipError_t e = hipMalloc(&pl->d_const, bytes);
  if (e != hipSuccess) { delete pl; return fail(BF_ENOMEM, "hipMalloc tables failed"); }
  e = hipMemcpy(pl->d_const, h.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) { hipFree(pl->d_const); delete pl; return hip_fail(e, "hipMemcpy tables"); }
  const int64_t vb = vol_state_bytes(depth, p.height, p.width, p.W, wide);
  e = hipMalloc(&pl->d_ls, vb);
  if (e == hipSuccess) {
    e = hipMemset(pl->d_ls, 0, vb);  // zero rows around the row-filtered images
    if (e != hipSuccess) hipFree(pl->d_ls);
  }
  if (e != hipSuccess) {
    hipFree(pl->d_const);
    delete pl;
    return e == hipErrorOutOfMemory ? fail(BF_ENOMEM, "hipMalloc volume state failed") : hip_fail(e, "volume state");
  }
  pl->ls_state = vol_layout(pl->d_ls, depth, p.height, p.width, p.W, &pl->vol, wide);
  pl->info.workspace_bytes = (int64_t)bytes + vb;
  *out = pl;
  if (ost == BF_WNOGUARANTEE) set_error("order below the bound: no +-delta guarantee");
  return ost;
}

int bf_forward_volume(const bf_plan_t* pl, const float* in, int64_t in_pitch, float* out, int64_t out_pitch,
                      void* stream) {
  if (!pl || !in || !out) return fail(BF_EINVAL, "NULL plan or volume pointer");
  if (pl->depth <= 0) return fail(BF_EINVAL, "plan was not built with bf_plan_volume");
  if (in_pitch < pl->p.width || out_pitch < pl->p.width) return fail(BF_EINVAL, "pitch smaller than width");
  if ((const void*)in == (const void*)out) return fail(BF_EINVAL, "in and out must not alias");
  TileParams tp;
  std::memset(&tp, 0, sizeof(tp));
  fill_common(pl, tp);
  tp.H = pl->depth * pl->p.height;  // slices stacked as one image
  tp.in = in;
  tp.in_pitch = in_pitch;
  tp.out = out;
  tp.out_pitch = out_pitch;
  hipError_t e = launch_forward_vol(tp, pl->ls_state, pl->vol, pl->depth, pl->p.height, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "volume forward launch");
  return BF_OK;
}

int bf_image_range(const float* in, int64_t pitch, int32_t height, int32_t width, float* minmax,
                   void* stream) {
  if (!in || !minmax) return fail(BF_EINVAL, "NULL image or output pointer");
  if (height < 0 || width < 0 || pitch < width) return fail(BF_EINVAL, "bad size or pitch");
  hipError_t e = launch_range(in, pitch, height, width, minmax, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "range launch");
  return BF_OK;
}

int bf_forward_joint(const bf_plan_t* pl, const float* in, int64_t in_pitch, const float* guide,
                     int64_t guide_pitch, float* out, int64_t out_pitch, void* stream) {
  if (!pl || !in || !guide || !out) return fail(BF_EINVAL, "NULL plan or image pointer");
  if (!(pl->p.flags & BF_FLAG_JOINT)) return fail(BF_EINVAL, "plan was built without BF_FLAG_JOINT");
  if (in_pitch < pl->p.width || guide_pitch < pl->p.width || out_pitch < pl->p.width)
    return fail(BF_EINVAL, "pitch smaller than width");
  if ((const void*)in == (const void*)out || (const void*)guide == (const void*)out)
    return fail(BF_EINVAL, "out must not alias in or guide");
  TileParams tp;
  std::memset(&tp, 0, sizeof(tp));
  fill_common(pl, tp);
  tp.in = in;
  tp.in_pitch = in_pitch;
  tp.guide = guide;
  tp.guide_pitch = guide_pitch;
  tp.out = out;
  tp.out_pitch = out_pitch;
  tp.TY = pl->TY;
  tp.tiles_x = (pl->p.width + kTileCols - 1) / kTileCols;
  hipError_t e = launch_joint(tp, pl->variant, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "cross-filter launch");
  return BF_OK;
}

int bf_backward(const bf_plan_t* pl, const float* in, int64_t in_pitch, const float* grad_out,
                int64_t gout_pitch, const float* saved, float* grad_in, int64_t gin_pitch,
                double* grad_sigma, void* stream) {
  if (!pl || !in || !grad_out) return fail(BF_EINVAL, "NULL plan or image pointer");
  if (!(pl->p.flags & BF_FLAG_GRAD) || (pl->bvariant < 0 && !pl->bls && !pl->mirror_adj))
    return fail(BF_EINVAL, "plan was built without BF_FLAG_GRAD");
  if (in_pitch < pl->p.width || gout_pitch < pl->p.width || (grad_in && gin_pitch < pl->p.width))
    return fail(BF_EINVAL, "pitch smaller than width");
  hipStream_t s = (hipStream_t)stream;
  if (pl->mirror_adj) {
    if (saved) return fail(BF_EUNSUPPORTED, "the reflecting border keeps no adjoint state: saved must be NULL");
    const int H = pl->p.height, Wd = pl->p.width, W = pl->p.W;
    const int64_t Wp = Wd + 2 * W;
    float* fpad = pl->d_mpad;
    float* gpad = fpad + pl->mpad_plane;
    float* ipad = gpad + pl->mpad_plane;
    hipError_t e = launch_mirror_pad(in, in_pitch, grad_out, gout_pitch, H, Wd, W, fpad, gpad, s);
    if (e != hipSuccess) return hip_fail(e, "reflecting-border pad launch");
    const int st = bf_backward(pl->mirror_adj, fpad, Wp, gpad, Wp, nullptr, grad_in ? ipad : nullptr, Wp,
                               grad_sigma, stream);
    if (st < 0) return st;
    if (grad_in) {
      e = launch_mirror_fold(ipad, H, Wd, W, grad_in, gin_pitch, s);
      if (e != hipSuccess) return hip_fail(e, "reflecting-border fold launch");
    }
    return BF_OK;
  }
  TileParams tp;
  std::memset(&tp, 0, sizeof(tp));
  fill_common(pl, tp);
  const bool acc64 = (pl->p.flags & BF_FLAG_FP32_ACCUM) == 0;
  if (!saved) {
    // recompute the forward state into the plan's workspace
    TileParams fp = tp;
    fp.in = in;
    fp.in_pitch = in_pitch;
    fp.out = nullptr;
    fp.out_pitch = 0;
    fp.saved = pl->d_work;
    fp.TY = pl->TY;
    fp.tiles_x = (pl->p.width + kTileCols - 1) / kTileCols;
    hipError_t e = pl->ls     ? launch_forward_ls(fp, pl->ls_state, true, s)
                              : launch_forward(fp, pl->variant, acc64, true, s);
    if (e != hipSuccess) return hip_fail(e, "forward (recompute) launch");
    saved = pl->d_work;
  }
  tp.in = in;
  tp.in_pitch = in_pitch;
  tp.gout = grad_out;
  tp.gout_pitch = gout_pitch;
  tp.saved = const_cast<float*>(saved);
  tp.out = grad_in;
  tp.out_pitch = grad_in ? gin_pitch : 0;
  tp.TY = pl->bTY;
  tp.tiles_x = (pl->p.width + kTileCols - 1) / kTileCols;
  const bool sigs = pl->p.kernel == BF_GAUSS && grad_sigma != nullptr;
  hipError_t e = pl->bls ? launch_backward_ls(tp, pl->bls_state, sigs, pl->d_partials, grad_sigma, s)
                         : launch_backward(tp, pl->bvariant, sigs, pl->d_partials, grad_sigma, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  return BF_OK;
}

}  // extern "C"
