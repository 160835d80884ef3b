// Single-image kernels: fused forward (Algorithm 2) and its adjoint.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "bf_device.h"
#include "bf_internal.h"

namespace bfgpa {

// ---------------------------------------------------------------------------
// Forward
// ---------------------------------------------------------------------------
template <int KT, int OPT, int MREG, bool ACC64, bool SAVE>
__global__ __launch_bounds__(kThreads) void gpa_forward_kernel(TileParams p) {
  extern __shared__ float lds[];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int ty = tile / p.tiles_x;
  const int tx = tile - ty * p.tiles_x;
  forward_tile<KT, OPT, MREG, ACC64, SAVE>(p, ty * 4 * OPT, tx * kTileCols, lds);
}

// (output rows per thread, region pixels per thread); tile rows = 4 * OPT.
static const Variant kFwdVariants[] = {{8, 12}, {8, 20}, {8, 32}, {16, 40}, {4, 32}, {4, 48}, {4, 72}, {8, 48}};
static constexpr int kNumFwdVariants = sizeof(kFwdVariants) / sizeof(kFwdVariants[0]);
int forward_variant_count() { return kNumFwdVariants; }
Variant forward_variant(int v) { return kFwdVariants[v]; }

int64_t forward_lds_bytes(int TY, int W) {
  const int64_t npx = region_floats(TY, W);
  return 4 * (((npx + 3) & ~3LL) + (int64_t)(TY + 2 * W) * kHPitch);
}

int max_lds_bytes() { return 160 * 1024; }

template <int KT, int OPT, int MREG, bool ACC64, bool SAVE>
static hipError_t launch_fwd_t(const TileParams& p, hipStream_t s) {
  auto kern = gpa_forward_kernel<KT, OPT, MREG, ACC64, SAVE>;
  const int64_t lds = forward_lds_bytes(4 * OPT, p.W);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       max_lds_bytes());
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int tiles = ((p.H + 4 * OPT - 1) / (4 * OPT)) * p.tiles_x;
  hipLaunchKernelGGL(kern, dim3(tiles), dim3(kThreads), (size_t)lds, s, p);
  return hipGetLastError();
}

template <int KT, int OPT, int MREG>
static hipError_t launch_fwd_v(const TileParams& p, bool acc64, bool save, hipStream_t s) {
  if (acc64)
    return save ? launch_fwd_t<KT, OPT, MREG, true, true>(p, s)
                : launch_fwd_t<KT, OPT, MREG, true, false>(p, s);
  return save ? launch_fwd_t<KT, OPT, MREG, false, true>(p, s)
              : launch_fwd_t<KT, OPT, MREG, false, false>(p, s);
}

template <int KT>
static hipError_t launch_fwd_k(const TileParams& p, int variant, bool acc64, bool save,
                               hipStream_t s) {
  switch (variant) {
    case 0: return launch_fwd_v<KT, 8, 12>(p, acc64, save, s);
    case 1: return launch_fwd_v<KT, 8, 20>(p, acc64, save, s);
    case 2: return launch_fwd_v<KT, 8, 32>(p, acc64, save, s);
    case 3: return launch_fwd_v<KT, 16, 40>(p, acc64, save, s);
    case 4: return launch_fwd_v<KT, 4, 32>(p, acc64, save, s);
    case 5: return launch_fwd_v<KT, 4, 48>(p, acc64, save, s);
    case 6: return launch_fwd_v<KT, 4, 72>(p, acc64, save, s);
    default: return launch_fwd_v<KT, 8, 48>(p, acc64, save, s);
  }
}

hipError_t launch_forward(const TileParams& p, int variant, bool acc64, bool save,
                          hipStream_t s) {
  if (variant < 0 || variant >= kNumFwdVariants) return hipErrorInvalidValue;
  const Variant v = forward_variant(variant);
  if (p.TY != 4 * v.opt) return hipErrorInvalidValue;
  if (region_floats(p.TY, p.W) > (int64_t)kThreads * v.mreg) return hipErrorInvalidValue;
  if (forward_lds_bytes(p.TY, p.W) > max_lds_bytes()) return hipErrorInvalidValue;
  if (p.H <= 0 || p.Wd <= 0) return hipSuccess;
  return p.kt == BF_BOX ? launch_fwd_k<BF_BOX>(p, variant, acc64, save, s)
                        : launch_fwd_k<BF_GAUSS>(p, variant, acc64, save, s);
}

// ---------------------------------------------------------------------------
// Adjoint.  With gbar = dL/dout, p_i = gbar sigma_r / Q~_i and
// rho_i = P~_i / Q~_i (saved by the forward), the scaled adjoint image of
// F~_m is  adj_m(i) = p_i (b_m(i) [m >= 1] - rho_i a_m(i) [m <= N-1])
// (a_m, b_m the forward's coefficient recursions).  Filtering adj_m with
// the (symmetric, zero-extended, hence self-adjoint) spatial kernel and
// multiplying by dF~_m/dx = m F~_{m-1}/r_m - x F~_m gives the part of
// dL/dx flowing through the auxiliary images; the part through the
// coefficients is p_i (D_P - rho_i D_Q), saved by the forward.
// dL/dsigma_r = sum gbar rho - sum dL/dx x / sigma_r;
// dL/dsigma_s = sum_m <adj_m, w' * F~_m>, w' = w |j|^2 / sigma_s^3, a sum of
// two separable filters.
// ---------------------------------------------------------------------------
template <int KT, int OPT, int MREG, bool SIGS>
__global__ __launch_bounds__(kThreads) void gpa_backward_kernel(TileParams p, double* partials) {
  extern __shared__ float lds[];
  __shared__ double red[2][kThreads];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tyi = tile / p.tiles_x;
  const int txi = tile - tyi * p.tiles_x;
  const int r0 = tyi * p.TY, c0 = txi * kTileCols;
  const int W = p.W, N = p.N;
  const RegionGeom g = region_geom(4 * OPT, W);
  const int np4 = align4(g.npx);
  float* As = lds;
  float* Hs = As + np4;
  float* Fs2 = Hs + g.RH * kHPitch;
  float* Hg = Fs2 + np4;
  float* Hg2 = Hg + g.RH * kHPitch;
  const float* tz = p.taps + kTapPad;
  const float* tz2 = p.taps2 + kTapPad;

  // region state: x, a', b' (a, b scaled by p_i), rho, F~
  float xr[MREG], ar[MREG], br[MREG], rr[MREG], fr[SIGS ? MREG : 1];
  for_region<MREG>(g, r0, c0, W, p.H, p.Wd, [&](int m, int q, bool inside, int gr, int gc) {
    float x = 0.f, a = 0.f, rho = 0.f, F = 0.f;
    if (inside) {
      x = (p.in[(int64_t)gr * p.in_pitch + gc] - p.center) / p.sigma_r;
      F = expf(-0.5f * x * x);
      const int64_t idx = (int64_t)gr * p.Wd + gc;
      const float Qs = p.saved[idx];
      rho = p.saved[p.saved_plane + idx];
      const float pb = p.gout[(int64_t)gr * p.gout_pitch + gc] * p.sigma_r / Qs;
      a = pb * F;
    }
    xr[m] = x;
    ar[m] = a;
    br[m] = 0.f;
    rr[m] = rho;
    if (SIGS) fr[m] = F;
  });

  const int lane = threadIdx.x & 63;
  const int orow0 = (threadIdx.x >> 6) * OPT;
  const int gc = c0 + lane;
  float xo[OPT], fp[OPT], fc[OPT];
  double dx[OPT], dss[OPT];
#pragma unroll
  for (int s = 0; s < OPT; ++s) {
    const int gr = r0 + orow0 + s;
    float x = 0.f, F = 0.f;
    if (gr < p.H && gc < p.Wd) {
      x = (p.in[(int64_t)gr * p.in_pitch + gc] - p.center) / p.sigma_r;
      F = expf(-0.5f * x * x);
    }
    xo[s] = x;
    fc[s] = F;     // F~_m at the output pixel
    fp[s] = 0.f;   // F~_{m-1}
    dx[s] = 0.0;
    dss[s] = 0.0;
  }

  for (int m = 0; m <= N; ++m) {
    const float sm = p.s_tab[m];
    const float rm1 = p.r_tab[m + 1];
    const float im1 = p.inv_tab[m + 1];
#pragma unroll
    for (int k = 0; k < MREG; ++k) {
      float adj = 0.f;
      if (m >= 1) adj = br[k];
      if (m <= N - 1) adj = fmaf(-rr[k], ar[k], adj);
      const int q = threadIdx.x + kThreads * k;
      if (q < g.npx) As[q] = adj;
      if (SIGS) {
        if (m > 0) fr[k] *= xr[k] * sm;
        if (q < g.npx) Fs2[q] = fr[k];
      }
      const float bn = ar[k] * rm1;
      ar[k] = bn * (xr[k] * im1);
      br[k] = bn;
    }
    __syncthreads();
    rowpass<KT>(As, g.RWp, Hs, g.RH, W, tz);
    if (SIGS) {
      rowpass_fir_any(Fs2, g.RWp, Hg, g.RH, W, tz);
      rowpass_fir_any(Fs2, g.RWp, Hg2, g.RH, W, tz2);
    }
    __syncthreads();
    float fa[OPT];
    colpass<KT, OPT>(Hs, orow0, lane, W, tz, fa);
    if (SIGS) {
      float u[OPT], u2[OPT];
      colpass<BF_GAUSS, OPT>(Hg, orow0, lane, W, tz2, u);   // d^2 g along rows of g-filtered
      colpass<BF_GAUSS, OPT>(Hg2, orow0, lane, W, tz, u2);  // g along rows of d^2 g-filtered
#pragma unroll
      for (int s = 0; s < OPT; ++s) {
        const float adj_i = As[(orow0 + s + W) * g.RWp + lane + W];
        dss[s] = fma((double)adj_i, (double)(u[s] + u2[s]), dss[s]);
      }
    }
    const float fm = (float)m * sm;
#pragma unroll
    for (int s = 0; s < OPT; ++s) {
      const float factor = fmaf(fm, fp[s], -xo[s] * fc[s]);  // dF~_m/dx
      dx[s] = fma((double)fa[s], (double)factor, dx[s]);
      fp[s] = fc[s];
      fc[s] *= xo[s] * p.s_tab[m + 1];
    }
    if (SIGS) __syncthreads();  // As is re-written by the next m
  }

  double dsr_loc = 0.0, dss_loc = 0.0;
#pragma unroll
  for (int s = 0; s < OPT; ++s) {
    const int gr = r0 + orow0 + s;
    if (gr < p.H && gc < p.Wd) {
      const int64_t idx = (int64_t)gr * p.Wd + gc;
      const float gb = p.gout[(int64_t)gr * p.gout_pitch + gc];
      const double Qs = p.saved[idx];
      const double rho = p.saved[p.saved_plane + idx];
      const double Dc = p.saved[2 * p.saved_plane + idx];
      const double pb = (double)gb * (double)p.sigma_r / Qs;
      const double dxt = dx[s] + pb * Dc;
      if (p.out) p.out[(int64_t)gr * p.out_pitch + gc] = (float)(dxt / (double)p.sigma_r);
      dsr_loc += (double)gb * rho - dxt * (double)xo[s] / (double)p.sigma_r;
      dss_loc += dss[s];
    }
  }
  // deterministic workgroup reduction
  red[0][threadIdx.x] = dsr_loc;
  red[1][threadIdx.x] = dss_loc * (double)p.inv_sigma_s3;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * (int64_t)tile] = red[0][0];
    partials[2 * (int64_t)tile + 1] = red[1][0];
  }
}

// Fixed-order sum of the per-tile partials.
__global__ __launch_bounds__(kThreads) void sigma_reduce_kernel(const double* partials, int ntiles,
                                                                 int has_ss, double* out) {
  __shared__ double red[2][kThreads];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < ntiles; i += kThreads) {
    a += partials[2 * (int64_t)i];
    b += partials[2 * (int64_t)i + 1];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0][0];
    out[1] = has_ss ? red[1][0] : __builtin_nan("");
  }
}

hipError_t launch_sigma_reduce(const double* partials, int n, bool has_ss, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sigma_reduce_kernel, dim3(1), dim3(kThreads), 0, s, partials, n, has_ss ? 1 : 0, out);
  return hipGetLastError();
}

static const Variant kBwdVariants[] = {{8, 24}, {4, 32}};
int backward_variant_count() { return 2; }
Variant backward_variant(int v) { return kBwdVariants[v]; }

int64_t backward_lds_bytes(int TY, int W, bool sigs) {
  const int64_t np4 = (region_floats(TY, W) + 3) & ~3LL;
  const int64_t hs = (int64_t)(TY + 2 * W) * kHPitch;
  return 4 * (np4 + hs + (sigs ? np4 + 2 * hs : 0));
}

template <int KT, int OPT, int MREG, bool SIGS>
static hipError_t launch_bwd_t(const TileParams& p, double* partials, hipStream_t s) {
  auto kern = gpa_backward_kernel<KT, OPT, MREG, SIGS>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       max_lds_bytes() - 2 * kThreads * 8);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int tiles = ((p.H + 4 * OPT - 1) / (4 * OPT)) * p.tiles_x;
  hipLaunchKernelGGL(kern, dim3(tiles), dim3(kThreads), (size_t)backward_lds_bytes(4 * OPT, p.W, SIGS),
                     s, p, partials);
  return hipGetLastError();
}

template <int KT, bool SIGS>
static hipError_t launch_bwd_k(const TileParams& p, int variant, double* partials, hipStream_t s) {
  return variant == 0 ? launch_bwd_t<KT, 8, 24, SIGS>(p, partials, s)
                      : launch_bwd_t<KT, 4, 32, SIGS>(p, partials, s);
}

hipError_t launch_backward(const TileParams& p, int variant, bool sigs, double* partials,
                           double* grad_sigma, hipStream_t s) {
  const Variant v = backward_variant(variant);
  if (p.TY != 4 * v.opt) return hipErrorInvalidValue;
  if (region_floats(p.TY, p.W) > (int64_t)kThreads * v.mreg) return hipErrorInvalidValue;
  if (backward_lds_bytes(p.TY, p.W, sigs) + 2 * kThreads * 8 > max_lds_bytes()) return hipErrorInvalidValue;
  if (p.H <= 0 || p.Wd <= 0) return hipSuccess;
  hipError_t e;
  if (p.kt == BF_BOX)
    e = launch_bwd_k<BF_BOX, false>(p, variant, partials, s);
  else
    e = sigs ? launch_bwd_k<BF_GAUSS, true>(p, variant, partials, s)
             : launch_bwd_k<BF_GAUSS, false>(p, variant, partials, s);
  if (e != hipSuccess || !grad_sigma) return e;
  const int tiles = ((p.H + p.TY - 1) / p.TY) * p.tiles_x;
  hipLaunchKernelGGL(sigma_reduce_kernel, dim3(1), dim3(kThreads), 0, s, (const double*)partials,
                     tiles, (p.kt == BF_GAUSS && sigs) ? 1 : 0, grad_sigma);
  return hipGetLastError();
}

}  // namespace bfgpa
