// Single-image kernels: fused forward (Algorithm 2) and its adjoint.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <cstdint>

#include "bf_device.h"
#include "bf_internal.h"

namespace bfgpa {

// ---------------------------------------------------------------------------
// Forward
// ---------------------------------------------------------------------------
template <int KT, int OPT, int MREG, bool ACC64, bool SAVE>
__global__ __launch_bounds__(kThreads, (OPT * MREG <= 256 ? 2 : 1)) void gpa_forward_kernel(TileParams p) {
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
  // the float64-sum forward at a support compiled as a constant (bf_fused_w.hip)
  if (acc64 && fixed_w_available(p.W, variant)) return launch_forward_fixed_w(p, save, s);
  return p.kt == BF_BOX ? launch_fwd_k<BF_BOX>(p, variant, acc64, save, s)
                        : launch_fwd_k<BF_GAUSS>(p, variant, acc64, save, s);
}

// ---------------------------------------------------------------------------
// Data range of an image (min and max), for planning with T and c taken from
// the data: with c = (min + max)/2 and T = (max - min)/2 every |f - c| <= T,
// so Prop. (accuracy) still holds, and a narrower range lowers lambda and N.
// NaNs are skipped.  Two launches: the output pair is set to (+inf, -inf),
// then every workgroup folds its share in with compare-and-swap loops.
// ---------------------------------------------------------------------------
__global__ void range_init_kernel(float* mm) {
  if (threadIdx.x == 0) {
    mm[0] = __builtin_huge_valf();
    mm[1] = -__builtin_huge_valf();
  }
}

__device__ __forceinline__ void atomic_fmin(float* a, float v) {
  int* ai = (int*)a;
  int old = __float_as_int(*(volatile float*)a);
  while (v < __int_as_float(old)) {
    const int assumed = old;
    old = atomicCAS(ai, assumed, __float_as_int(v));
    if (old == assumed) break;
  }
}

__device__ __forceinline__ void atomic_fmax(float* a, float v) {
  int* ai = (int*)a;
  int old = __float_as_int(*(volatile float*)a);
  while (v > __int_as_float(old)) {
    const int assumed = old;
    old = atomicCAS(ai, assumed, __float_as_int(v));
    if (old == assumed) break;
  }
}

__global__ __launch_bounds__(kThreads) void range_kernel(const float* __restrict__ in, int64_t pitch, int H, int Wd,
                                                         float* mm) {
  __shared__ float smin[kThreads], smax[kThreads];
  float lo = __builtin_huge_valf(), hi = -__builtin_huge_valf();
  const int64_t npx = (int64_t)H * Wd;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < npx; i += (int64_t)gridDim.x * kThreads) {
    const int r = (int)(i / Wd), c = (int)(i - (int64_t)r * Wd);
    const float v = in[(int64_t)r * pitch + c];
    lo = fminf(lo, v);  // fminf/fmaxf return the other operand for a NaN
    hi = fmaxf(hi, v);
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + w]);
      smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomic_fmin(mm, smin[0]);
    atomic_fmax(mm + 1, smax[0]);
  }
}

hipError_t launch_range(const float* in, int64_t pitch, int H, int Wd, float* mm, hipStream_t s) {
  hipLaunchKernelGGL(range_init_kernel, dim3(1), dim3(64), 0, s, mm);
  const int64_t npx = (int64_t)H * Wd;
  const int g = (int)std::max<int64_t>(1, std::min<int64_t>((npx + kThreads - 1) / kThreads, 1024));
  hipLaunchKernelGGL(range_kernel, dim3(g), dim3(kThreads), 0, s, in, pitch, H, Wd, mm);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cross (joint) filter: fused tiles only (joint_tile, bf_device.h).
// ---------------------------------------------------------------------------
template <int KT, int OPT, int MREG>
__global__ __launch_bounds__(kThreads) void gpa_joint_kernel(TileParams p) {
  extern __shared__ float lds[];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int ty = tile / p.tiles_x;
  const int tx = tile - ty * p.tiles_x;
  joint_tile<KT, OPT, MREG>(p, ty * 4 * OPT, tx * kTileCols, lds);
}

// three region arrays per thread (F^, y, f): the smaller register budgets only
static const Variant kJointVariants[] = {{8, 12}, {8, 20}, {8, 32}, {4, 32}};
int joint_variant_count() { return 4; }
Variant joint_variant(int v) { return kJointVariants[v]; }

int64_t joint_lds_bytes(int TY, int W) {
  const int64_t npx = region_floats(TY, W);
  return 4 * (2 * ((npx + 3) & ~3LL) + 2 * (int64_t)(TY + 2 * W) * kHPitch);
}

template <int KT, int OPT, int MREG>
static hipError_t launch_joint_t(const TileParams& p, hipStream_t s) {
  auto kern = gpa_joint_kernel<KT, OPT, MREG>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
  if (e != hipSuccess) return e;
  const int tiles = ((p.H + 4 * OPT - 1) / (4 * OPT)) * p.tiles_x;
  hipLaunchKernelGGL(kern, dim3(tiles), dim3(kThreads), (size_t)joint_lds_bytes(4 * OPT, p.W), s, p);
  return hipGetLastError();
}

template <int KT>
static hipError_t launch_joint_k(const TileParams& p, int variant, hipStream_t s) {
  switch (variant) {
    case 0: return launch_joint_t<KT, 8, 12>(p, s);
    case 1: return launch_joint_t<KT, 8, 20>(p, s);
    case 2: return launch_joint_t<KT, 8, 32>(p, s);
    default: return launch_joint_t<KT, 4, 32>(p, s);
  }
}

hipError_t launch_joint(const TileParams& p, int variant, hipStream_t s) {
  if (variant < 0 || variant >= joint_variant_count() || !p.guide) return hipErrorInvalidValue;
  const Variant v = joint_variant(variant);
  if (p.TY != 4 * v.opt) return hipErrorInvalidValue;
  if (region_floats(p.TY, p.W) > (int64_t)kThreads * v.mreg) return hipErrorInvalidValue;
  if (joint_lds_bytes(p.TY, p.W) > max_lds_bytes()) return hipErrorInvalidValue;
  if (p.H <= 0 || p.Wd <= 0) return hipSuccess;
  return p.kt == BF_BOX ? launch_joint_k<BF_BOX>(p, variant, s) : launch_joint_k<BF_GAUSS>(p, variant, s);
}

// ---------------------------------------------------------------------------
// Adjoint kernels (the per-tile arithmetic, backward_tile, is in bf_device.h).
// ---------------------------------------------------------------------------
template <int KT, int OPT, int MREG, bool SIGS>
__global__ __launch_bounds__(kThreads, (OPT * MREG <= 256 ? 2 : 1)) void gpa_backward_kernel(TileParams pk, double* partials) {
  const TileParams p = with_dyn(pk);
  extern __shared__ float lds[];
  __shared__ double red[2 * kThreads];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tyi = tile / p.tiles_x;
  const int txi = tile - tyi * p.tiles_x;
  backward_tile<KT, OPT, MREG, SIGS>(p, tyi * p.TY, txi * kTileCols, lds, red, partials + 2 * (int64_t)tile);
}

// Fixed-order sum of the per-tile partials.
__global__ __launch_bounds__(kThreads) void sigma_reduce_kernel(const double* partials, int ntiles,
                                                                 int has_ss, double* out, const TileParams* dyn) {
  __shared__ double red[2][kThreads];
  if (dyn) out = dyn->gsig;  // uniform
  if (!out) return;
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

hipError_t launch_sigma_reduce(const double* partials, int n, bool has_ss, double* out, const TileParams* dyn,
                               hipStream_t s) {
  hipLaunchKernelGGL(sigma_reduce_kernel, dim3(1), dim3(kThreads), 0, s, partials, n, has_ss ? 1 : 0, out, dyn);
  return hipGetLastError();
}

// {4, 20} first: its LDS (about 75 KB at W = 15) lets two workgroups share a
// CU, where the 32-row tiles' 100 KB allow one
static const Variant kBwdVariants[] = {{4, 20}, {8, 24}, {4, 32}};
int backward_variant_count() { return 3; }
Variant backward_variant(int v) { return kBwdVariants[v]; }

int64_t backward_lds_bytes(int TY, int W, bool sigs) {
  const int64_t np4 = (region_floats_bwd(TY, W) + 3) & ~3LL;
  const int64_t hs = (int64_t)(TY + 2 * W) * kHPitchBwd;
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
  return variant == 0   ? launch_bwd_t<KT, 4, 20, SIGS>(p, partials, s)
         : variant == 1 ? launch_bwd_t<KT, 8, 24, SIGS>(p, partials, s)
                        : launch_bwd_t<KT, 4, 32, SIGS>(p, partials, s);
}

hipError_t launch_backward(const TileParams& p, int variant, bool sigs, double* partials,
                           double* grad_sigma, hipStream_t s) {
  const Variant v = backward_variant(variant);
  if (p.TY != 4 * v.opt) return hipErrorInvalidValue;
  if (region_floats_bwd(p.TY, p.W) > (int64_t)kThreads * v.mreg) return hipErrorInvalidValue;
  if (backward_lds_bytes(p.TY, p.W, sigs) + 2 * kThreads * 8 > max_lds_bytes()) return hipErrorInvalidValue;
  if (p.H <= 0 || p.Wd <= 0) return hipSuccess;
  hipError_t e;
  if (fixed_w_bwd_available(p.W, variant))
    e = launch_backward_fixed_w(p, sigs, partials, s);
  else if (p.kt == BF_BOX)
    e = launch_bwd_k<BF_BOX, false>(p, variant, partials, s);
  else
    e = sigs ? launch_bwd_k<BF_GAUSS, true>(p, variant, partials, s)
             : launch_bwd_k<BF_GAUSS, false>(p, variant, partials, s);
  if (e != hipSuccess || (!grad_sigma && !p.dyn)) return e;
  const int tiles = ((p.H + p.TY - 1) / p.TY) * p.tiles_x;
  hipLaunchKernelGGL(sigma_reduce_kernel, dim3(1), dim3(kThreads), 0, s, (const double*)partials,
                     tiles, (p.kt == BF_GAUSS && sigs) ? 1 : 0, grad_sigma, p.dyn);
  return hipGetLastError();
}

}  // namespace bfgpa

// ---------------------------------------------------------------------------
// Adjoint with the reflecting border.  With reflection every output pixel's
// window lies inside the image extended by W on each side, so the forward is
// the zero-border filter of that extension cropped back to the image.  The
// adjoint therefore runs the zero-border adjoint on the extension (output
// gradient zero outside the image) and sums the extension's gradient back
// onto the pixels each extended sample reflects.
// ---------------------------------------------------------------------------
namespace bfgpa {

// fpad: the extension by reflection (period 2n, edge samples repeated);
// gpad: the output gradient, zero outside the image.  Both (H + 2W) x (Wd + 2W), pitch Wd + 2W.
__global__ __launch_bounds__(kThreads) void mirror_pad_kernel(const float* in, int64_t in_pitch, const float* gout,
                                                              int64_t gout_pitch, int H, int Wd, int W, float* fpad,
                                                              float* gpad) {
  const int Wp = Wd + 2 * W;
  const int64_t n = (int64_t)(H + 2 * W) * Wp;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const int R = (int)(i / Wp);
    const int r = R - W, c = (int)(i - (int64_t)R * Wp) - W;
    fpad[i] = in[(int64_t)reflect_index(r, H) * in_pitch + reflect_index(c, Wd)];
    gpad[i] = (r >= 0 && r < H && c >= 0 && c < Wd) ? gout[(int64_t)r * gout_pitch + c] : 0.f;
  }
}

// first offset u >= -W of the extension with u = u0 (mod 2n)
__device__ __forceinline__ int first_image(int u0, int n, int W) { return u0 - ((u0 + W) / (2 * n)) * (2 * n); }

// gin(r, c) = sum of gpad over the extended samples (u, v) in [-W, H + W) x [-W, Wd + W)
// that reflect onto (r, c): u = r or 2H - 1 - r modulo 2H, likewise v.
__global__ __launch_bounds__(kThreads) void mirror_fold_kernel(const float* gpad, int H, int Wd, int W, float* gin,
                                                               int64_t gin_pitch) {
  const int Wp = Wd + 2 * W;
  const int64_t n = (int64_t)H * Wd;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const int r = (int)(i / Wd), c = (int)(i - (int64_t)r * Wd);
    float acc = 0.f;
    for (int a = 0; a < 2; ++a) {
      for (int u = first_image(a ? 2 * H - 1 - r : r, H, W); u < H + W; u += 2 * H) {
        const float* row = gpad + (int64_t)(u + W) * Wp + W;
        for (int b = 0; b < 2; ++b)
          for (int v = first_image(b ? 2 * Wd - 1 - c : c, Wd, W); v < Wd + W; v += 2 * Wd) acc += row[v];
      }
    }
    gin[(int64_t)r * gin_pitch + c] = acc;
  }
}

static int grid_for(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 8192));
}

hipError_t launch_mirror_pad(const float* in, int64_t in_pitch, const float* gout, int64_t gout_pitch, int H, int Wd,
                             int W, float* fpad, float* gpad, hipStream_t s) {
  const int64_t n = (int64_t)(H + 2 * W) * (Wd + 2 * W);
  hipLaunchKernelGGL(mirror_pad_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, in, in_pitch, gout, gout_pitch, H, Wd,
                     W, fpad, gpad);
  return hipGetLastError();
}

hipError_t launch_mirror_fold(const float* gpad, int H, int Wd, int W, float* gin, int64_t gin_pitch, hipStream_t s) {
  hipLaunchKernelGGL(mirror_fold_kernel, dim3(grid_for((int64_t)H * Wd)), dim3(kThreads), 0, s, gpad, H, Wd, W, gin,
                     gin_pitch);
  return hipGetLastError();
}

}  // namespace bfgpa
