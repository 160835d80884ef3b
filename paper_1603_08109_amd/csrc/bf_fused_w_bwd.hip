// The fused adjoint tile (backward_tile, bf_device.h) compiled for fixed
// supports W = 1 .. 17 in the 16-row variant {4, 20}, the one the planner
// picks for every such support.  With W a compile-time constant the row and
// column passes unroll completely and the taps stay in scalar registers
// across the orders; the arithmetic and its order are those of the generic
// kernel, so the outputs are bit-identical.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bf_device.h"
#include "bf_internal.h"

namespace bfgpa {

constexpr int kBwdWOpt = 4, kBwdWMreg = 20, kBwdWMax = 17;

template <int KT, bool SIGS, int WC>
__global__ __launch_bounds__(kThreads, 2) void gpa_backward_w_kernel(TileParams pk, double* partials) {
  extern __shared__ float lds[];
  __shared__ double red[2 * kThreads];
  const TileParams p = with_dyn(pk);
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tyi = tile / p.tiles_x;
  const int txi = tile - tyi * p.tiles_x;
  backward_tile<KT, kBwdWOpt, kBwdWMreg, SIGS, WC>(p, tyi * p.TY, txi * kTileCols, lds, red,
                                                   partials + 2 * (int64_t)tile);
}

template <int KT, bool SIGS, int WC>
static hipError_t launch_bw(const TileParams& p, double* partials, hipStream_t s) {
  auto kern = gpa_backward_w_kernel<KT, SIGS, WC>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       max_lds_bytes() - 2 * kThreads * 8);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int tiles = ((p.H + 4 * kBwdWOpt - 1) / (4 * kBwdWOpt)) * p.tiles_x;
  hipLaunchKernelGGL(kern, dim3(tiles), dim3(kThreads), (size_t)backward_lds_bytes(4 * kBwdWOpt, WC, SIGS), s, p,
                     partials);
  return hipGetLastError();
}

template <int KT, bool SIGS>
static hipError_t launch_bw_ks(const TileParams& p, double* partials, hipStream_t s) {
  switch (p.W) {
    case 1: return launch_bw<KT, SIGS, 1>(p, partials, s);
    case 2: return launch_bw<KT, SIGS, 2>(p, partials, s);
    case 3: return launch_bw<KT, SIGS, 3>(p, partials, s);
    case 4: return launch_bw<KT, SIGS, 4>(p, partials, s);
    case 5: return launch_bw<KT, SIGS, 5>(p, partials, s);
    case 6: return launch_bw<KT, SIGS, 6>(p, partials, s);
    case 7: return launch_bw<KT, SIGS, 7>(p, partials, s);
    case 8: return launch_bw<KT, SIGS, 8>(p, partials, s);
    case 9: return launch_bw<KT, SIGS, 9>(p, partials, s);
    case 10: return launch_bw<KT, SIGS, 10>(p, partials, s);
    case 11: return launch_bw<KT, SIGS, 11>(p, partials, s);
    case 12: return launch_bw<KT, SIGS, 12>(p, partials, s);
    case 13: return launch_bw<KT, SIGS, 13>(p, partials, s);
    case 14: return launch_bw<KT, SIGS, 14>(p, partials, s);
    case 15: return launch_bw<KT, SIGS, 15>(p, partials, s);
    case 16: return launch_bw<KT, SIGS, 16>(p, partials, s);
    case 17: return launch_bw<KT, SIGS, 17>(p, partials, s);
    default: return hipErrorInvalidValue;
  }
}

bool fixed_w_bwd_available(int W, int variant) { return W >= 1 && W <= kBwdWMax && variant == 0; }

// The tile rows, grid and LDS are those launch_backward checks for variant 0.
hipError_t launch_backward_fixed_w(const TileParams& p, bool sigs, double* partials, hipStream_t s) {
  if (p.W < 1 || p.W > kBwdWMax || p.TY != 4 * kBwdWOpt) return hipErrorInvalidValue;
  if (p.kt == BF_BOX) return launch_bw_ks<BF_BOX, false>(p, partials, s);
  return sigs ? launch_bw_ks<BF_GAUSS, true>(p, partials, s) : launch_bw_ks<BF_GAUSS, false>(p, partials, s);
}

}  // namespace bfgpa
