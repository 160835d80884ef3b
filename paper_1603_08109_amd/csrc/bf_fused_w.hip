// The fused forward tile (forward_tile, bf_device.h) compiled for fixed
// supports W = 1 .. 21 with float64 sums, plain and keeping the adjoint's
// state.  With W a
// compile-time constant the FIR and box loops unroll completely and the taps
// stay in scalar registers across the orders; the arithmetic and its order
// are those of the generic kernel, so outputs are bit-identical.  Measured on
// 4096^2 (sigma_r = 10): box W = 10 6.45 -> 4.11 ms, Gaussian W = 9 9.32 ->
// 8.25 ms.  Each W is compiled for the tile variant the planner picks for it
// on images of at least 256 tiles: (8, 12) for W <= 4, (8, 20) for W = 5 .. 12,
// (8, 32) for W = 13 .. 21; other variants take the generic kernel.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bf_device.h"
#include "bf_internal.h"

namespace bfgpa {

// The plain forward of the smaller register shapes asks for three waves per
// SIMD (its registers then fit in 168 without spills; the form keeping the
// adjoint's state would spill there and keeps two): 4096^2, sigma_r = 30,
// Gaussian W = 9 1.81 -> 1.72 ms, box W = 10 0.93 -> 0.85 ms.
template <int KT, int OPT, int MREG, int WC, bool SAVE>
__global__ __launch_bounds__(kThreads, (!SAVE && OPT * MREG <= 160 ? 3 : OPT * MREG <= 256 ? 2 : 1)) void gpa_forward_w_kernel(TileParams p) {
  extern __shared__ float lds[];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int ty = tile / p.tiles_x;
  const int tx = tile - ty * p.tiles_x;
  forward_tile<KT, OPT, MREG, true, SAVE, WC>(p, ty * 4 * OPT, tx * kTileCols, lds);
}

// the variant compiled for support W (index into the forward variant table)
constexpr int fixed_w_variant(int W) { return W <= 4 ? 0 : W <= 12 ? 1 : 2; }

template <int KT, int WC, bool SAVE>
static hipError_t launch_w(const TileParams& p, hipStream_t s) {
  constexpr int V = fixed_w_variant(WC);
  constexpr int OPT = 8;
  constexpr int MREG = V == 0 ? 12 : V == 1 ? 20 : 32;
  auto kern = gpa_forward_w_kernel<KT, OPT, MREG, WC, SAVE>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       max_lds_bytes());
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int tiles = ((p.H + 4 * OPT - 1) / (4 * OPT)) * p.tiles_x;
  hipLaunchKernelGGL(kern, dim3(tiles), dim3(kThreads), (size_t)forward_lds_bytes(4 * OPT, WC), s, p);
  return hipGetLastError();
}

template <int KT, bool SAVE>
static hipError_t launch_w_kt(const TileParams& p, hipStream_t s) {
  switch (p.W) {
    case 1: return launch_w<KT, 1, SAVE>(p, s);
    case 2: return launch_w<KT, 2, SAVE>(p, s);
    case 3: return launch_w<KT, 3, SAVE>(p, s);
    case 4: return launch_w<KT, 4, SAVE>(p, s);
    case 5: return launch_w<KT, 5, SAVE>(p, s);
    case 6: return launch_w<KT, 6, SAVE>(p, s);
    case 7: return launch_w<KT, 7, SAVE>(p, s);
    case 8: return launch_w<KT, 8, SAVE>(p, s);
    case 9: return launch_w<KT, 9, SAVE>(p, s);
    case 10: return launch_w<KT, 10, SAVE>(p, s);
    case 11: return launch_w<KT, 11, SAVE>(p, s);
    case 12: return launch_w<KT, 12, SAVE>(p, s);
    case 13: return launch_w<KT, 13, SAVE>(p, s);
    case 14: return launch_w<KT, 14, SAVE>(p, s);
    case 15: return launch_w<KT, 15, SAVE>(p, s);
    case 16: return launch_w<KT, 16, SAVE>(p, s);
    case 17: return launch_w<KT, 17, SAVE>(p, s);
    case 18: return launch_w<KT, 18, SAVE>(p, s);
    case 19: return launch_w<KT, 19, SAVE>(p, s);
    case 20: return launch_w<KT, 20, SAVE>(p, s);
    default: return launch_w<KT, 21, SAVE>(p, s);
  }
}

bool fixed_w_available(int W, int variant) { return W >= 1 && W <= 21 && variant == fixed_w_variant(W); }

hipError_t launch_forward_fixed_w(const TileParams& p, bool save, hipStream_t s) {
  if (p.W < 1 || p.W > 21) return hipErrorInvalidValue;
  if (save) return p.kt == BF_BOX ? launch_w_kt<BF_BOX, true>(p, s) : launch_w_kt<BF_GAUSS, true>(p, s);
  return p.kt == BF_BOX ? launch_w_kt<BF_BOX, false>(p, s) : launch_w_kt<BF_GAUSS, false>(p, s);
}

}  // namespace bfgpa
