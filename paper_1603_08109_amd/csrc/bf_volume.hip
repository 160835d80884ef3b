// Video and volume data (the extension Sec. 1 and Sec. 5 name): D slices of
// Hs x Wd, kernel w1 x w1 x w1 on the cube [-W, W]^3, zero extension or (with
// p.mirror) reflection about every face, edge samples repeated.
// Algorithm 2 is unchanged; only the spatial filtering runs over three axes.
//
// The slices are stacked as one image of D Hs rows (voxel (d, r, c) at row
// d Hs + r), so the lift, the row pass of each block of 16 orders and
// eq. (PbyQ) are the streamed image kernels as they are.  Per block:
//   vol_cols  : the column FIR inside each slice (taps that would cross a
//               slice boundary are dropped), 64 x 64 tiles staged in LDS,
//               writing the row- and column-filtered volume of each order;
//   vol_depth : the FIR across slices at each (r, c), folded into the
//               float64 sums of eqs. (P), (Q) of kVolDepth voxels per thread.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <type_traits>

#include "bf_device.h"
#include "bf_internal.h"
#include "bf_toeplitz.h"

namespace bfgpa {

constexpr int kVolTile = 64;   // rows and columns of a column-pass tile
constexpr int kVolDepth = 8;   // voxels per thread along the depth axis

// Column FIR inside each slice for orders n0 .. n0 + K - 1.  Thread: column
// c = tid % 64 of the tile, output rows 16 (tid / 64) .. + 15.
__global__ __launch_bounds__(256) void vol_cols_kernel(TileParams p, LsState st, VolBufs g, int K, int Hs) {
  extern __shared__ float lds[];
  const int W = p.W;
  const int rows = kVolTile + 2 * W;
  const int tiles_x = (p.Wd + kVolTile - 1) / kVolTile;
  const int ty = blockIdx.x / tiles_x, tx = blockIdx.x - (blockIdx.x / tiles_x) * tiles_x;
  const int R0 = ty * kVolTile, c0 = tx * kVolTile;
  const int c = threadIdx.x & 63;
  const int rg = threadIdx.x >> 6;
  const float* tz = p.taps + kTapPad;  // tz[a + W] = w1(a)
  // the first row of the slice that holds this thread's first output row (its
  // rows advance one at a time, so each step starts the next slice at most once)
  const int Rt = R0 + 16 * rg;
  const int dfirst = (Rt / Hs) * Hs;
  for (int k = 0; k < K; ++k) {
    __syncthreads();  // the previous order's reads are done
    // stage rows R0 - W .. R0 + 63 + W (row-filtered images carry W zero rows
    // above; padded row R0 + i is stacked row R0 - W + i), rounded up to whole
    // groups of four by direct-to-LDS loads (the zero rows below cover them;
    // columns past the image are never written by the row pass and stay zero)
    stage_rows_lds<256>(st.h(k) + (int64_t)R0 * st.pitch + c0, st.pitch, lds, (rows + 3) & ~3);
    __syncthreads();
    float* Gk = g.G[k];
    int dcur = dfirst;
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
      const int R = Rt + j;  // stacked row
      if (R >= dcur + Hs) dcur += Hs;
      if (R >= p.H || c0 + c >= p.Wd) continue;
      const int d0 = dcur;  // first row of this slice
      float acc = 0.f;
      if (p.mirror) {
        // reflected rows stay in this slice and within W of R: inside the staged window
        const float* base = lds + (d0 - R0 + W) * kVolTile + c;
        for (int a = -W; a <= W; ++a) acc += tz[a + W] * base[reflect_index(R - d0 + a, Hs) * kVolTile];
      } else {
        const int lo = max(-W, d0 - R), hi = min(W, d0 + Hs - 1 - R);
        const float* col = lds + (R - R0 + W) * kVolTile + c;
        for (int a = lo; a <= hi; ++a) acc += tz[a + W] * col[a * kVolTile];
      }
      Gk[(int64_t)R * p.Wd + c0 + c] = acc;
    }
  }
}

// FIR across slices and the fold into eqs. (P), (Q): thread q of the slice
// plane, voxels at depths d0 .. d0 + kVolDepth - 1.
// WIDE: the wide-range float64 states (see ls_rows_x3_kernel), folded without the X of eq. (P)
// WC > 0: the support W = WC with zero extension, compiled as a constant: the
// kVolDepth + 2W samples of the thread's column are loaded once per order
// into registers (zeros outside the volume) and every output sums its 2W + 1
// of them in the same order as the runtime-W loop, so the sums are the same.
template <bool WIDE, int WC = 0>
__global__ __launch_bounds__(256) void vol_depth_kernel(TileParams p, LsState st, VolBufs g, int n0, int K, int Hs,
                                                        int D) {
  const int64_t plane = (int64_t)Hs * p.Wd;
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int d0 = blockIdx.y * kVolDepth;
  const bool live = q < plane;
  const int nok = live ? std::min(kVolDepth, D - d0) : 0;
  const int W = p.W;
  const float* tz = p.taps + kTapPad;
  typename std::conditional<WIDE, WidePix<kVolDepth>, LsPix<kVolDepth, false>>::type px;
  const int64_t i0 = (int64_t)d0 * plane + (live ? q : 0);
  px.load(st, i0, plane, nok, n0 == 0);
  for (int k = 0; k < K; ++k) {
    const float* Gk = g.G[k] + (live ? q : 0);
    const int n = n0 + k;
    const float in1 = p.inv_tab[n + 1];
    const double g1 = WIDE ? p.isq[n + 1] : 0.0, sn = WIDE ? p.sq[n] : 0.0;
    if constexpr (WC > 0) {
      float win[kVolDepth + 2 * WC];
#pragma unroll
      for (int i = 0; i < kVolDepth + 2 * WC; ++i) {
        const int d = d0 - WC + i;
        win[i] = (live && d >= 0 && d < D) ? Gk[(int64_t)d * plane] : 0.f;
      }
#pragma unroll
      for (int t = 0; t < kVolDepth; ++t) {
        float acc = 0.f;
#pragma unroll
        for (int a = 0; a <= 2 * WC; ++a) acc += tz[a] * win[t + a];
        if constexpr (WIDE)
          px.fold(t, n, p.N, acc, g1, sn);
        else
          px.fold(t, n, p.N, acc, in1);
      }
      continue;
    }
#pragma unroll
    for (int t = 0; t < kVolDepth; ++t) {
      const int d = d0 + t;
      float acc = 0.f;
      if (t < nok) {
        if (p.mirror) {
          for (int a = -W; a <= W; ++a) acc += tz[a + W] * Gk[(int64_t)reflect_index(d + a, D) * plane];
        } else {
          const int lo = max(-W, -d), hi = min(W, D - 1 - d);
          for (int a = lo; a <= hi; ++a) acc += tz[a + W] * Gk[(int64_t)(d + a) * plane];
        }
      }
      if constexpr (WIDE)
        px.fold(t, n, p.N, acc, g1, sn);
      else
        px.fold(t, n, p.N, acc, in1);
    }
  }
  px.store(st, i0, plane, nok);
}

int64_t vol_state_bytes(int D, int Hs, int Wd, int W, bool wide) {
  const int64_t H = (int64_t)D * Hs;
  return ls_state_bytes((int)H, Wd, W, false, wide) + kLsBlockSmall * (H * Wd * 4 + 256);
}

LsState vol_layout(void* base, int D, int Hs, int Wd, int W, VolBufs* g, bool wide) {
  const int H = D * Hs;
  LsState st = ls_layout(base, H, Wd, W, false, wide);
  char* q = (char*)base + ls_state_bytes(H, Wd, W, false, wide);
  for (int k = 0; k < kLsBlockSmall; ++k) {
    g->G[k] = (float*)q;
    q += ((int64_t)H * Wd * 4 + 255) & ~255LL;
  }
  return st;
}

template <bool WIDE>
static hipError_t launch_vol_depth_w(const TileParams& p, const LsState& st, const VolBufs& g, int n0, int K,
                                     int Hs, int D, dim3 grid, hipStream_t s) {
  if (!p.mirror) {
    switch (p.W) {
#define BF_VD_CASE(w) \
  case w: hipLaunchKernelGGL((vol_depth_kernel<WIDE, w>), grid, dim3(256), 0, s, p, st, g, n0, K, Hs, D); return hipSuccess;
      BF_VD_CASE(1) BF_VD_CASE(2) BF_VD_CASE(3) BF_VD_CASE(4) BF_VD_CASE(5) BF_VD_CASE(6) BF_VD_CASE(7) BF_VD_CASE(8)
#undef BF_VD_CASE
      default: break;
    }
  }
  hipLaunchKernelGGL((vol_depth_kernel<WIDE, 0>), grid, dim3(256), 0, s, p, st, g, n0, K, Hs, D);
  return hipSuccess;
}

// the depth pass: compiled for W = 1 .. 8 with zero extension, else the runtime-W loop
static hipError_t launch_vol_depth(const TileParams& p, const LsState& st, const VolBufs& g, int n0, int K, int Hs,
                                   int D, dim3 grid, hipStream_t s) {
  return p.wide ? launch_vol_depth_w<true>(p, st, g, n0, K, Hs, D, grid, s)
                : launch_vol_depth_w<false>(p, st, g, n0, K, Hs, D, grid, s);
}

hipError_t launch_forward_vol(const TileParams& p, const LsState& st, const VolBufs& g, int D, int Hs,
                              hipStream_t s) {
  if (p.H <= 0 || p.Wd <= 0) return hipSuccess;
  if (p.W > kVolMaxW || p.H != D * Hs) return hipErrorInvalidValue;
  if (p.wide && (p.kt != BF_GAUSS || !st.Fd[0])) return hipErrorInvalidValue;
  hipError_t e = p.wide ? wide_launch_init(p, st, s) : ls_launch_init(p, st, s);
  if (e != hipSuccess) return e;
  const int tiles = ((p.H + kVolTile - 1) / kVolTile) * ((p.Wd + kVolTile - 1) / kVolTile);
  const size_t clds = (size_t)((kVolTile + 2 * p.W + 3) & ~3) * kVolTile * 4;
  const dim3 gdep((unsigned)((int64_t)Hs * p.Wd + 255) / 256, (D + kVolDepth - 1) / kVolDepth);
  int src = 0;
  for (int n0 = 0; n0 <= p.N; n0 += kLsBlockSmall) {
    const int K = std::min(kLsBlockSmall, p.N + 1 - n0);
    e = p.wide ? launch_rows_x3_wide(p, st, n0, K, src, s) : ls_launch_rows(p, st, n0, K, src, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(vol_cols_kernel, dim3(tiles), dim3(256), clds, s, p, st, g, K, Hs);
    e = launch_vol_depth(p, st, g, n0, K, Hs, D, gdep, s);
    if (e != hipSuccess) return e;
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    src ^= 1;
  }
  return ls_launch_final(p, st, s);
}

}  // namespace bfgpa
