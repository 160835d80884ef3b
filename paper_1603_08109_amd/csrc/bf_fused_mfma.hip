// Fused Gaussian tile on the matrix cores: Algorithm 2 for one 64 x 64 output
// tile with the whole (64 + 2W)^2 region of the auxiliary images resident in
// LDS, both passes of the separable FIR as banded Toeplitz products
// (bf_toeplitz.h), and no trip through device memory between orders.
//
// Per order n (two barriers):
//   row pass   region rows (16-row blocks) x 64 output columns -> Hs, eight
//              waves taking (row block, column half) units;
//   column pass 64 x 64 outputs from Hs (Toeplitz table as A), wave w a
//              16 x 32 block, folded into eqs. (P), (Q) of its 8 pixels;
//   powers     F^_{n+1} = F^_n y in place (each thread owns fixed LDS slots
//              and keeps their y in registers).
// Region slots outside the image are zero (zero extension) or, with the
// mirror border, hold the reflected pixels.  Same range-safe scaling and
// float64 sums as the other paths.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "bf_device.h"
#include "bf_internal.h"
#include "bf_toeplitz.h"

namespace bfgpa {

constexpr int kFmThreads = 512;  // eight waves
constexpr int kFmHs = 80;        // row pitch of the row-pass output (4 rows on distinct bank groups)
constexpr int kFmRegs = 50;      // region slots per thread: Rp * RWp <= 50 * 512 (W <= 45)

struct FmGeom {
  int R;    // region rows and columns: 64 + 2W
  int Rp;   // rows kept in LDS: the column pass's last k-step reads row 66 + 2W
  int RWp;  // row pitch: the row pass's last k-step reads column 66 + 2W
  int KK;   // k-steps per 16x16 block
};

__host__ __device__ inline FmGeom fm_geom(int W) {
  FmGeom g;
  g.R = 64 + 2 * W;
  g.Rp = (67 + 2 * W + 15) & ~15;
  const int need = 68 + 2 * W;
  g.RWp = (need % 4 == 2) ? need : need + 2;
  g.KK = ls_kk(W);
  return g;
}

int64_t fused_mfma_lds_bytes(int W) {
  const FmGeom g = fm_geom(W);
  return 4 * ((int64_t)g.Rp * g.RWp + (int64_t)g.Rp * kFmHs + (int64_t)g.KK * 64);
}

bool fused_mfma_supported(int W) {
  const FmGeom g = fm_geom(W);
  return (int64_t)g.Rp * g.RWp <= (int64_t)kFmRegs * kFmThreads && fused_mfma_lds_bytes(W) <= max_lds_bytes();
}

template <bool SAVE>
__global__ __launch_bounds__(kFmThreads) void gpa_fused_mfma_kernel(TileParams p) {
  extern __shared__ float lds[];
  const int W = p.W, N = p.N;
  const FmGeom g = fm_geom(W);
  float* Fs = lds;                     // Rp x RWp region of F^_n
  float* Hs = Fs + g.Rp * g.RWp;       // Rp x kFmHs row-pass output
  float* Tt = Hs + g.Rp * kFmHs;       // Toeplitz table
  const int tiles_x = (p.Wd + 63) / 64;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int ty = tile / tiles_x, tx = tile - (tile / tiles_x) * tiles_x;
  const int r0 = ty * 64, c0 = tx * 64;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  fill_toeplitz<kFmThreads>(Tt, W, p.taps + kTapPad);

  // region: slot q = threadIdx.x + 512 j at (q / RWp, q % RWp)
  const int nslot = g.Rp * g.RWp;
  float Y[kFmRegs];
#pragma unroll
  for (int j = 0; j < kFmRegs; ++j) {
    const int q = threadIdx.x + j * kFmThreads;
    const int row = q / g.RWp, col = q - (q / g.RWp) * g.RWp;
    int gr = r0 - W + row, gc = c0 - W + col;
    bool inside = q < nslot && row < g.R && col < g.R;
    if (p.mirror) {
      gr = reflect_index(gr, p.H);
      gc = reflect_index(gc, p.Wd);
    } else {
      inside = inside && gr >= 0 && gr < p.H && gc >= 0 && gc < p.Wd;
    }
    float f = 0.f;
    if (inside) f = p.in[(int64_t)gr * p.in_pitch + gc];
    const float x = (f - p.center) / p.sigma_r;
    Y[j] = inside ? (f - p.center) * p.inv_T : 0.f;
    if (q < nslot) Fs[q] = inside ? expf(-0.5f * x * x) : 0.f;
  }

  // this lane's 8 pixels: block j (columns 32 ch + 16 j), accumulator v (row 16 rb + 4(l/16) + v)
  const int rb = wv & 3, ch = wv >> 2;
  const int pr0 = r0 + rb * 16 + 4 * (lane >> 4);
  const int pc0 = c0 + ch * 32 + (lane & 15);
  LsPix<8, SAVE> px;
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int s = 4 * j + v;
      const float f = p.in[(int64_t)min(pr0 + v, p.H - 1) * p.in_pitch + min(pc0 + 16 * j, p.Wd - 1)];
      const float x = (f - p.center) / p.sigma_r;  // pixels past the image: harmless, never stored
      px.z[s] = x * p.X;
      px.a[s] = expf(-0.5f * x * x);
      px.ap[s] = 0.f;
      px.app[s] = 0.f;
      px.P[s] = 0.0;
      px.Q[s] = 0.0;
      px.DP[s] = 0.0;
      px.DQ[s] = 0.0;
    }
  __syncthreads();

  const int nunits = 2 * (g.Rp / 16);
  for (int n = 0; n <= N; ++n) {
    // row pass: (16-row block, column half) units
    for (int u = wv; u < nunits; u += kFmThreads / 64) {
      const int ub = u >> 1, half = u & 1;
      mf4 acc[2];
#pragma unroll
      for (int bb = 0; bb < 2; ++bb) acc[bb] = mf4{0.f, 0.f, 0.f, 0.f};
      toeplitz_rows<2>(Fs + ub * 16 * g.RWp, g.RWp, half * 32, Tt, g.KK, acc);
#pragma unroll
      for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          Hs[(ub * 16 + 4 * (lane >> 4) + v) * kFmHs + half * 32 + bb * 16 + (lane & 15)] = acc[bb][v];
    }
    __syncthreads();
    // column pass and fold
    mf4 ca[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) ca[j] = mf4{0.f, 0.f, 0.f, 0.f};
    toeplitz_cols<2>(Hs, rb * 16, ch * 32, Tt, g.KK, ca, kFmHs);
    const float in1 = p.inv_tab[n + 1];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) px.fold(4 * j + v, n, N, ca[j][v], in1);
    // powers (the row pass has read this order's F^ before the barrier above)
    if (n < N) {
#pragma unroll
      for (int j = 0; j < kFmRegs; ++j) {
        const int q = threadIdx.x + j * kFmThreads;
        if (q < nslot) Fs[q] *= Y[j];
      }
    }
    __syncthreads();
  }

  const double X = (double)p.X;
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int s = 4 * j + v;
      const int r = pr0 + v, c = pc0 + 16 * j;
      if (r < p.H && c < p.Wd) {
        const double q = px.Q[s];
        const double ratio = X * px.P[s] / q;
        if (p.out) p.out[(int64_t)r * p.out_pitch + c] = (float)((double)p.sigma_r * ratio + (double)p.center);
        if (SAVE && p.saved) {
          const int64_t idx = (int64_t)r * p.Wd + c;
          p.saved[idx] = (float)q;
          p.saved[p.saved_plane + idx] = (float)ratio;
          p.saved[2 * p.saved_plane + idx] = (float)(X * X * px.DP[s] - ratio * X * px.DQ[s]);
        }
      }
    }
}

hipError_t launch_fused_mfma(const TileParams& p, bool save, hipStream_t s) {
  if (p.kt != BF_GAUSS || !fused_mfma_supported(p.W)) return hipErrorInvalidValue;
  if (p.H <= 0 || p.Wd <= 0) return hipSuccess;
  auto k = save ? gpa_fused_mfma_kernel<true> : gpa_fused_mfma_kernel<false>;
  static bool attr_set[2] = {false, false};
  if (!attr_set[save]) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
    if (e != hipSuccess) return e;
    attr_set[save] = true;
  }
  const int tiles = ((p.H + 63) / 64) * ((p.Wd + 63) / 64);
  hipLaunchKernelGGL(k, dim3(tiles), dim3(kFmThreads), (size_t)fused_mfma_lds_bytes(p.W), s, p);
  return hipGetLastError();
}

}  // namespace bfgpa
