// Device code shared by the forward, adjoint and batched kernels.
//
// One workgroup (256 threads, four wave64 waves) owns an output tile of
// 64 columns x TY rows.  The tile grown by W on every side is the region
// whose pixels enter its sums.  For every n = 0..N (Algorithm 2, Sec. 3):
//   1. each thread advances the auxiliary-image values of the region pixels
//      it owns (registers) by one power, eq. (intImg), and stores them in LDS;
//   2. the row pass filters every region row onto the 64 tile columns;
//   3. the column pass filters those onto the tile rows, giving the
//      filtered image F_bar_n of eq. (spatialFiltering) at the thread's own
//      output pixels;
//   4. the thread folds F_bar_n into its numerator / denominator sums,
//      eqs. (P), (Q).
// The auxiliary images never leave the chip.  Box rows and columns are
// summed with a prefix-difference over a register block (O(1) in W per
// output); Gaussian ones with a register-blocked FIR whose taps are
// wave-uniform scalar loads.
#pragma once

#include <hip/hip_runtime.h>

#include "bf_internal.h"

namespace bfgpa {

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so that neighbouring tiles, which read the
// same halo rows, share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nblk) {
  constexpr int nx = 8;
  const int per = nblk / nx, rem = nblk % nx;
  const int xcd = b % nx, k = b / nx;
  return xcd * per + min(xcd, rem) + k;
}

__device__ __forceinline__ int align4(int n) { return (n + 3) & ~3; }

// ---------------------------------------------------------------------------
// Row pass: region rows (RH of them, pitch RWp) -> Hs rows (pitch kHPitch),
// 64 outputs per row.  Output column c sums region columns c .. c + 2W.
// ---------------------------------------------------------------------------

// Box: each work item covers S consecutive outputs of one row.  With the
// running prefix s(k) = sum of the first k region values of the segment,
// out[j] = s(j + 2W + 1) - s(j); s(j) for j < S is kept in registers and the
// leading prefix advances one value per output.
template <int S>
__device__ __forceinline__ void rowpass_box(const float* __restrict__ Fs, int RWp,
                                            float* __restrict__ Hs, int RH, int W) {
  constexpr int nseg = kTileCols / S;
  const int L = 2 * W + 1;
  const int items = RH * nseg;
  for (int it = threadIdx.x; it < items; it += kThreads) {
    const int seg = it / RH;
    const int r = it - seg * RH;
    const float* row = Fs + r * RWp + seg * S;
    float start[S];
    float acc = 0.f;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      start[s] = acc;
      acc += row[s];
    }
    float lead;
    if (L >= S) {
      lead = acc;
      for (int k = S; k < L; ++k) lead += row[k];
    } else {
      lead = 0.f;
      for (int k = 0; k < L; ++k) lead += row[k];
    }
    float* h = Hs + r * kHPitch + seg * S;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      h[s] = lead - start[s];
      if (s + 1 < S) lead += row[L + s];
    }
  }
}

// Gaussian: out[j] = sum_d tap[d] F[j + d]; loop over the inputs of the
// segment, each contributing to all S register accumulators.  tz points at
// the tap array with kTapPad zeros in front, so tz[k - s] is tap[k - s] or
// zero outside [0, 2W].
template <int S>
__device__ __forceinline__ void rowpass_fir(const float* __restrict__ Fs, int RWp,
                                            float* __restrict__ Hs, int RH, int W,
                                            const float* __restrict__ tz) {
  constexpr int nseg = kTileCols / S;
  const int L = 2 * W + 1;
  const int items = RH * nseg;
  for (int it = threadIdx.x; it < items; it += kThreads) {
    const int seg = it / RH;
    const int r = it - seg * RH;
    const float* row = Fs + r * RWp + seg * S;
    float acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = 0.f;
    const int K = L + S - 1;
    for (int k = 0; k < K; ++k) {
      const float v = row[k];
#pragma unroll
      for (int s = 0; s < S; ++s) acc[s] = fmaf(tz[k - s], v, acc[s]);
    }
    float* h = Hs + r * kHPitch + seg * S;
#pragma unroll
    for (int s = 0; s < S; ++s) h[s] = acc[s];
  }
}

// ---------------------------------------------------------------------------
// Column pass: the thread owns column `lane` of the tile and output rows
// orow0 .. orow0 + opt - 1 (opt <= OPT); it reads Hs rows orow0 .. orow0 +
// opt - 1 + 2W and writes its opt filtered values to v[].
// ---------------------------------------------------------------------------
template <int OPT>
__device__ __forceinline__ void colpass_box(const float* __restrict__ Hs, int orow0, int lane,
                                            int opt, int W, float (&v)[OPT]) {
  const float* col = Hs + orow0 * kHPitch + lane;
  const int L = 2 * W + 1;
  float start[OPT];
  float acc = 0.f;
#pragma unroll
  for (int s = 0; s < OPT; ++s) {
    if (s < opt) {
      start[s] = acc;
      acc += col[s * kHPitch];
    }
  }
  float lead;
  if (L >= opt) {
    lead = acc;
    for (int k = opt; k < L; ++k) lead += col[k * kHPitch];
  } else {
    lead = 0.f;
    for (int k = 0; k < L; ++k) lead += col[k * kHPitch];
  }
#pragma unroll
  for (int s = 0; s < OPT; ++s) {
    if (s < opt) {
      v[s] = lead - start[s];
      if (s + 1 < opt) lead += col[(L + s) * kHPitch];
    }
  }
}

template <int OPT>
__device__ __forceinline__ void colpass_fir(const float* __restrict__ Hs, int orow0, int lane,
                                            int opt, int W, const float* __restrict__ tz,
                                            float (&v)[OPT]) {
  const float* col = Hs + orow0 * kHPitch + lane;
  const int L = 2 * W + 1;
#pragma unroll
  for (int s = 0; s < OPT; ++s) v[s] = 0.f;
  const int K = L + opt - 1;
  for (int k = 0; k < K; ++k) {
    const float x = col[k * kHPitch];
#pragma unroll
    for (int s = 0; s < OPT; ++s) v[s] = fmaf(tz[k - s], x, v[s]);
  }
}

// Row S for the box (prefix trick) and for the FIR (register block).
constexpr int kRowSegBox = 16;
constexpr int kRowSegFir = 8;

template <int KT>
__device__ __forceinline__ void rowpass(const float* Fs, int RWp, float* Hs, int RH, int W,
                                        const float* tz) {
  if (KT == BF_BOX)
    rowpass_box<kRowSegBox>(Fs, RWp, Hs, RH, W);
  else
    rowpass_fir<kRowSegFir>(Fs, RWp, Hs, RH, W, tz);
}

template <int KT, int OPT>
__device__ __forceinline__ void colpass(const float* Hs, int orow0, int lane, int opt, int W,
                                        const float* tz, float (&v)[OPT]) {
  if (KT == BF_BOX)
    colpass_box<OPT>(Hs, orow0, lane, opt, W, v);
  else
    colpass_fir<OPT>(Hs, orow0, lane, opt, W, tz, v);
}

// ---------------------------------------------------------------------------
// Region set-up: the thread owns region pixels q = t + 256 m (row-major over
// the padded region, pitch RWp).  x = (f - center) / sigma_r, F~_0 = e^{-x^2/2};
// pixels outside the image (and the pad column) hold x = F = 0 and so never
// contribute (zero extension).
// ---------------------------------------------------------------------------
struct RegionGeom {
  int RH, RW, RWp, npx;
};

__device__ __forceinline__ RegionGeom region_geom(int TY, int W) {
  RegionGeom g;
  g.RH = TY + 2 * W;
  g.RW = kTileCols + 2 * W;
  g.RWp = g.RW | 1;
  g.npx = g.RH * g.RWp;
  return g;
}

// Visit the thread's region pixels: fn(m, q, inside, gr, gc).
template <int MREG, typename Fn>
__device__ __forceinline__ void for_region(const RegionGeom& g, int r0, int c0, int W, int H,
                                           int Wd, Fn&& fn) {
  const int t = threadIdx.x;
  int row = t / g.RWp, col = t - row * g.RWp;
  const int srow = kThreads / g.RWp, scol = kThreads - srow * g.RWp;
#pragma unroll
  for (int m = 0; m < MREG; ++m) {
    const int q = t + kThreads * m;
    const int gr = r0 - W + row, gc = c0 - W + col;
    const bool inside = q < g.npx && col < g.RW && gr >= 0 && gr < H && gc >= 0 && gc < Wd;
    fn(m, q, inside, gr, gc);
    col += scol;
    row += srow;
    if (col >= g.RWp) {
      col -= g.RWp;
      ++row;
    }
  }
}

// ---------------------------------------------------------------------------
// Fused forward tile body (Algorithm 2 with the range-safe scaling).
// ---------------------------------------------------------------------------
template <typename Acc>
struct AccOps;
template <>
struct AccOps<double> {
  static __device__ __forceinline__ double fma_(float a, float b, double c) {
    return fma((double)a, (double)b, c);
  }
};
template <>
struct AccOps<float> {
  static __device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
};

template <int KT, int OPT, int MREG, typename Acc, bool SAVE>
__device__ __forceinline__ void forward_tile(const TileParams& p, int r0, int c0, float* lds) {
  const int W = p.W;
  const int N = p.N;
  const RegionGeom g = region_geom(p.TY, W);
  float* Fs = lds;
  float* Hs = lds + align4(g.npx);
  const float* tz = p.taps + kTapPad;

  float Fr[MREG], xr[MREG];
  for_region<MREG>(g, r0, c0, W, p.H, p.Wd, [&](int m, int q, bool inside, int gr, int gc) {
    float x = 0.f, F = 0.f;
    if (inside) {
      const float f = p.in[(int64_t)gr * p.in_pitch + gc];
      x = (f - p.center) / p.sigma_r;
      F = expf(-0.5f * x * x);
    }
    Fr[m] = F;
    xr[m] = x;
  });

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int opt = p.TY >> 2;
  const int orow0 = wv * opt;
  const int gc = c0 + lane;
  float xo[OPT], ao[OPT], bo[OPT], bp[OPT];
  Acc P[OPT], Q[OPT], DP[OPT], DQ[OPT];
#pragma unroll
  for (int s = 0; s < OPT; ++s) {
    const int gr = r0 + orow0 + s;
    float x = 0.f;
    if (s < opt && gr < p.H && gc < p.Wd) x = (p.in[(int64_t)gr * p.in_pitch + gc] - p.center) / p.sigma_r;
    xo[s] = x;
    ao[s] = expf(-0.5f * x * x);  // a_0 = e^{-x^2/2} M_0 / 0!
    bo[s] = 0.f;                  // b_n = a_{n-1} r_n (none at n = 0)
    bp[s] = 0.f;
    P[s] = Q[s] = DP[s] = DQ[s] = Acc(0);
  }

  for (int n = 0; n <= N; ++n) {
    const float sn = p.s_tab[n];
#pragma unroll
    for (int m = 0; m < MREG; ++m) {
      if (n > 0) Fr[m] *= xr[m] * sn;  // F~_n = F~_{n-1} x / r_n
      const int q = threadIdx.x + kThreads * m;
      if (q < g.npx) Fs[q] = Fr[m];
    }
    __syncthreads();
    rowpass<KT>(Fs, g.RWp, Hs, g.RH, W, tz);
    __syncthreads();
    float v[OPT];
    colpass<KT, OPT>(Hs, orow0, lane, opt, W, tz, v);
    const float rn = p.r_tab[n];
    const float rn1 = p.r_tab[n + 1];
    const float in1 = p.inv_tab[n + 1];
#pragma unroll
    for (int s = 0; s < OPT; ++s) {
      if (n >= 1) P[s] = AccOps<Acc>::fma_(bo[s], v[s], P[s]);  // eq. (P): F_bar_{n} term
      if (n < N) Q[s] = AccOps<Acc>::fma_(ao[s], v[s], Q[s]);   // eq. (Q): F_bar_{n} term
      if (SAVE) {
        if (n >= 1 && n < N) DQ[s] = AccOps<Acc>::fma_(bo[s], v[s], DQ[s]);
        if (n >= 2) DP[s] = AccOps<Acc>::fma_(bp[s] * rn, v[s], DP[s]);
        bp[s] = bo[s];
      }
      const float bn = ao[s] * rn1;  // b_{n+1} = a_n r_{n+1}
      ao[s] = bn * (xo[s] * in1);    // a_{n+1} = b_{n+1} x / (n+1)
      bo[s] = bn;
    }
  }

#pragma unroll
  for (int s = 0; s < OPT; ++s) {
    const int gr = r0 + orow0 + s;
    if (s < opt && gr < p.H && gc < p.Wd) {
      const double ratio = (double)P[s] / (double)Q[s];
      if (p.out) p.out[(int64_t)gr * p.out_pitch + gc] = (float)((double)p.sigma_r * ratio + (double)p.center);
      if (SAVE && p.saved) {
        const int64_t idx = (int64_t)gr * p.Wd + gc;
        p.saved[idx] = (float)Q[s];
        p.saved[p.saved_plane + idx] = (float)ratio;
        p.saved[2 * p.saved_plane + idx] = (float)((double)DP[s] - ratio * (double)DQ[s]);
      }
    }
  }
}

}  // namespace bfgpa
