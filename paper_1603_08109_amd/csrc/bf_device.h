// Device code shared by the forward, adjoint and batched kernels.
//
// One workgroup (256 threads, four wave64 waves) owns an output tile of
// 64 columns x TY rows (TY = 4 * OPT: each wave owns OPT consecutive rows,
// lane = column).  The tile grown by W on every side is the region whose
// pixels enter its sums.  For every n = 0..N (Algorithm 2, Sec. 3):
//   1. the row pass filters every region row onto the 64 tile columns
//      (region values in LDS -> row-pass buffer in LDS);
//   2. each thread advances the auxiliary-image values of the region pixels
//      it owns (registers) by one power, eq. (intImg), and stores them for
//      the next n;
//   3. the column pass filters the row-pass buffer onto the thread's OPT
//      output pixels, giving F_bar_n of eq. (spatialFiltering) there;
//   4. the thread folds F_bar_n into its numerator / denominator sums,
//      eqs. (P), (Q).
// The auxiliary images never leave the chip.  Box rows and columns are
// summed with a prefix-difference over a register block (O(1) in W per
// output); Gaussian ones with a register-blocked FIR whose taps are
// wave-uniform scalar loads.  Runtime-length loops are unrolled by four so
// that several LDS reads are in flight per wait.
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

// The adjoint kernels' parameters with the call's image pointers (and the
// sigma-gradient destination) taken from the device copy p.dyn when set: a
// launch recorded once into a graph then reads each call's pointers.
__device__ __forceinline__ TileParams with_dyn(const TileParams& p) {
  TileParams q = p;
  if (p.dyn) {
    const TileParams& d = *p.dyn;
    q.in = d.in;
    q.in_pitch = d.in_pitch;
    q.gout = d.gout;
    q.gout_pitch = d.gout_pitch;
    q.out = d.out;
    q.out_pitch = d.out_pitch;
    q.saved = d.saved;
    q.gsig = d.gsig;
  }
  return q;
}

// Workgroup barrier that orders LDS accesses only: global loads and stores
// issued before it stay in flight (a full __syncthreads waits for them).
// For kernels whose waves exchange data through LDS alone.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum of p[k * STRIDE] for k in [k0, k1), four loads in flight per step.
__device__ __forceinline__ float strided_sum(const float* __restrict__ p, int STRIDE, int k0, int k1) {
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  int k = k0;
  for (; k + 4 <= k1; k += 4) {
    a0 += p[k * STRIDE];
    a1 += p[(k + 1) * STRIDE];
    a2 += p[(k + 2) * STRIDE];
    a3 += p[(k + 3) * STRIDE];
  }
  for (; k < k1; ++k) a0 += p[k * STRIDE];
  return (a0 + a1) + (a2 + a3);
}

// ---------------------------------------------------------------------------
// 1-D box and FIR over a strided LDS vector.  `src` points at the first
// input; output j (0 <= j < S) sums inputs j .. j + 2W (weights tz[0..2W]).
// ---------------------------------------------------------------------------

// Box: with s(k) the sum of the first k inputs, out[j] = s(j + L) - s(j),
// L = 2W + 1.  s(j) for j < S comes from the first S inputs (registers);
// the leading sum s(j + L) advances by one input per output.
template <int S>
__device__ __forceinline__ void box1d(const float* __restrict__ src, int STRIDE, int L, float (&out)[S]) {
  float a[S], b[S];
#pragma unroll
  for (int s = 0; s < S; ++s) a[s] = src[s * STRIDE];
#pragma unroll
  for (int s = 0; s < S - 1; ++s) b[s] = src[(L + s) * STRIDE];
  float start[S];
  float acc = 0.f;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    start[s] = acc;
    acc += a[s];
  }
  float lead = (L >= S) ? acc + strided_sum(src, STRIDE, S, L) : strided_sum(src, STRIDE, 0, L);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    out[s] = lead - start[s];
    if (s + 1 < S) lead += b[s];
  }
}

// FIR: out[j] = sum_k tz[k - j] src[k], k = 0 .. S + 2W - 1, tz zero outside
// [0, 2W].  Input k feeds outputs max(0, k - 2W) .. min(S - 1, k): the first
// and last S - 1 inputs (compile-time loops) touch only the accumulators
// whose taps are non-zero, the middle ones (runtime loop, unrolled by four)
// touch all S, so exactly S (2W + 1) multiply-adds are issued.  For L < S - 1
// the padded form (zero taps kTapPad deep) is used.
template <int S>
__device__ __forceinline__ void fir1d(const float* __restrict__ src, int STRIDE, int L,
                                      const float* __restrict__ tz, float (&out)[S]) {
  constexpr int U = 4;
#pragma unroll
  for (int s = 0; s < S; ++s) out[s] = 0.f;
  if (L >= S - 1) {
#pragma unroll
    for (int k = 0; k < S - 1; ++k) {  // head
      const float v = src[k * STRIDE];
#pragma unroll
      for (int s = 0; s <= k; ++s) out[s] = fmaf(tz[k - s], v, out[s]);
    }
    int k = S - 1;
    for (; k + U <= L; k += U) {  // body
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = src[(k + u) * STRIDE];
      float tw[S + U - 1];
#pragma unroll
      for (int i = 0; i < S + U - 1; ++i) tw[i] = tz[k - (S - 1) + i];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int s = 0; s < S; ++s) out[s] = fmaf(tw[u - s + S - 1], v[u], out[s]);
    }
    for (; k < L; ++k) {
      const float v = src[k * STRIDE];
#pragma unroll
      for (int s = 0; s < S; ++s) out[s] = fmaf(tz[k - s], v, out[s]);
    }
    const float* tl = tz + L;
#pragma unroll
    for (int j = 0; j < S - 1; ++j) {  // tail: input L + j feeds outputs j+1 .. S-1
      const float v = src[(L + j) * STRIDE];
#pragma unroll
      for (int s = j + 1; s < S; ++s) out[s] = fmaf(tl[j - s], v, out[s]);
    }
  } else {
    const int K = L + S - 1;
    for (int k = 0; k < K; ++k) {
      const float v = src[k * STRIDE];
#pragma unroll
      for (int s = 0; s < S; ++s) out[s] = fmaf(tz[k - s], v, out[s]);
    }
  }
}

// ---------------------------------------------------------------------------
// Row pass: region rows (RH of them, pitch RWp) -> Hs rows (pitch kHPitch),
// 64 outputs per row.  Output column c sums region columns c .. c + 2W.
// Work items are (row, segment of S outputs); consecutive lanes take
// consecutive rows, so with the odd pitches every LDS access is conflict-free.
// ---------------------------------------------------------------------------
constexpr int kRowSegBox = kRowSegBoxHost;
constexpr int kRowSegFir = kRowSegFirHost;

template <int KT, int HP = kHPitch>
__device__ __forceinline__ void rowpass(const float* __restrict__ Fs, int RWp, float* __restrict__ Hs,
                                        int RH, int W, const float* __restrict__ tz) {
  constexpr int S = (KT == BF_BOX) ? kRowSegBox : kRowSegFir;
  constexpr int nseg = kTileCols / S;
  const int L = 2 * W + 1;
  const int items = RH * nseg;
  for (int it = threadIdx.x; it < items; it += kThreads) {
    const int seg = it / RH;
    const int r = it - seg * RH;
    float o[S];
    if (KT == BF_BOX)
      box1d<S>(Fs + r * RWp + seg * S, 1, L, o);
    else
      fir1d<S>(Fs + r * RWp + seg * S, 1, L, tz, o);
    float* h = Hs + r * HP + seg * S;
#pragma unroll
    for (int s = 0; s < S; ++s) h[s] = o[s];
  }
}

// Row pass with the FIR regardless of the tile's kernel (adjoint's sigma_s term).
template <int HP>
__device__ __forceinline__ void rowpass_fir_any(const float* __restrict__ Fs, int RWp,
                                                float* __restrict__ Hs, int RH, int W,
                                                const float* __restrict__ tz) {
  rowpass<BF_GAUSS, HP>(Fs, RWp, Hs, RH, W, tz);
}

// Column pass: the thread owns column `lane` and output rows orow0 ..
// orow0 + OPT - 1; it reads Hs rows orow0 .. orow0 + OPT - 1 + 2W.
template <int KT, int OPT, int HP = kHPitch>
__device__ __forceinline__ void colpass(const float* __restrict__ Hs, int orow0, int lane, int W,
                                        const float* __restrict__ tz, float (&v)[OPT]) {
  const float* col = Hs + orow0 * HP + lane;
  if (KT == BF_BOX)
    box1d<OPT>(col, HP, 2 * W + 1, v);
  else
    fir1d<OPT>(col, HP, 2 * W + 1, tz, v);
}

// ---------------------------------------------------------------------------
// Region ownership: the thread owns region pixels q = t + 256 m (row-major
// over the padded region, pitch RWp).
// ---------------------------------------------------------------------------
struct RegionGeom {
  int RH, RW, RWp, npx;
};

// bwd: the adjoint tile's pitch (region_pitch_bwd)
__device__ __forceinline__ RegionGeom region_geom(int TY, int W, bool bwd = false) {
  RegionGeom g;
  g.RH = TY + 2 * W;
  g.RW = kTileCols + 2 * W;
  g.RWp = bwd ? region_pitch_bwd(W) : region_pitch(W);
  g.npx = g.RH * g.RWp;
  return g;
}

// Visit the thread's region pixels: fn(m, q, inside, gr, gc).
// Index into the reflected extension of [0, n) (edge samples repeated,
// period 2n): the mirror-border reading of the image outside its domain.
__host__ __device__ __forceinline__ int reflect_index(int i, int n) {
  int m = i % (2 * n);
  if (m < 0) m += 2 * n;
  return m < n ? m : 2 * n - 1 - m;
}

// Visit this thread's MREG region slots: fn(slot, q, inside, gr, gc).  With
// zero extension, `inside` marks slots on the image; with `mirror` every slot
// of the region is inside and (gr, gc) are reflected onto the image.
template <int MREG, typename Fn>
__device__ __forceinline__ void for_region(const RegionGeom& g, int r0, int c0, int W, int H,
                                           int Wd, Fn&& fn, bool mirror = false) {
  const int t = threadIdx.x;
  int row = t / g.RWp, col = t - row * g.RWp;
  const int srow = kThreads / g.RWp, scol = kThreads - srow * g.RWp;
#pragma unroll
  for (int m = 0; m < MREG; ++m) {
    const int q = t + kThreads * m;
    int gr = r0 - W + row, gc = c0 - W + col;
    bool inside = q < g.npx && col < g.RW;
    if (mirror) {
      gr = reflect_index(gr, H);
      gc = reflect_index(gc, Wd);
    } else {
      inside = inside && gr >= 0 && gr < H && gc >= 0 && gc < Wd;
    }
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
// Fused forward tile body.
//
// Range-safe form of Algorithm 2.  With X = T / sigma_r and y = x / X =
// (f - center) / T (|y| <= 1 on the dynamic range), the kernels keep
//     F^_n(j) = e^{-x_j^2/2} y_j^n                 (region, one multiply per n)
//     a_n(i)  = e^{-x_i^2/2} x_i^n X^n / n!        (coefficient, per output)
// so that a_n(i) F^_n(j) = e^{-x_i^2/2} e^{-x_j^2/2} (x_i x_j)^n / n!: the
// terms of eq. (Q) times e^{-x_i^2/2}, which cancels in eq. (PbyQ).  For
// T / sigma_r <= 13 every factor stays in the float32 range (the plan
// rejects smaller sigma_r).  With F_bar^_n the filtered F^_n:
//     Q = sum_{n<N} a_n F_bar^_n,   P = X sum_{n<N} a_n F_bar^_{n+1},
//     out = sigma_r P / Q + center.
// Products are formed in float32; with ACC64 the running sums are float32
// partials over blocks of 8 orders folded into float64 totals.
// SAVE additionally stores, per pixel, Q, P/Q and the coefficient-side
// derivative D_P - (P/Q) D_Q used by the adjoint, with
//     D_Q = X sum_{n=1}^{N-1} a_{n-1} F_bar^_n,
//     D_P = X^2 sum_{n=1}^{N-1} a_{n-1} F_bar^_{n+1}.
// ---------------------------------------------------------------------------
template <bool ACC64>
struct Accum {
  float part;
  double tot;
  __device__ __forceinline__ void zero() { part = 0.f; tot = 0.0; }
  __device__ __forceinline__ void add(float a, float b) { part = fmaf(a, b, part); }
  __device__ __forceinline__ void fold() { tot += (double)part; part = 0.f; }
  __device__ __forceinline__ double value() const { return tot + (double)part; }
};
template <>
struct Accum<false> {
  float part;
  __device__ __forceinline__ void zero() { part = 0.f; }
  __device__ __forceinline__ void add(float a, float b) { part = fmaf(a, b, part); }
  __device__ __forceinline__ void fold() {}
  __device__ __forceinline__ double value() const { return (double)part; }
};

template <int KT, int OPT, int MREG, bool ACC64, bool SAVE, int WC = 0>
__device__ __forceinline__ void forward_tile(const TileParams& p, int r0, int c0, float* lds) {
  // WC > 0: the support is a compile-time constant (the FIR and box loops
  // unroll completely and the taps stay in scalar registers across orders)
  const int W = WC > 0 ? WC : p.W;
  const int N = p.N;
  const RegionGeom g = region_geom(4 * OPT, W);
  float* Fs = lds;
  float* Hs = lds + align4(g.npx);
  const float* tz = p.taps + kTapPad;

  // region: F^_0 = e^{-x^2/2} into LDS, y kept in registers
  // region: F^_0 = e^{-x^2/2} into LDS, y kept in registers.  Loads use
  // clamped (always valid) addresses and no branches, so all MREG are in flight.
  float Fr[MREG], yr[MREG];
  for_region<MREG>(g, r0, c0, W, p.H, p.Wd, [&](int m, int q, bool inside, int gr, int gc) {
    const int cr = min(max(gr, 0), p.H - 1), cc = min(max(gc, 0), p.Wd - 1);
    Fr[m] = p.in[(int64_t)cr * p.in_pitch + cc];
    yr[m] = inside ? 1.f : 0.f;
  }, p.mirror != 0);
#pragma unroll
  for (int m = 0; m < MREG; ++m) {
    const float f = Fr[m];
    const bool inside = yr[m] != 0.f;
    const float x = (f - p.center) / p.sigma_r;
    yr[m] = inside ? (f - p.center) * p.inv_T : 0.f;
    Fr[m] = inside ? expf(-0.5f * x * x) : 0.f;
    const int q = threadIdx.x + kThreads * m;
    if (q < g.npx) Fs[q] = Fr[m];
  }

  const int lane = threadIdx.x & 63;
  const int orow0 = (threadIdx.x >> 6) * OPT;
  const int gc = c0 + lane;
  float z[OPT], a[OPT], ap[OPT], app[OPT];
  Accum<ACC64> P[OPT], Q[OPT], DP[OPT], DQ[OPT];
  const int gcc = min(gc, p.Wd - 1);
#pragma unroll
  for (int s = 0; s < OPT; ++s) z[s] = p.in[(int64_t)min(r0 + orow0 + s, p.H - 1) * p.in_pitch + gcc];
#pragma unroll
  for (int s = 0; s < OPT; ++s) {
    const float x = (z[s] - p.center) / p.sigma_r;  // pixels past the image: harmless, never stored
    z[s] = x * p.X;                // a_{n+1} = a_n x X / (n+1)
    a[s] = expf(-0.5f * x * x);    // a_0
    ap[s] = 0.f;                   // a_{n-1}
    app[s] = 0.f;                  // a_{n-2}
    P[s].zero();
    Q[s].zero();
    if (SAVE) {
      DP[s].zero();
      DQ[s].zero();
    }
  }
  __syncthreads();

  for (int n = 0; n <= N; ++n) {
    rowpass<KT>(Fs, g.RWp, Hs, g.RH, W, tz);
    __syncthreads();
    if (n < N) {
#pragma unroll
      for (int m = 0; m < MREG; ++m) {
        Fr[m] *= yr[m];  // F^_{n+1} = F^_n y
        const int q = threadIdx.x + kThreads * m;
        if (q < g.npx) Fs[q] = Fr[m];
      }
    }
    float v[OPT];
    colpass<KT, OPT>(Hs, orow0, lane, W, tz, v);
    const float in1 = p.inv_tab[n + 1];
#pragma unroll
    for (int s = 0; s < OPT; ++s) {
      if (n < N) Q[s].add(a[s], v[s]);      // eq. (Q)
      if (n >= 1) P[s].add(ap[s], v[s]);    // eq. (P), term of F_bar_n
      if (SAVE) {
        if (n >= 1 && n < N) DQ[s].add(ap[s], v[s]);
        if (n >= 2) DP[s].add(app[s], v[s]);
        app[s] = ap[s];
      }
      ap[s] = a[s];
      a[s] *= z[s] * in1;
    }
    if (ACC64 && ((n & 7) == 7)) {
#pragma unroll
      for (int s = 0; s < OPT; ++s) {
        P[s].fold();
        Q[s].fold();
        if (SAVE) {
          DP[s].fold();
          DQ[s].fold();
        }
      }
    }
    __syncthreads();
  }

  const double X = (double)p.X;
#pragma unroll
  for (int s = 0; s < OPT; ++s) {
    const int gr = r0 + orow0 + s;
    if (gr < p.H && gc < p.Wd) {
      const double q = Q[s].value();
      const double ratio = X * P[s].value() / q;
      if (p.out) p.out[(int64_t)gr * p.out_pitch + gc] = (float)((double)p.sigma_r * ratio + (double)p.center);
      if (SAVE && p.saved) {
        const int64_t idx = (int64_t)gr * p.Wd + gc;
        p.saved[idx] = (float)q;
        p.saved[p.saved_plane + idx] = (float)ratio;
        p.saved[2 * p.saved_plane + idx] = (float)(X * X * DP[s].value() - ratio * X * DQ[s].value());
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Cross (joint) filter, one 64 x 4*OPT tile: the range kernel acts on the
// guide h, the averaged values come from f (named as an extension in Sec. 1
// and Sec. 5).  With F^_n = e^{-x^2/2} y^n from the guide and a_n as in
// forward_tile (guide value at the output pixel),
//   Q = sum_{n<N} a_n (w * F^_n),  P = sum_{n<N} a_n (w * (F^_n f)),
//   out = P / Q:
// N orders, two filterings each (no order shift, the numerator is f).
// ---------------------------------------------------------------------------
template <int KT, int OPT, int MREG>
__device__ __forceinline__ void joint_tile(const TileParams& p, int r0, int c0, float* lds) {
  const int W = p.W;
  const int N = p.N;
  const RegionGeom g = region_geom(4 * OPT, W);
  const int np4 = align4(g.npx);
  float* Fs = lds;                  // F^_n
  float* Gs = lds + np4;            // F^_n f
  float* Hs = Gs + np4;             // row pass of F^_n
  float* Hg = Hs + g.RH * kHPitch;  // row pass of F^_n f
  const float* tz = p.taps + kTapPad;

  float Fr[MREG], yr[MREG], fr[MREG];
  for_region<MREG>(g, r0, c0, W, p.H, p.Wd, [&](int m, int q, bool inside, int gr, int gc) {
    const int cr = min(max(gr, 0), p.H - 1), cc = min(max(gc, 0), p.Wd - 1);
    Fr[m] = p.guide[(int64_t)cr * p.guide_pitch + cc];
    fr[m] = p.in[(int64_t)cr * p.in_pitch + cc];
    yr[m] = inside ? 1.f : 0.f;
  }, p.mirror != 0);
#pragma unroll
  for (int m = 0; m < MREG; ++m) {
    const float h = Fr[m];
    const bool inside = yr[m] != 0.f;
    const float x = (h - p.center) / p.sigma_r;
    yr[m] = inside ? (h - p.center) * p.inv_T : 0.f;
    Fr[m] = inside ? expf(-0.5f * x * x) : 0.f;
    fr[m] = inside ? fr[m] : 0.f;
    const int q = threadIdx.x + kThreads * m;
    if (q < g.npx) {
      Fs[q] = Fr[m];
      Gs[q] = Fr[m] * fr[m];
    }
  }

  const int lane = threadIdx.x & 63;
  const int orow0 = (threadIdx.x >> 6) * OPT;
  const int gc = c0 + lane;
  const int gcc = min(gc, p.Wd - 1);
  float z[OPT], a[OPT];
  Accum<true> P[OPT], Q[OPT];
#pragma unroll
  for (int s = 0; s < OPT; ++s) {
    const float h = p.guide[(int64_t)min(r0 + orow0 + s, p.H - 1) * p.guide_pitch + gcc];
    const float x = (h - p.center) / p.sigma_r;  // pixels past the image: harmless, never stored
    z[s] = x * p.X;
    a[s] = expf(-0.5f * x * x);
    P[s].zero();
    Q[s].zero();
  }
  __syncthreads();

  for (int n = 0; n < N; ++n) {
    rowpass<KT>(Fs, g.RWp, Hs, g.RH, W, tz);
    rowpass<KT>(Gs, g.RWp, Hg, g.RH, W, tz);
    __syncthreads();
    if (n + 1 < N) {
#pragma unroll
      for (int m = 0; m < MREG; ++m) {
        Fr[m] *= yr[m];
        const int q = threadIdx.x + kThreads * m;
        if (q < g.npx) {
          Fs[q] = Fr[m];
          Gs[q] = Fr[m] * fr[m];
        }
      }
    }
    float v[OPT], u[OPT];
    colpass<KT, OPT>(Hs, orow0, lane, W, tz, v);
    colpass<KT, OPT>(Hg, orow0, lane, W, tz, u);
    const float in1 = p.inv_tab[n + 1];
#pragma unroll
    for (int s = 0; s < OPT; ++s) {
      Q[s].add(a[s], v[s]);
      P[s].add(a[s], u[s]);
      a[s] *= z[s] * in1;
    }
    if ((n & 7) == 7) {
#pragma unroll
      for (int s = 0; s < OPT; ++s) {
        P[s].fold();
        Q[s].fold();
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int s = 0; s < OPT; ++s) {
    const int gr = r0 + orow0 + s;
    if (gr < p.H && gc < p.Wd) p.out[(int64_t)gr * p.out_pitch + gc] = (float)(P[s].value() / Q[s].value());
  }
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
// One 64 x 4*OPT tile of the adjoint: writes dL/df for its pixels and the
// tile's two sigma-gradient sums to part[0], part[1] (deterministic
// workgroup reduction in red, 2 x kThreads doubles of LDS).  WC > 0: the
// support is a compile-time constant, as in forward_tile.
template <int KT, int OPT, int MREG, bool SIGS, int WC = 0>
__device__ __forceinline__ void backward_tile(const TileParams& p, int r0, int c0, float* lds, double* red,
                                              double* part) {
  const int W = WC > 0 ? WC : p.W, N = p.N;
  const RegionGeom g = region_geom(4 * OPT, W, true);
  const int np4 = align4(g.npx);
  float* As = lds;
  float* Hs = As + np4;
  float* Fs2 = Hs + g.RH * kHPitchBwd;
  float* Hg = Fs2 + np4;
  float* Hg2 = Hg + g.RH * kHPitchBwd;
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
    rowpass<KT, kHPitchBwd>(As, g.RWp, Hs, g.RH, W, tz);
    if (SIGS) {
      rowpass_fir_any<kHPitchBwd>(Fs2, g.RWp, Hg, g.RH, W, tz);
      rowpass_fir_any<kHPitchBwd>(Fs2, g.RWp, Hg2, g.RH, W, tz2);
    }
    __syncthreads();
    float fa[OPT];
    colpass<KT, OPT, kHPitchBwd>(Hs, orow0, lane, W, tz, fa);
    if (SIGS) {
      float u[OPT], u2[OPT];
      colpass<BF_GAUSS, OPT, kHPitchBwd>(Hg, orow0, lane, W, tz2, u);   // d^2 g along rows of g-filtered
      colpass<BF_GAUSS, OPT, kHPitchBwd>(Hg2, orow0, lane, W, tz, u2);  // g along rows of d^2 g-filtered
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
  red[threadIdx.x] = dsr_loc;
  red[kThreads + threadIdx.x] = dss_loc * (double)p.inv_sigma_s3;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      red[kThreads + threadIdx.x] += red[kThreads + threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[0] = red[0];
    part[1] = red[kThreads];
  }
}


// Per-pixel coefficient state (a_n, a_{n-1}, a_{n-2}, z = x X) and float64
// sums of eqs. (P), (Q) (and the adjoint's D_P, D_Q) for CH output pixels,
// held in registers while orders are folded in; load/store move it to and
// from the streamed path's state images.  At the first block (first: n0 = 0)
// a_{-1}, a_{-2} and the sums start at zero and are not read: the lift
// writes only a_0 and z.
template <int CH, bool SAVE>
struct LsPix {
  float a[CH], ap[CH], app[CH], z[CH];
  double P[CH], Q[CH], DP[CH], DQ[CH];

  __device__ __forceinline__ void load(const LsState& st, int64_t i0, int64_t stride, int n_ok, bool first) {
#pragma unroll
    for (int s = 0; s < CH; ++s) {
      const bool ok = s < n_ok;
      const bool rd = ok && !first;
      const int64_t i = i0 + s * stride;
      a[s] = ok ? st.a[i] : 0.f;
      ap[s] = rd ? st.ap[i] : 0.f;
      z[s] = ok ? st.z[i] : 0.f;
      P[s] = rd ? st.P[i] : 0.0;
      Q[s] = rd ? st.Q[i] : 0.0;
      if (SAVE) {
        app[s] = rd ? st.app[i] : 0.f;
        DP[s] = rd ? st.DP[i] : 0.0;
        DQ[s] = rd ? st.DQ[i] : 0.0;
      }
    }
  }
  // pixels s0 .. s0 + M - 1 at i0 + (s - s0) * stride, the first n_ok of them inside the image
  template <int M>
  __device__ __forceinline__ void load_part(const LsState& st, int s0, int64_t i0, int64_t stride, int n_ok,
                                            bool first) {
#pragma unroll
    for (int u = 0; u < M; ++u) {
      const int s = s0 + u;
      const bool ok = u < n_ok;
      const bool rd = ok && !first;
      const int64_t i = ok ? i0 + u * stride : 0;
      a[s] = ok ? st.a[i] : 0.f;
      ap[s] = rd ? st.ap[i] : 0.f;
      z[s] = ok ? st.z[i] : 0.f;
      P[s] = rd ? st.P[i] : 0.0;
      Q[s] = rd ? st.Q[i] : 0.0;
      if (SAVE) {
        app[s] = rd ? st.app[i] : 0.f;
        DP[s] = rd ? st.DP[i] : 0.0;
        DQ[s] = rd ? st.DQ[i] : 0.0;
      }
    }
  }
  template <int M>
  __device__ __forceinline__ void store_part(const LsState& st, int s0, int64_t i0, int64_t stride,
                                             int n_ok) const {
#pragma unroll
    for (int u = 0; u < M; ++u) {
      const int s = s0 + u;
      if (u < n_ok) {
        const int64_t i = i0 + u * stride;
        st.a[i] = a[s];
        st.ap[i] = ap[s];
        st.P[i] = P[s];
        st.Q[i] = Q[s];
        if (SAVE) {
          st.app[i] = app[s];
          st.DP[i] = DP[s];
          st.DQ[i] = DQ[s];
        }
      }
    }
  }
  __device__ __forceinline__ void store(const LsState& st, int64_t i0, int64_t stride, int n_ok) const {
#pragma unroll
    for (int s = 0; s < CH; ++s) {
      if (s < n_ok) {
        const int64_t i = i0 + s * stride;
        st.a[i] = a[s];
        st.ap[i] = ap[s];
        st.P[i] = P[s];
        st.Q[i] = Q[s];
        if (SAVE) {
          st.app[i] = app[s];
          st.DP[i] = DP[s];
          st.DQ[i] = DQ[s];
        }
      }
    }
  }
  // fold F_bar_n (value v at pixel s) into eqs. (P), (Q) and advance a_n
  __device__ __forceinline__ void fold(int s, int n, int N, float v, float in1) {
    if (n < N) Q[s] = fma((double)a[s], (double)v, Q[s]);
    if (n >= 1) P[s] = fma((double)ap[s], (double)v, P[s]);
    if (SAVE) {
      if (n >= 1 && n < N) DQ[s] = fma((double)ap[s], (double)v, DQ[s]);
      if (n >= 2) DP[s] = fma((double)app[s], (double)v, DP[s]);
      app[s] = ap[s];
    }
    ap[s] = a[s];
    a[s] *= z[s] * in1;
  }
};

// Wide range: per-pixel a~_n = e^{-x_i^2/2} x_i^n / sqrt(n!) in float64, so
// a~_n F~_n is the term of eq. (Q) and sqrt(n) a~_{n-1} F~_n that of eq. (P)
// (without the X of the range-safe form); every factor is at most 1.
template <int CH>
struct WidePix {
  double a[CH], ap[CH], P[CH], Q[CH];
  float z[CH];
  // first: as for LsPix (the wide lift writes a~_0 and z only)
  __device__ __forceinline__ void load(const LsState& st, int64_t i0, int64_t stride, int n_ok, bool first) {
    load_part<CH>(st, 0, i0, stride, n_ok, first);
  }
  __device__ __forceinline__ void store(const LsState& st, int64_t i0, int64_t stride, int n_ok) const {
    store_part<CH>(st, 0, i0, stride, n_ok);
  }
  template <int M>
  __device__ __forceinline__ void load_part(const LsState& st, int s0, int64_t i0, int64_t stride, int n_ok,
                                            bool first) {
#pragma unroll
    for (int u = 0; u < M; ++u) {
      const int s = s0 + u;
      const bool ok = u < n_ok;
      const bool rd = ok && !first;
      const int64_t i = ok ? i0 + u * stride : 0;
      a[s] = ok ? st.ad[i] : 0.0;
      ap[s] = rd ? st.apd[i] : 0.0;
      z[s] = ok ? st.z[i] : 0.f;
      P[s] = rd ? st.P[i] : 0.0;
      Q[s] = rd ? st.Q[i] : 0.0;
    }
  }
  template <int M>
  __device__ __forceinline__ void store_part(const LsState& st, int s0, int64_t i0, int64_t stride,
                                             int n_ok) const {
#pragma unroll
    for (int u = 0; u < M; ++u) {
      const int s = s0 + u;
      if (u < n_ok) {
        const int64_t i = i0 + u * stride;
        st.ad[i] = a[s];
        st.apd[i] = ap[s];
        st.P[i] = P[s];
        st.Q[i] = Q[s];
      }
    }
  }
  // fold F~_bar_n (value v at pixel s); g1 = 1 / sqrt(n + 1), sn = sqrt(n)
  __device__ __forceinline__ void fold(int s, int n, int N, float v, double g1, double sn) {
    if (n < N) Q[s] = fma(a[s], (double)v, Q[s]);
    if (n >= 1) P[s] = fma(ap[s] * sn, (double)v, P[s]);
    ap[s] = a[s];
    a[s] = a[s] * (double)z[s] * g1;
  }
};

}  // namespace bfgpa
