// Streamed adjoint: the vector-Jacobian product of the GPA forward for
// supports too wide for the fused adjoint tiles.  It computes what the fused
// adjoint kernel does (same scaled recursions, same float64 sums), with the
// N + 1 filterings of the adjoint images adj_m moved through device memory in
// blocks of st.block orders, as in the streamed forward:
//   bls_init  : a_0 = (g sigma_r / Q) E and b_0 = 0 on the image, F~_0 = E and
//               zeroed sums at each pixel;
//   bls_rows  : per block, adj_m = b_m [m >= 1] - rho a_m [m <= N - 1] on a
//               16 x (256 + 2W) window, its row pass with the taps (and with
//               the d^2 taps for the sigma_s gradient) on the matrix cores,
//               written to row-filtered images; a, b advance in registers;
//   bls_cols  : the column passes (taps on the first image; for sigma_s the
//               d^2 taps on the first plus the taps on the second) and the
//               per-pixel folds  dx += (w * adj_m) dF~_m/dx,
//               dss += F~_m (w' * adj_m);
//   bls_final : dL/df, and per-workgroup partials of the sigma gradients,
//               summed in a fixed order.
// The sigma_s term uses <adj_m, w' * F_m> = <w' * adj_m, F_m> (the
// zero-extended symmetric filter is self-adjoint), so only adj_m is filtered.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "bf_device.h"
#include "bf_internal.h"
#include "bf_toeplitz.h"

namespace bfgpa {

constexpr int kBlsThreads = 512;  // eight waves
constexpr int kBlsRows = 16;      // window rows per row-pass workgroup
constexpr int kBlsCols = 256;     // output columns per row-pass workgroup
constexpr int kBlsRegs = 16;      // window values per thread: 16 (256 + 2W) <= 16 x 512

__global__ __launch_bounds__(kThreads) void bls_init_kernel(TileParams pk, BlsState st) {
  const TileParams p = with_dyn(pk);
  const int64_t npx = (int64_t)p.H * p.Wd;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < npx;
       i += (int64_t)gridDim.x * kThreads) {
    const int r = (int)(i / p.Wd), c = (int)(i - (int64_t)r * p.Wd);
    const float x = (p.in[(int64_t)r * p.in_pitch + c] - p.center) / p.sigma_r;
    const float E = expf(-0.5f * x * x);
    const float Qs = p.saved[i];
    const float pb = p.gout[(int64_t)r * p.gout_pitch + c] * p.sigma_r / Qs;
    const int64_t j = (int64_t)r * st.pitch + c;
    st.A[0][j] = pb * E;
    st.B[0][j] = 0.f;
    st.fc[i] = E;
    st.fp[i] = 0.f;
    st.dx[i] = 0.0;
    st.dss[i] = 0.0;
  }
}

// box1d on a contiguous, 8-byte aligned run, read in pairs (half the LDS
// instructions): out[s] = src[s] + ... + src[s + L - 1], s < S, for an odd
// L >= S + 1 and even S.  The window sum is that of src[0 .. L - 1], then
// advanced by one entering and one leaving value per output.
template <int S>
__device__ __forceinline__ void box1d_pairs(const float* __restrict__ src, int L, float (&out)[S]) {
  static_assert(S % 2 == 0, "pairs");
  const float2* p2 = (const float2*)src;
  float a[S];
#pragma unroll
  for (int i = 0; i < S / 2; ++i) {
    const float2 v = p2[i];
    a[2 * i] = v.x;
    a[2 * i + 1] = v.y;
  }
  float start[S];
  float acc = 0.f;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    start[s] = acc;
    acc += a[s];
  }
  // src[S .. L - 2]: pairs S / 2 .. (L - 1) / 2 - 1
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  const int iend = (L - 1) / 2;
  int i = S / 2;
  for (; i + 2 <= iend; i += 2) {
    const float2 u = p2[i], w = p2[i + 1];
    s0 += u.x;
    s1 += u.y;
    s2 += w.x;
    s3 += w.y;
  }
  for (; i < iend; ++i) {
    const float2 u = p2[i];
    s0 += u.x;
    s1 += u.y;
  }
  // e[t] = src[L - 1 + t], t < S
  float e[S];
#pragma unroll
  for (int j = 0; j < S / 2; ++j) {
    const float2 v = p2[iend + j];
    e[2 * j] = v.x;
    e[2 * j + 1] = v.y;
  }
  float lead = (acc + ((s0 + s1) + (s2 + s3))) + e[0];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    out[s] = lead - start[s];
    if (s + 1 < S) lead += e[s + 1];
  }
}

// Row pass of adj_m for orders n0 .. n0 + K - 1.  Thread t owns the window
// values q = t + 512 j and keeps x, rho, a, b for them in registers; adj_m
// goes to one of two LDS buffers (one barrier per order); wave w computes
// columns 32w .. 32w + 31 of the 16 rows as two 16x16 Toeplitz products per
// tap set and stores them from the accumulators.  BOX: the box kernel's
// unit taps as running sums on the VALU instead (thread t: row t % 16, eight
// consecutive output columns 8 (t / 16) .. + 7, prefix differences over its
// LDS row; no matrix-core product and no Toeplitz table).
template <bool SIGS, bool BOX = false>
__global__ __launch_bounds__(kBlsThreads) void bls_rows_kernel(TileParams pk, BlsState st, int n0, int K,
                                                               int src) {
  static_assert(!(SIGS && BOX), "the box kernel has no sigma_s gradient");
  const TileParams p = with_dyn(pk);
  extern __shared__ float lds[];
  const int W = p.W, N = p.N;
  const int RW = kBlsCols + 2 * W;
  const int RWp = ls_rows_pitch_mfma(W);
  const int KK = ls_kk(W);
  const int npx = kBlsRows * RWp;
  const int fls = align4(npx);
  float* Lb = lds;  // two buffers of fls
  float* Tt = lds + 2 * fls;
  float* Tt2 = Tt + KK * 64;
  const int tiles_x = (p.Wd + kBlsCols - 1) / kBlsCols;
  const int ty = blockIdx.x / tiles_x, tx = blockIdx.x - (blockIdx.x / tiles_x) * tiles_x;
  const int r0 = ty * kBlsRows, c0 = tx * kBlsCols;
  if (!BOX) fill_toeplitz<kBlsThreads>(Tt, W, p.taps + kTapPad);
  if (SIGS) fill_toeplitz<kBlsThreads>(Tt2, W, p.taps2 + kTapPad);
  float x[kBlsRegs], rho[kBlsRegs], a[kBlsRegs], b[kBlsRegs];
#pragma unroll
  for (int j = 0; j < kBlsRegs; ++j) {
    const int q = threadIdx.x + j * kBlsThreads;
    const int row = q / RWp, col = q - row * RWp;
    const int gr = r0 + row, gc = c0 - W + col;
    const bool ok = q < npx && col < RW && gr < p.H && gc >= 0 && gc < p.Wd;
    x[j] = ok ? (p.in[(int64_t)gr * p.in_pitch + gc] - p.center) / p.sigma_r : 0.f;
    rho[j] = ok ? p.saved[p.saved_plane + (int64_t)gr * p.Wd + gc] : 0.f;
    const int64_t i = ok ? (int64_t)gr * st.pitch + gc : 0;
    a[j] = ok ? st.A[src][i] : 0.f;
    b[j] = ok ? st.B[src][i] : 0.f;
  }
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int cbase = wv * 32;                  // this wave's two 16-column blocks
  const int orow = r0 + 4 * (lane >> 4);      // output row of accumulator v: orow + v
  const int ocol = c0 + cbase + (lane & 15);  // output column of block bb: ocol + 16 bb
  for (int k = 0; k < K; ++k) {
    const int m = n0 + k;
    const float rm1 = p.r_tab[m + 1];
    const float im1 = p.inv_tab[m + 1];
    float* Lc = Lb + (k & 1) * fls;
#pragma unroll
    for (int j = 0; j < kBlsRegs; ++j) {
      float adj = (m >= 1) ? b[j] : 0.f;
      if (m <= N - 1) adj = fmaf(-rho[j], a[j], adj);
      const int q = threadIdx.x + j * kBlsThreads;
      if (q < npx) Lc[q] = adj;
      const float bn = a[j] * rm1;
      a[j] = bn * (x[j] * im1);
      b[j] = bn;
    }
    __syncthreads();
    if constexpr (BOX) {
      // 16 rows x 32 runs of 8 columns, one per thread (kBlsThreads = 512)
      const int r = threadIdx.x & 15, c8 = 8 * (threadIdx.x >> 4);
      float o[8];
      if (2 * W + 1 >= 9)
        box1d_pairs<8>(Lc + r * RWp + c8, 2 * W + 1, o);  // RWp and c8 even: 8-byte aligned
      else
        box1d<8>(Lc + r * RWp + c8, 1, 2 * W + 1, o);
      const int gr = r0 + r, gc = c0 + c8;
      if (gr < p.H && gc < p.Wd) {
        float* d = st.r(k) + (int64_t)(W + gr) * st.pitch + gc;  // W zero rows above the image
        if (gc + 8 <= p.Wd) {
          *(float4*)d = make_float4(o[0], o[1], o[2], o[3]);
          *(float4*)(d + 4) = make_float4(o[4], o[5], o[6], o[7]);
        } else {
#pragma unroll
          for (int s = 0; s < 8; ++s)
            if (gc + s < p.Wd) d[s] = o[s];
        }
      }
      continue;
    }
    mf4 acc[2], acc2[2];
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) acc[bb] = acc2[bb] = mf4{0.f, 0.f, 0.f, 0.f};
    toeplitz_rows<2>(Lc, RWp, cbase, Tt, KK, acc);
    if (SIGS) toeplitz_rows<2>(Lc, RWp, cbase, Tt2, KK, acc2);
    float* R1 = st.r(k) + (int64_t)W * st.pitch;  // W zero rows above the image
    float* R2 = st.r2(k) + (int64_t)W * st.pitch;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (orow + v < p.H) {
#pragma unroll
        for (int bb = 0; bb < 2; ++bb) {
          if (ocol + 16 * bb < p.Wd) {
            const int64_t o = (int64_t)(orow + v) * st.pitch + ocol + 16 * bb;
            R1[o] = acc[bb][v];
            if (SIGS) R2[o] = acc2[bb][v];
          }
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kBlsRegs; ++j) {
    const int q = threadIdx.x + j * kBlsThreads;
    const int row = q / RWp, col = q - row * RWp;
    const int gr = r0 + row, gc = c0 - W + col;
    if (q < npx && col >= W && col < W + kBlsCols && gr < p.H && gc < p.Wd) {
      const int64_t i = (int64_t)gr * st.pitch + gc;
      st.A[src ^ 1][i] = a[j];
      st.B[src ^ 1][i] = b[j];
    }
  }
}

int64_t bls_rows_lds_bytes(int W, bool sigs) {
  const int64_t npx = (int64_t)kBlsRows * ls_rows_pitch_mfma(W);
  return 4 * (2 * ((npx + 3) & ~3LL) + (sigs ? 2 : 1) * (int64_t)ls_kk(W) * 64);
}

// Column passes and folds for a 64 x 64 tile: wave w covers rows
// 16 (w % 4) .. + 15 and columns 32 (w / 4) .. + 31, 8 pixels per lane.
template <bool SIGS>
__global__ __launch_bounds__(kBlsThreads) void bls_cols_kernel(TileParams pk, BlsState st, int n0, int K) {
  const TileParams p = with_dyn(pk);
  extern __shared__ float lds[];
  const int tiles_x = (p.Wd + kTileCols - 1) / kTileCols;
  const int tiles_y = (p.H + 63) / 64;
  int ty, tx;
  band_tile(xcd_remap(blockIdx.x, gridDim.x), tiles_x, tiles_y, ty, tx);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int rb = wv & 3, ch = wv >> 2;
  const int tr0 = ty * 64, c0 = tx * kTileCols;
  const int W = p.W;
  const int KK = ls_kk(W);
  const int rows = ls_cols_rows(W);
  float* S1 = lds;  // rows x 64 each
  float* S2 = S1 + rows * 64;
  float* Tt = SIGS ? S2 + rows * 64 : S2;
  float* Tt2 = Tt + KK * 64;
  fill_toeplitz<kBlsThreads>(Tt, W, p.taps + kTapPad);
  if (SIGS) fill_toeplitz<kBlsThreads>(Tt2, W, p.taps2 + kTapPad);
  // this lane's 8 pixels: block j (columns 32 ch + 16 j), accumulator v (row 4(l/16) + v)
  const int pr0 = tr0 + rb * 16 + 4 * (lane >> 4);
  const int pc0 = c0 + ch * 32 + (lane & 15);
  float x[8], fc[8], fp[8];
  double dx[8], dss[8];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int s = 4 * j + v;
      const int r = pr0 + v, c = pc0 + 16 * j;
      const bool ok = r < p.H && c < p.Wd;
      const int64_t i = ok ? (int64_t)r * p.Wd + c : 0;
      x[s] = ok ? (p.in[(int64_t)r * p.in_pitch + c] - p.center) / p.sigma_r : 0.f;
      fc[s] = ok ? st.fc[i] : 0.f;
      fp[s] = ok ? st.fp[i] : 0.f;
      dx[s] = ok ? st.dx[i] : 0.0;
      dss[s] = ok ? st.dss[i] : 0.0;
    }
  for (int k = 0; k < K; ++k) {
    const int m = n0 + k;
    __syncthreads();
    stage_rows_lds<kBlsThreads>(st.r(k) + (int64_t)tr0 * st.pitch + c0, st.pitch, S1, rows);
    if (SIGS) stage_rows_lds<kBlsThreads>(st.r2(k) + (int64_t)tr0 * st.pitch + c0, st.pitch, S2, rows);
    __syncthreads();
    mf4 fa[2], gs[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) fa[j] = gs[j] = mf4{0.f, 0.f, 0.f, 0.f};
    toeplitz_cols<2>(S1, rb * 16, ch * 32, Tt, KK, fa);
    if (SIGS) {
      toeplitz_cols<2>(S1, rb * 16, ch * 32, Tt2, KK, gs);
      toeplitz_cols<2>(S2, rb * 16, ch * 32, Tt, KK, gs);
    }
    const float sm = p.s_tab[m];
    const float sm1 = p.s_tab[m + 1];
    const float fm = (float)m * sm;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int s = 4 * j + v;
        const float factor = fmaf(fm, fp[s], -x[s] * fc[s]);  // dF~_m/dx
        dx[s] = fma((double)fa[j][v], (double)factor, dx[s]);
        if (SIGS) dss[s] = fma((double)fc[s], (double)gs[j][v], dss[s]);
        fp[s] = fc[s];
        fc[s] *= x[s] * sm1;
      }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int s = 4 * j + v;
      const int r = pr0 + v, c = pc0 + 16 * j;
      if (r < p.H && c < p.Wd) {
        const int64_t i = (int64_t)r * p.Wd + c;
        st.fc[i] = fc[s];
        st.fp[i] = fp[s];
        st.dx[i] = dx[s];
        st.dss[i] = dss[s];
      }
    }
}

// The box kernel's column pass and fold on the VALU: thread t owns column
// t % 64 of a 64 x 64 tile and its output rows 8 (t / 64) .. + 7, and sums
// each staged column window by prefix differences (box1d); the fold is that
// of bls_cols_kernel (the box has no sigma_s gradient: dss stays zero).
__global__ __launch_bounds__(kBlsThreads) void bls_cols_box_kernel(TileParams pk, BlsState st, int n0, int K) {
  const TileParams p = with_dyn(pk);
  extern __shared__ float lds[];
  const int tiles_x = (p.Wd + kTileCols - 1) / kTileCols;
  const int tiles_y = (p.H + 63) / 64;
  int ty, tx;
  band_tile(xcd_remap(blockIdx.x, gridDim.x), tiles_x, tiles_y, ty, tx);
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int tr0 = ty * 64, c0 = tx * kTileCols;
  const int W = p.W;
  const int rows = ls_cols_rows(W);
  float* S1 = lds;  // rows x 64
  const int pc = c0 + c, pr0 = tr0 + 8 * g;
  float x[8], fc[8], fp[8];
  double dx[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int r = pr0 + v;
    const bool ok = r < p.H && pc < p.Wd;
    const int64_t i = ok ? (int64_t)r * p.Wd + pc : 0;
    x[v] = ok ? (p.in[(int64_t)r * p.in_pitch + pc] - p.center) / p.sigma_r : 0.f;
    fc[v] = ok ? st.fc[i] : 0.f;
    fp[v] = ok ? st.fp[i] : 0.f;
    dx[v] = ok ? st.dx[i] : 0.0;
  }
  for (int k = 0; k < K; ++k) {
    const int m = n0 + k;
    __syncthreads();
    stage_rows_lds<kBlsThreads>(st.r(k) + (int64_t)tr0 * st.pitch + c0, st.pitch, S1, rows);
    __syncthreads();
    float fa[8];
    box1d<8>(S1 + 8 * g * 64 + c, 64, 2 * W + 1, fa);  // rows 8g + v .. 8g + v + 2W of the window
    const float sm = p.s_tab[m];
    const float sm1 = p.s_tab[m + 1];
    const float fm = (float)m * sm;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const float factor = fmaf(fm, fp[v], -x[v] * fc[v]);  // dF~_m/dx
      dx[v] = fma((double)fa[v], (double)factor, dx[v]);
      fp[v] = fc[v];
      fc[v] *= x[v] * sm1;
    }
  }
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int r = pr0 + v;
    if (r < p.H && pc < p.Wd) {
      const int64_t i = (int64_t)r * p.Wd + pc;
      st.fc[i] = fc[v];
      st.fp[i] = fp[v];
      st.dx[i] = dx[v];
    }
  }
}

int64_t bls_cols_lds_bytes(int W, bool sigs) {
  const int64_t n = sigs ? 2 : 1;
  return 4 * n * ((int64_t)ls_cols_rows(W) * 64 + (int64_t)ls_kk(W) * 64);
}

// dL/df and the per-workgroup partials of the sigma gradients.
__global__ __launch_bounds__(kThreads) void bls_final_kernel(TileParams pk, BlsState st, double* partials) {
  const TileParams p = with_dyn(pk);
  __shared__ double red[2][kThreads];
  const int64_t npx = (int64_t)p.H * p.Wd;
  double dsr = 0.0, dss = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < npx;
       i += (int64_t)gridDim.x * kThreads) {
    const int r = (int)(i / p.Wd), c = (int)(i - (int64_t)r * p.Wd);
    const float x = (p.in[(int64_t)r * p.in_pitch + c] - p.center) / p.sigma_r;
    const float gb = p.gout[(int64_t)r * p.gout_pitch + c];
    const double Qs = p.saved[i];
    const double rho = p.saved[p.saved_plane + i];
    const double Dc = p.saved[2 * p.saved_plane + i];
    const double pb = (double)gb * (double)p.sigma_r / Qs;
    const double dxt = st.dx[i] + pb * Dc;
    if (p.out) p.out[(int64_t)r * p.out_pitch + c] = (float)(dxt / (double)p.sigma_r);
    dsr += (double)gb * rho - dxt * (double)x / (double)p.sigma_r;
    dss += st.dss[i];
  }
  red[0][threadIdx.x] = dsr;
  red[1][threadIdx.x] = dss * (double)p.inv_sigma_s3;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * (int64_t)blockIdx.x] = red[0][0];
    partials[2 * (int64_t)blockIdx.x + 1] = red[1][0];
  }
}

bool bls_supported(int W, bool sigs) {
  return (int64_t)kBlsRows * ls_rows_pitch_mfma(W) <= (int64_t)kBlsRegs * kBlsThreads &&
         bls_rows_lds_bytes(W, sigs) <= max_lds_bytes() && bls_cols_lds_bytes(W, sigs) <= max_lds_bytes();
}

// Orders per block of the streamed adjoint: 32 from 4 Mpx (the per-pixel
// state crosses HBM once per block), else 8, which bounds the row-filtered
// images of smaller images (the batch shares one state among its images).
int bls_block_orders(int H, int Wd) { return (int64_t)H * Wd >= (int64_t)4 << 20 ? kBlsBlock : kBlsBlockSmall; }

int64_t bls_state_bytes(int H, int Wd, int W, bool sigs, int nblock) {
  const int64_t pitch = ((Wd + 63) / 64) * 64;
  const int64_t img = pitch * H;
  const int64_t himg = pitch * ls_hrows(H, W);
  const int64_t npx = (int64_t)H * Wd;
  const int64_t nr = (sigs ? 2 : 1) * nblock;
  const int64_t b = 4 * img * 4 + nr * himg * 4 + 2 * npx * 4 + 2 * npx * 8;
  return b + 256 * (4 + nr + 4);  // alignment of each buffer
}

BlsState bls_layout(void* base, int H, int Wd, int W, bool sigs, int nblock) {
  BlsState st = {};
  st.block = nblock;
  const int64_t pitch = ((Wd + 63) / 64) * 64;
  const int64_t img = pitch * H;
  const int64_t himg = pitch * ls_hrows(H, W);
  const int64_t npx = (int64_t)H * Wd;
  char* q = (char*)base;
  auto take = [&](int64_t bytes) {
    char* r = q;
    q += (bytes + 255) & ~255LL;
    return (void*)r;
  };
  st.pitch = pitch;
  for (int i = 0; i < 2; ++i) st.A[i] = (float*)take(img * 4);
  for (int i = 0; i < 2; ++i) st.B[i] = (float*)take(img * 4);
  st.r_stride = ((himg * 4 + 255) & ~255LL) / 4;  // take()'s rounding
  st.R0 = (float*)take(nblock * 4 * st.r_stride);
  st.R20 = sigs ? (float*)take(nblock * 4 * st.r_stride) : nullptr;
  st.fc = (float*)take(npx * 4);
  st.fp = (float*)take(npx * 4);
  st.dx = (double*)take(npx * 8);
  st.dss = (double*)take(npx * 8);
  return st;
}

hipError_t launch_backward_ls(const TileParams& p, const BlsState& st, bool sigs, double* partials,
                              double* grad_sigma, hipStream_t s) {
  if (p.H <= 0 || p.Wd <= 0) return hipSuccess;
  if (st.block <= 0 || st.block > kBlsBlock || (sigs && !st.R20)) return hipErrorInvalidValue;
  if (!bls_supported(p.W, sigs)) return hipErrorInvalidValue;
  const int64_t npx = (int64_t)p.H * p.Wd;
  const int g1 = (int)std::min<int64_t>((npx + kThreads - 1) / kThreads, 4096);
  hipLaunchKernelGGL(bls_init_kernel, dim3(g1), dim3(kThreads), 0, s, p, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the box kernel (no sigma_s gradient) filters with running sums on the VALU
  const bool box = p.kt == BF_BOX && !sigs;
  auto rk = sigs ? bls_rows_kernel<true> : box ? bls_rows_kernel<false, true> : bls_rows_kernel<false>;
  auto ck = sigs ? bls_cols_kernel<true> : box ? bls_cols_box_kernel : bls_cols_kernel<false>;
  e = hipFuncSetAttribute((const void*)rk, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)ck, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
  if (e != hipSuccess) return e;
  const size_t rl = (size_t)bls_rows_lds_bytes(p.W, sigs);
  const size_t cl = (size_t)bls_cols_lds_bytes(p.W, sigs);
  const int grow = ((p.H + kBlsRows - 1) / kBlsRows) * ((p.Wd + kBlsCols - 1) / kBlsCols);
  const int gcol = ((p.H + 63) / 64) * ((p.Wd + kTileCols - 1) / kTileCols);
  int src = 0;
  for (int n0 = 0; n0 <= p.N; n0 += st.block) {
    const int K = std::min(st.block, p.N + 1 - n0);
    hipLaunchKernelGGL(rk, dim3(grow), dim3(kBlsThreads), rl, s, p, st, n0, K, src);
    hipLaunchKernelGGL(ck, dim3(gcol), dim3(kBlsThreads), cl, s, p, st, n0, K);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    src ^= 1;
  }
  hipLaunchKernelGGL(bls_final_kernel, dim3(kBlsPartials), dim3(kThreads), 0, s, p, st, partials);
  e = hipGetLastError();
  if (e != hipSuccess || (!grad_sigma && !p.dyn)) return e;
  return launch_sigma_reduce(partials, kBlsPartials, p.kt == BF_GAUSS && sigs, grad_sigma, p.dyn, s);
}

}  // namespace bfgpa
