// Large-support forward: Algorithm 2 for supports W too wide for one tile's
// region to stay on chip (the fused kernels hold (TY + 2W) x (64 + 2W) region
// values per workgroup).  The N+1 filterings run in blocks of st.block orders
// orders through device memory:
//   ls_init  : F^_0 = e^{-x^2/2}, y, and the per-pixel coefficient state;
//   ls_rows  : per block, F^_n for the block's orders and the row pass of
//              each (rows staged in LDS with their W-column halo), written to
//              st.block row-filtered images; the state image advances by the
//              block length (double-buffered);
//   ls_cols  : the column pass of each row-filtered image (read straight
//              from device memory, coalesced along rows) folded into the
//              per-pixel sums of eqs. (P), (Q) held in registers for the block;
//   ls_final : eq. (PbyQ) and the optional adjoint state.
// The range-safe scaling is the same as in the fused kernels (bf_device.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "bf_device.h"
#include "bf_internal.h"
#include "bf_toeplitz.h"

namespace bfgpa {

constexpr int kLsOpt = 16;        // output rows per thread in ls_cols
constexpr int kLsColPitch = 80;   // LDS pitch of staged column windows (paired reads conflict-free)

// Compute units of the current device (queried once per process and device).
static int num_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

__global__ __launch_bounds__(kThreads) void ls_init_kernel(TileParams p, LsState st) {
  const int64_t npx = (int64_t)p.H * p.Wd;
  const float* in = p.dyn ? p.dyn->in : p.in;
  const int64_t in_pitch = p.dyn ? p.dyn->in_pitch : p.in_pitch;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < npx;
       i += (int64_t)gridDim.x * kThreads) {
    const int r = (int)(i / p.Wd), c = (int)(i - (int64_t)r * p.Wd);
    const float f = in[(int64_t)r * in_pitch + c];
    const float x = (f - p.center) / p.sigma_r;
    const float E = expf(-0.5f * x * x);
    const int64_t j = (int64_t)r * st.pitch + c;
    st.F[0][j] = E;
    st.Y[j] = (f - p.center) * p.inv_T;
    st.a[i] = E;  // a_{-1}, a_{-2} and the sums start at zero in the first block's column pass
    st.z[i] = x * p.X;
  }
}

// Row pass for orders n0 .. n0 + K - 1.  LDS: F^ and y for kLsRows rows x
// (kLsCols + 2W) columns (pitch = region_pitch-style), and the row-pass
// output of one order (kLsRows x kLsCols) staged for a coalesced store.
template <int KT>
__global__ __launch_bounds__(kThreads) void ls_rows_kernel(TileParams p, LsState st, int n0, int K,
                                                           int src) {
  extern __shared__ float lds[];
  const int W = p.W;
  const int RW = kLsCols + 2 * W;
  const int RWp = (RW % 4 == 2) ? RW : RW + 2;
  const int HP = kLsCols + 2;
  const int npx = kLsRows * RWp;
  float* Fl = lds;
  float* Yl = lds + align4(npx);
  float* Hl = Yl + align4(npx);
  const int tiles_x = (p.Wd + kLsCols - 1) / kLsCols;
  const int tile = blockIdx.x;
  const int ty = tile / tiles_x, tx = tile - (tile / tiles_x) * tiles_x;
  const int r0 = ty * kLsRows, c0 = tx * kLsCols;
  const float* Fin = st.F[src];
  float* Fout = st.F[src ^ 1];
  for (int q0 = threadIdx.x; q0 < npx; q0 += 4 * kThreads) {
    float F[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + u * kThreads;
      const int row = q / RWp, col = q - row * RWp;
      const int gr = r0 + row;
      int gc = c0 - W + col;
      F[u] = 0.f;
      y[u] = 0.f;
      if (p.mirror) gc = reflect_index(gc, p.Wd);  // mirror border: halo columns read their reflections
      if (q < npx && col < RW && gr < p.H && gc >= 0 && gc < p.Wd) {
        const int64_t j = (int64_t)gr * st.pitch + gc;
        F[u] = Fin[j];
        y[u] = st.Y[j];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + u * kThreads;
      if (q < npx) {
        Fl[q] = F[u];
        Yl[q] = y[u];
      }
    }
  }
  const float* tz = p.taps + kTapPad;
  constexpr int S = (KT == BF_BOX) ? kRowSegBox : kRowSegFir;
  constexpr int nseg = kLsCols / S;
  for (int k = 0; k < K; ++k) {
    __syncthreads();
    for (int it = threadIdx.x; it < kLsRows * nseg; it += kThreads) {
      const int seg = it / kLsRows;
      const int r = it - seg * kLsRows;
      float o[S];
      if (KT == BF_BOX)
        box1d<S>(Fl + r * RWp + seg * S, 1, 2 * W + 1, o);
      else
        fir1d<S>(Fl + r * RWp + seg * S, 1, 2 * W + 1, tz, o);
#pragma unroll
      for (int s = 0; s < S; ++s) Hl[r * HP + seg * S + s] = o[s];
    }
    __syncthreads();
    // coalesced store of this order's row-filtered rows; advance F^ by one power
    float* Hk = st.h(k) + (int64_t)W * st.pitch;  // W zero rows above the image
    for (int q = threadIdx.x; q < kLsRows * kLsCols; q += kThreads) {
      const int row = q / kLsCols, col = q - row * kLsCols;
      const int gr = r0 + row, gc = c0 + col;
      if (gr < p.H && gc < p.Wd) Hk[(int64_t)gr * st.pitch + gc] = Hl[row * HP + col];
    }
    for (int q = threadIdx.x; q < npx; q += kThreads) Fl[q] *= Yl[q];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kLsRows * kLsCols; q += kThreads) {
    const int row = q / kLsCols, col = q - row * kLsCols;
    const int gr = r0 + row, gc = c0 + col;
    if (gr < p.H && gc < p.Wd) Fout[(int64_t)gr * st.pitch + gc] = Fl[row * RWp + col + W];
  }
}

// ---------------------------------------------------------------------------
// Gaussian passes on the matrix cores (Toeplitz products, bf_toeplitz.h).
// ---------------------------------------------------------------------------

// Row pass on the matrix cores.  Each thread owns the staged values
// q = threadIdx.x + 256 j of the workgroup's kLsRows x (256 + 2W) window and
// keeps F^_n and y for them in registers; per order it writes F^_n to one of
// two LDS buffers (so one barrier per order suffices), the four waves each
// compute 16 rows x 64 columns of the row-filtered image as four 16x16
// products and store them straight from the accumulators, and F^ advances
// by one power in registers.
constexpr int kLsRowsRegs = 32;  // staged values per thread: 16 (256 + 2W) <= 32 x 256

bool ls_rows_mfma_fits(int W) { return kLsRows * ls_rows_pitch_mfma(W) <= kLsRowsRegs * kThreads; }

__global__ __launch_bounds__(kThreads) void ls_rows_mfma_kernel(TileParams p, LsState st, int n0, int K,
                                                                int src) {
  extern __shared__ float lds[];
  const int W = p.W;
  const int RW = kLsCols + 2 * W;
  const int RWp = ls_rows_pitch_mfma(W);
  const int KK = ls_kk(W);
  const int npx = kLsRows * RWp;
  const int fls = align4(npx);
  float* Fl = lds;  // two buffers of fls
  float* Tt = lds + 2 * fls;
  const int tiles_x = (p.Wd + kLsCols - 1) / kLsCols;
  const int tile = blockIdx.x;
  const int ty = tile / tiles_x, tx = tile - (tile / tiles_x) * tiles_x;
  const int r0 = ty * kLsRows, c0 = tx * kLsCols;
  const float* Fin = st.F[src];
  float* Fout = st.F[src ^ 1];
  fill_toeplitz<kThreads>(Tt, W, p.taps + kTapPad);
  float F[kLsRowsRegs], Y[kLsRowsRegs];
#pragma unroll
  for (int j = 0; j < kLsRowsRegs; ++j) {
    const int q = threadIdx.x + j * kThreads;
    const int row = q / RWp, col = q - row * RWp;
    const int gr = r0 + row;
    int gc = c0 - W + col;
    bool ok = q < npx && col < RW && gr < p.H;
    if (p.mirror)
      gc = reflect_index(gc, p.Wd);
    else
      ok = ok && gc >= 0 && gc < p.Wd;
    const int64_t i = ok ? (int64_t)gr * st.pitch + gc : 0;
    F[j] = ok ? Fin[i] : 0.f;
    Y[j] = ok ? st.Y[i] : 0.f;
  }
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int cbase = wv * 64;                         // this wave's four 16-column blocks
  const int orow = r0 + 4 * (lane >> 4);             // output row of accumulator v: orow + v
  const int ocol = c0 + cbase + (lane & 15);         // output column of block bb: ocol + 16 bb
  for (int k = 0; k < K; ++k) {
    float* Fc = Fl + (k & 1) * fls;
#pragma unroll
    for (int j = 0; j < kLsRowsRegs; ++j) {
      const int q = threadIdx.x + j * kThreads;
      if (q < npx) Fc[q] = F[j];
    }
    __syncthreads();
    mf4 acc[4];
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) acc[bb] = mf4{0.f, 0.f, 0.f, 0.f};
    toeplitz_rows<4>(Fc, RWp, cbase, Tt, KK, acc);
    float* Hk = st.h(k) + (int64_t)W * st.pitch;  // W zero rows above the image
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (orow + v < p.H) {
#pragma unroll
        for (int bb = 0; bb < 4; ++bb)
          if (ocol + 16 * bb < p.Wd) Hk[(int64_t)(orow + v) * st.pitch + ocol + 16 * bb] = acc[bb][v];
      }
    }
#pragma unroll
    for (int j = 0; j < kLsRowsRegs; ++j) F[j] *= Y[j];
  }
#pragma unroll
  for (int j = 0; j < kLsRowsRegs; ++j) {
    const int q = threadIdx.x + j * kThreads;
    const int row = q / RWp, col = q - row * RWp;
    const int gr = r0 + row, gc = c0 - W + col;
    if (q < npx && col >= W && col < W + kLsCols && gr < p.H && gc < p.Wd)
      Fout[(int64_t)gr * st.pitch + gc] = F[j];
  }
}

int64_t ls_rows_mfma_lds_bytes(int W) {
  const int64_t npx = (int64_t)kLsRows * ls_rows_pitch_mfma(W);
  const int64_t KK = (16 + 2 * W + 3) / 4;
  return 4 * (2 * ((npx + 3) & ~3LL) + KK * 64);
}

// Column pass on the matrix cores: a workgroup of eight waves stages
// ls_cols_rows(W) rows x 64 columns of one order's row-filtered image with
// direct-to-LDS loads; wave w computes output rows 16 (w % 4) .. + 15 and
// columns 32 (w / 4) .. + 31 as two 16x16 blocks and folds them into its 8
// pixels per lane.  The staged window never leaves the row-filtered image:
// it carries W zero rows above and W + 8 below a height padded to a
// multiple of 64.
constexpr int kColsThreads = 512;

template <bool SAVE>
__global__ __launch_bounds__(kColsThreads) void ls_cols_mfma_kernel(TileParams p, LsState st, int n0, int K) {
  extern __shared__ float lds[];
  const int tiles_x = (p.Wd + kTileCols - 1) / kTileCols;
  const int tiles_y = (p.H + 63) / 64;
  int ty, tx;
  band_tile(xcd_remap(blockIdx.x, gridDim.x), tiles_x, tiles_y, ty, tx);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int rb = wv & 3, ch = wv >> 2;  // row block, column half
  const int tr0 = ty * 64, c0 = tx * kTileCols;
  const int W = p.W;
  const int KK = ls_kk(W);
  const int rows = ls_cols_rows(W);
  float* Sl = lds;  // rows x 64, pitch 64
  float* Tt = lds + rows * 64;
  fill_toeplitz<kColsThreads>(Tt, W, p.taps + kTapPad);
  // this lane's 8 pixels: block j (columns 32 ch + 16 j ..), accumulator v (row 4(l/16)+v)
  const int pr0 = tr0 + rb * 16 + 4 * (lane >> 4);  // pixel row of accumulator v = pr0 + v
  const int pc0 = c0 + ch * 32 + (lane & 15);       // pixel column of block j = pc0 + 16 j
  LsPix<8, SAVE> px;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int nr = (pc0 + 16 * j < p.Wd) ? max(0, min(4, p.H - pr0)) : 0;
    px.template load_part<4>(st, j * 4, (int64_t)pr0 * p.Wd + pc0 + 16 * j, p.Wd, nr, n0 == 0);
  }
  for (int k = 0; k < K; ++k) {
    const int n = n0 + k;
    __syncthreads();
    if (p.mirror)
      stage_rows_lds_mirror<kColsThreads>(st.h(k), st.pitch, tr0, c0, W, p.H, Sl, rows);
    else
      stage_rows_lds<kColsThreads>(st.h(k) + (int64_t)tr0 * st.pitch + c0, st.pitch, Sl, rows);
    __syncthreads();
    mf4 acc[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[j] = mf4{0.f, 0.f, 0.f, 0.f};
    toeplitz_cols<2>(Sl, rb * 16, ch * 32, Tt, KK, acc);
    const float in1 = p.inv_tab[n + 1];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) px.fold(j * 4 + v, n, p.N, acc[j][v], in1);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int nr = (pc0 + 16 * j < p.Wd) ? max(0, min(4, p.H - pr0)) : 0;
    px.template store_part<4>(st, j * 4, (int64_t)pr0 * p.Wd + pc0 + 16 * j, p.Wd, nr);
  }
}

int64_t ls_cols_mfma_lds_bytes(int W) {
  const int64_t KK = (16 + 2 * W + 3) / 4;
  return 4 * ((int64_t)ls_cols_rows(W) * 64 + KK * 64);
}

// Box column pass: each thread walks a column segment of `seg_rows` rows
// with one running window sum per order of the block (two reads per output),
// CH pixels at a time.  Row-filtered images carry W zero rows above and
// below the image, so the window never leaves the buffer.
template <bool SAVE>
__global__ __launch_bounds__(kThreads) void ls_cols_box_kernel(TileParams p, LsState st, int n0, int K,
                                                               int seg_rows) {
  constexpr int CH = 8;
  const int c = blockIdx.x * kTileCols + (threadIdx.x & 63);
  const int rs = (blockIdx.y * 4 + (threadIdx.x >> 6)) * seg_rows;
  if (c >= p.Wd || rs >= p.H) return;  // no barriers in this kernel
  const int re = min(rs + seg_rows, p.H);
  const int L = 2 * p.W + 1;
  const int64_t pitch = st.pitch;
  float V[kLsBlockSmall];
#pragma unroll
  for (int k = 0; k < kLsBlockSmall; ++k)
    V[k] = (k < K) ? strided_sum(st.h(k) + (int64_t)rs * pitch + c, (int)pitch, 0, L) : 0.f;
  LsPix<CH, SAVE> px;
  for (int r = rs; r < re; r += CH) {
    const int nr = min(CH, re - r);
    px.load(st, (int64_t)r * p.Wd + c, p.Wd, nr, n0 == 0);
#pragma unroll
    for (int k = 0; k < kLsBlockSmall; ++k) {
      if (k < K) {
        const int n = n0 + k;
        const float in1 = p.inv_tab[n + 1];
        const float* hk = st.h(k) + c;
        float enter[CH], leave[CH];
#pragma unroll
        for (int s = 0; s < CH; ++s) {
          enter[s] = s < nr ? hk[(int64_t)(r + s + L) * pitch] : 0.f;
          leave[s] = s < nr ? hk[(int64_t)(r + s) * pitch] : 0.f;
        }
#pragma unroll
        for (int s = 0; s < CH; ++s) {
          if (s < nr) {
            px.fold(s, n, p.N, V[k], in1);
            V[k] += enter[s] - leave[s];
          }
        }
      }
    }
    px.store(st, (int64_t)r * p.Wd + c, p.Wd, nr);
  }
}

// FIR column pass: the workgroup stages the column window of one order's
// row-filtered image (4*OPT + 2W rows x 64 columns) in LDS; each thread
// filters its column over OPT output rows.  LDS pitch 80 keeps the paired
// reads of adjacent rows conflict-free.

template <int OPT, bool SAVE>
__global__ __launch_bounds__(kThreads) void ls_cols_fir_kernel(TileParams p, LsState st, int n0, int K) {
  extern __shared__ float lds[];
  const int tiles_x = (p.Wd + kTileCols - 1) / kTileCols;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int ty = tile / tiles_x, tx = tile - (tile / tiles_x) * tiles_x;
  const int lane = threadIdx.x & 63;
  const int tr0 = ty * 4 * OPT;
  const int orow = (threadIdx.x >> 6) * OPT;
  const int c0 = tx * kTileCols;
  const int c = c0 + lane;
  const int W = p.W;
  const int rows = 4 * OPT + 2 * W;
  const float* tz = p.taps + kTapPad;
  const int nr = max(0, min(OPT, p.H - (tr0 + orow)));
  LsPix<OPT, SAVE> px;
  if (c < p.Wd) px.load(st, (int64_t)(tr0 + orow) * p.Wd + c, p.Wd, nr, n0 == 0);
  for (int k = 0; k < K; ++k) {
    const int n = n0 + k;
    __syncthreads();
    const float* hk = st.h(k) + (int64_t)tr0 * st.pitch + c0;  // padded row tr0 = image row tr0 - W
    // eight loads in flight per thread before any LDS store
    const int total = rows * kTileCols;
    const bool col_ok = (c0 + (threadIdx.x & 63)) < p.Wd;  // q & 63 == threadIdx.x & 63 below
    for (int q0 = threadIdx.x; q0 < total; q0 += 8 * kThreads) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * kThreads;
        v[u] = (q < total && col_ok) ? hk[(int64_t)(q >> 6) * st.pitch + (q & 63)] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * kThreads;
        if (q < total) lds[(q >> 6) * kLsColPitch + (q & 63)] = v[u];
      }
    }
    __syncthreads();
    float v[OPT];
    fir1d<OPT>(lds + orow * kLsColPitch + lane, kLsColPitch, 2 * W + 1, tz, v);
    const float in1 = p.inv_tab[n + 1];
#pragma unroll
    for (int s = 0; s < OPT; ++s) px.fold(s, n, p.N, v[s], in1);
  }
  if (c < p.Wd) px.store(st, (int64_t)(tr0 + orow) * p.Wd + c, p.Wd, nr);
}

// ---------------------------------------------------------------------------
// Box kernel in column strips.  With C_n(r, c) = sum_{|dr| <= W} F^_n(r + dr, c)
// (zero outside the image), the box sum is F_bar_n(r, c) = sum_{|dc| <= W}
// C_n(r, c + dc).
// ---------------------------------------------------------------------------
// Segmented inclusive prefix sum of a float over the 64 lanes of a wave, in
// chunks of CH = 16, 32 or 64 lanes: row_shr steps inside each 16-lane row,
// then row_bcast:15 into rows 1 and 3 (chunks of 32) and row_bcast:31 into
// rows 2 and 3 (one chunk of 64).  Source lanes outside the row (or rows the
// mask leaves out) contribute 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, true));
}

// G independent segmented scans, step by step, so that each step's DPP
// operand of one value fills the wait states of the others
template <int G>
__device__ __forceinline__ void wave_scan_seg_n(float (&v)[G], int ch) {
#pragma unroll
  for (int g = 0; g < G; ++g) v[g] += dpp_f<0x111, 0xF>(v[g]);  // row_shr:1
#pragma unroll
  for (int g = 0; g < G; ++g) v[g] += dpp_f<0x112, 0xF>(v[g]);  // row_shr:2
#pragma unroll
  for (int g = 0; g < G; ++g) v[g] += dpp_f<0x114, 0xF>(v[g]);  // row_shr:4
#pragma unroll
  for (int g = 0; g < G; ++g) v[g] += dpp_f<0x118, 0xF>(v[g]);  // row_shr:8
  if (ch >= 32) {
#pragma unroll
    for (int g = 0; g < G; ++g) v[g] += dpp_f<0x142, 0xA>(v[g]);  // row_bcast:15 into rows 1, 3
  }
  if (ch >= 64) {
#pragma unroll
    for (int g = 0; g < G; ++g) v[g] += dpp_f<0x143, 0xC>(v[g]);  // row_bcast:31 into rows 2, 3
  }
}

constexpr int kStripThreads = 256;

// ---------------------------------------------------------------------------
// Box kernel in column strips, single-pass form used for every box support
// from 16 on large images.  A workgroup owns a strip of SC = 256 CPT columns
// (CPT per thread, halo included; OC = SC - 2W outputs) and a segment of
// rows, and processes the KB orders n0 .. n0 + KB - 1 of one launch; their
// column sums C_n(r, c) stay in float64 registers down the rows.  Per output
// row:
//   1. every thread writes the column sums of its columns for the KB orders
//      into LDS (rounded to float32);
//   2. (barrier) wave w takes the orders w, w + 4, ...  The strip row is cut
//      into chunks of L = CH CPL >= 2W + 1 columns (CH lanes of CPL = 4 CPT
//      columns each).  Lane l sums its CPL columns, a segmented DPP scan
//      joins the lanes of each chunk, and the prefix S within the chunk
//      overwrites the column sums in place (float32);
//   3. (barrier) each thread forms the window sums of its output columns c
//      from S and folds them into eqs. (P), (Q) in float64.  With a = c - W -
//      1 and b = c + W: S(b) - S(a) when both lie in one chunk, else S(b) +
//      (T - S(a)) with T the total of a's chunk (a window of 2W + 1 <= L
//      columns meets at most two chunks).  Every partial sum is therefore
//      bounded by two chunk sums, so the float32 rounding is that of a direct
//      sum over two windows, not of a prefix over the whole strip.
// Then every thread slides its column sums down one row: the entering and
// leaving rows' F^_n follow from F^_{n0} and y by the power recursion, in
// float64.  The fold has no per-order tests: the factor 1/(n + 1) that
// advances a_n is taken as 0 where n + 1 >= N, so a_n = 0 for every n >= N,
// and the orders past N in the last block add nothing (eq. (Q) stops at
// n = N - 1 and eq. (P) at n = N).  The per-pixel state between launches is
// a_{n0 - 1}, z and the two sums: a_{n0} = a_{n0 - 1} (z / n0) is recomputed
// with the rounding the chain itself applied, so it is the same float.  The
// rows entering the segment advance the F^ state image.
// ---------------------------------------------------------------------------
template <int CPT, int KB>
struct StripGeom {
  static constexpr int SC = 256 * CPT;              // strip columns
  static constexpr int CPL = 4 * CPT;               // columns per lane in the row scan
  static constexpr int CPITCH = SC + 4 * (SC / 32);  // float32 row: 4 floats of padding per 32 columns
  static constexpr int LDS_BYTES = 2 * KB * CPITCH * 4;  // two sets of rows, used by alternate image rows
};
// float32 column c of a row, 4 floats of padding after every 32: the 16-byte
// reads of 8 lanes (one LDS cycle) fall on distinct banks for runs of 16 or
// 32 bytes per lane, and 32 consecutive columns stay contiguous for the
// 4- and 8-byte accesses
__device__ __forceinline__ int strip_cpos(int c) { return c + 4 * (c >> 5); }

// lanes per scan chunk: the smallest of 16, 32, 64 whose CPL-column chunks
// hold a whole window of 2W + 1 columns
__host__ __device__ inline int strip_chunk_lanes(int cpl, int W) {
  return 16 * cpl >= 2 * W + 1 ? 16 : (32 * cpl >= 2 * W + 1 ? 32 : 64);
}

template <int CPT, bool SAVE, int KB>
__global__ __launch_bounds__(kStripThreads, 2) void ls_box_strip_kernel(TileParams p, LsState st, int n0, int src,
                                                                      int seg_rows) {
  using G = StripGeom<CPT, KB>;
  constexpr int SC = G::SC, CPL = G::CPL, NW = KB / 4;
  constexpr int SG = CPT == 1 ? NW : 2;  // orders a wave scans together
  extern __shared__ float Cbuf[];  // 2 x KB x CPITCH
  const int W = p.W;
  const int OC = SC - 2 * W;
  const int nstrips = (p.Wd + OC - 1) / OC;
  const int strip = blockIdx.x % nstrips, seg = blockIdx.x / nstrips;
  const int c0 = strip * OC;
  const int r_lo = seg * seg_rows, r_hi = min(r_lo + seg_rows, p.H);
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int ch = strip_chunk_lanes(CPL, W);
  const int L = ch * CPL;  // columns per scan chunk
  // this thread's strip columns CPT t + j (image columns c0 - W + CPT t + j)
  int gcs[CPT];
  bool col_ok[CPT], central[CPT];
  int gcol[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int sc = CPT * t + j, gc = c0 - W + sc;
    col_ok[j] = p.mirror || (gc >= 0 && gc < p.Wd);
    gcs[j] = p.mirror ? reflect_index(gc, p.Wd) : gc;
    central[j] = sc >= W && sc < W + OC && gc < p.Wd;  // an output column of this strip
    gcol[j] = gc;
  }
  // the fold's columns: output o = t + 256 j of the strip, strip column W + o
  // (consecutive lanes, consecutive columns; a wave whose lanes hold no output
  // skips that fold)
  int fcol[CPT];
  bool fout[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int o = t + 256 * j, gc = c0 + o;
    fout[j] = o < OC && gc < p.Wd;
    fcol[j] = gc;
  }
  const float* Fin = st.F[src];
  float* Fout = st.F[src ^ 1];
  // 1/(n + 1) for the block's orders, 0 from n + 1 = N on (wave-uniform)
  float in1[KB];
  float dqm[KB], dpm[KB];  // adjoint sums: eq. (Q)'s derivative stops at N - 1, (P)'s at N
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int n = n0 + k;
    in1[k] = (n + 1 < p.N) ? p.inv_tab[n + 1] : 0.f;
    dqm[k] = (n == p.N) ? 0.f : 1.f;
    dpm[k] = (n == p.N + 1) ? 0.f : 1.f;
  }
  // the factor that took a_{n0 - 1} to a_{n0} at the end of the previous block
  const float in1_prev = (n0 >= 1 && n0 < p.N) ? p.inv_tab[n0] : 0.f;
  double C[KB][CPT];
#pragma unroll
  for (int k = 0; k < KB; ++k)
#pragma unroll
    for (int j = 0; j < CPT; ++j) C[k][j] = 0.0;
  // clamped (always in bounds) load addresses; samples off the image read 0
#pragma unroll
  for (int j = 0; j < CPT; ++j) gcs[j] = min(max(gcs[j], 0), p.Wd - 1);
  auto load_row = [&](int q, float (&f)[CPT], float (&y)[CPT]) {
    const bool in_rows = p.mirror || (q >= 0 && q < p.H);
    q = p.mirror ? reflect_index(q, p.H) : min(max(q, 0), p.H - 1);
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int64_t i = (int64_t)q * st.pitch + gcs[j];
      const float fv = Fin[i], yv = st.Y[i];
      const bool ok = col_ok[j] && in_rows;
      f[j] = ok ? fv : 0.f;
      y[j] = ok ? yv : 0.f;
    }
  };
  // warm-up: the window of rows r_lo - W .. r_lo + W
  for (int q = r_lo - W; q <= r_lo + W; ++q) {
    float f[CPT], y[CPT];
    load_row(q, f, y);
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      double fd = (double)f[j];
      const double yd = (double)y[j];
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        C[k][j] += fd;
        fd *= yd;
      }
      if (central[j] && q >= r_lo && q < r_hi) Fout[(int64_t)q * st.pitch + gcol[j]] = (float)fd;
    }
  }
  // per-pixel state of a row (non-output columns read pixel (r, 0) and store
  // nothing); with one column per thread the next row's is loaded a row ahead
  constexpr bool PF = CPT == 1 && !SAVE;
  struct PixState {
    float ap, z, a;
    double P, Q;
  };
  // (the first block starts a_{-1} and the sums at zero: the lift writes a_0 and z only)
  auto load_state = [&](int r, PixState (&ps)[CPT]) {
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int64_t pi = (int64_t)r * p.Wd + (fout[j] ? fcol[j] : 0);
      ps[j].ap = n0 == 0 ? 0.f : st.ap[pi];
      ps[j].z = st.z[pi];
      ps[j].P = n0 == 0 ? 0.0 : st.P[pi];
      ps[j].Q = n0 == 0 ? 0.0 : st.Q[pi];
      ps[j].a = n0 == 0 ? st.a[pi] : 0.f;
    }
  };
  PixState nxt[CPT];
  if (PF && r_lo < r_hi) load_state(r_lo, nxt);
  for (int r = r_lo; r < r_hi; ++r) {
    // rows entering and leaving after this one, and this row's pixel state
    float fe[CPT], ye[CPT], fl[CPT], yl[CPT];
    load_row(r + W + 1, fe, ye);
    load_row(r - W, fl, yl);
    PixState cur[CPT];
    if (PF) {
#pragma unroll
      for (int j = 0; j < CPT; ++j) cur[j] = nxt[j];
      load_state(min(r + 1, r_hi - 1), nxt);
    } else {
      load_state(r, cur);
    }
    // the sums of even and odd orders are kept apart (two shorter dependency
    // chains); a_n advances in float32
    float af[CPT], ap[CPT], app[CPT], z[CPT];
    double P[CPT], Q[CPT], P1[CPT], Q1[CPT], DP[CPT], DQ[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int64_t pi = (int64_t)r * p.Wd + (fout[j] ? fcol[j] : 0);
      ap[j] = cur[j].ap;
      z[j] = cur[j].z;
      P[j] = cur[j].P;
      Q[j] = cur[j].Q;
      P1[j] = 0.0;
      Q1[j] = 0.0;
      if (n0 == 0)
        af[j] = cur[j].a;
      else
        af[j] = ap[j] * (z[j] * in1_prev);
      if (SAVE) {
        app[j] = n0 == 0 ? 0.f : st.app[pi];
        DP[j] = n0 == 0 ? 0.0 : st.DP[pi];
        DQ[j] = n0 == 0 ? 0.0 : st.DQ[pi];
      }
    }
    double ad[CPT], apd[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      ad[j] = (double)af[j];
      apd[j] = (double)ap[j];
    }
    // column sums of row r into LDS (the set of this row's parity: the fold
    // of row r - 1 may still read the other set)
    float* Cb = Cbuf + (r & 1) * KB * G::CPITCH;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      float* row = Cb + k * G::CPITCH + strip_cpos(CPT * t);
#pragma unroll
      for (int j = 0; j < CPT; ++j) row[j] = (float)C[k][j];
    }
    lds_barrier();
    // chunk prefixes of the orders wv, wv + 4, ..., SG of them together; each
    // lane rewrites its own CPL columns in place
#pragma unroll
    for (int jg = 0; jg < NW; jg += SG) {
      float x[SG][CPL];
#pragma unroll
      for (int g = 0; g < SG; ++g) {
        const float* crow = Cb + (wv + 4 * (jg + g)) * G::CPITCH;
#pragma unroll
        for (int u = 0; u < CPL; u += 4) {
          const float4 v4 = *(const float4*)(crow + strip_cpos(CPL * lane + u));
          x[g][u] = v4.x;
          x[g][u + 1] = v4.y;
          x[g][u + 2] = v4.z;
          x[g][u + 3] = v4.w;
        }
      }
      float v[SG];
#pragma unroll
      for (int g = 0; g < SG; ++g) {
#pragma unroll
        for (int u = 1; u < CPL; ++u) x[g][u] += x[g][u - 1];
        v[g] = x[g][CPL - 1];
      }
      wave_scan_seg_n<SG>(v, ch);
#pragma unroll
      for (int g = 0; g < SG; ++g) {
        const float ex = v[g] - x[g][CPL - 1];
        float* crow = Cb + (wv + 4 * (jg + g)) * G::CPITCH;
#pragma unroll
        for (int u = 0; u < CPL; u += 4)
          *(float4*)(crow + strip_cpos(CPL * lane + u)) =
              make_float4(ex + x[g][u], ex + x[g][u + 1], ex + x[g][u + 2], ex + x[g][u + 3]);
      }
    }
    lds_barrier();
    // window sums and the fold of this thread's output pixels: float64
    // products and sums (the terms of eqs. (P), (Q) cancel heavily at small
    // sigma_r; float32 partial sums cost about 5e-4 there).  The fold reads
    // other threads' columns; row r + 1 writes the other set, and row r + 2
    // writes this one only after the barrier of row r + 1, which every
    // thread reaches after this fold.
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (j > 0 && __builtin_amdgcn_ballot_w64(fout[j]) == 0) continue;  // wave-uniform
      // window ends b = c + W, a = c - W - 1, and the last column of a's chunk
      const int sc = W + t + 256 * j;
      const int b = min(sc + W, SC - 1), a = sc - W - 1;
      const int ac = min(max(a, 0), SC - 1);
      const int pb = strip_cpos(b), pa = strip_cpos(ac), pt = strip_cpos((ac / L) * L + L - 1);
      const float fa = a >= 0 ? 1.f : 0.f;
      const float ft = (a >= 0 && ac / L != b / L) ? 1.f : 0.f;
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const float* row = Cb + k * G::CPITCH;
        const float wsum = fmaf(-fa, row[pa], fmaf(ft, row[pt], row[pb]));
        const double vd = (double)wsum;
        if (k & 1) {
          Q1[j] = fma(ad[j], vd, Q1[j]);
          P1[j] = fma(apd[j], vd, P1[j]);
        } else {
          Q[j] = fma(ad[j], vd, Q[j]);
          P[j] = fma(apd[j], vd, P[j]);
        }
        if (SAVE) {
          DQ[j] = fma((double)(ap[j] * dqm[k]), vd, DQ[j]);
          DP[j] = fma((double)(app[j] * dpm[k]), vd, DP[j]);
          app[j] = ap[j];
        }
        ap[j] = af[j];
        apd[j] = ad[j];
        af[j] *= z[j] * in1[k];
        ad[j] = (double)af[j];
      }
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (fout[j]) {
        const int64_t pi = (int64_t)r * p.Wd + fcol[j];
        st.ap[pi] = ap[j];
        st.P[pi] = P[j] + P1[j];
        st.Q[pi] = Q[j] + Q1[j];
        if (SAVE) {
          st.app[pi] = app[j];
          st.DP[pi] = DP[j];
          st.DQ[pi] = DQ[j];
        }
      }
    }
    // slide the window to r + 1
    const int qe = r + W + 1;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      double fed = (double)fe[j], fld = (double)fl[j];
      const double yed = (double)ye[j], yld = (double)yl[j];
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        C[k][j] = (C[k][j] + fed) - fld;
        fed *= yed;
        fld *= yld;
      }
      if (central[j] && qe >= r_lo && qe < r_hi) Fout[(int64_t)qe * st.pitch + gcol[j]] = (float)fed;
    }
  }
}

bool ls_box_strip_supported(int W) { return 256 - 2 * W >= 64; }

// The strip kernel for a launch of kb orders (the shape's block, or 16 at
// the tail), and its LDS bytes.
static const void* box_strip_kernel(int cpt, bool save, int kb) {
  if (save) return (const void*)ls_box_strip_kernel<1, true, 16>;  // the saved state runs 256-column strips
  if (cpt == 2) return kb == 8 ? (const void*)ls_box_strip_kernel<2, false, 8> : (const void*)ls_box_strip_kernel<2, false, 16>;
  if (kb == 8) return (const void*)ls_box_strip_kernel<1, false, 8>;
  return kb == 32 ? (const void*)ls_box_strip_kernel<1, false, 32> : (const void*)ls_box_strip_kernel<1, false, 16>;
}
static int64_t box_strip_lds(int cpt, int kb) {
  if (cpt == 2) return kb == 8 ? StripGeom<2, 8>::LDS_BYTES : StripGeom<2, 16>::LDS_BYTES;
  if (kb == 8) return StripGeom<1, 8>::LDS_BYTES;
  return kb == 32 ? StripGeom<1, 32>::LDS_BYTES : StripGeom<1, 16>::LDS_BYTES;
}
// orders of the launch that starts at n0 (orders n0 .. N are left): the
// 32-order form runs 16 where they fit in 16 (splitting a 32-order tail costs
// more launches than its idle orders: 4096^2, W = 30, sigma_r = 30, 53
// orders: 1.46 ms as 32 + 32 against 1.55 as 32 + 16 + 8); the 512-column
// form runs 8 where they fit in 8 (W = 75, sigma_r = 30, 55 orders: 1.97 ms
// against 2.10 with 16 for the last 7); the saved state always 16.
static int box_strip_block(const StripShape& sh, bool save, int n0, int N) {
  const int left = N + 1 - n0;
  if (save) return 16;
  if (sh.kb == 32) return left <= 16 ? 16 : 32;
  return left <= 8 ? 8 : 16;
}

// Shape of the box strips on an H x Wd image: the 512-column form for the
// plain forward from W = 48 (its halo is shared by more outputs), else 256
// columns (4096^2, sigma_r = 10, W = 30: 5.3 ms against 6.2 for 512
// columns).  The plain 256-column form takes 32 orders per launch (the
// per-pixel state crosses HBM half as often; W = 30: 5.4 ms against 6.1 with
// 16 orders); the others 16.  Row segments: one wave of resident
// workgroups, so none trails; each pays a 2W + 1 row warm-up.
StripShape ls_box_strip_shape(int H, int Wd, int W, bool save) {
  StripShape sh;
  sh.cpt = (!save && W >= 48) ? 2 : 1;
  sh.kb = (save || sh.cpt == 2) ? 16 : 32;
  const int resident = (sh.cpt == 1 && sh.kb == 16 && !save) ? 3 : 2;
  sh.oc = 256 * sh.cpt - 2 * W;
  const int nstrips = (Wd + sh.oc - 1) / sh.oc;
  const int nseg = std::max(1, std::min((H + 31) / 32, num_cus() * resident / nstrips));
  sh.seg_rows = (H + nseg - 1) / nseg;
  sh.grid = nstrips * ((H + sh.seg_rows - 1) / sh.seg_rows);
  sh.lds = box_strip_lds(sh.cpt, sh.kb);
  return sh;
}

// The streamed kernels that implement the mirror border: box strips, and the
// matrix-core row and column passes of the Gaussian.
bool ls_mirror_supported(int kernel, int W) {
  if (kernel == BF_BOX) return ls_box_strip_supported(W);
  return ls_rows_mfma_fits(W) && ls_rows_mfma_lds_bytes(W) <= max_lds_bytes() &&
         ls_cols_mfma_lds_bytes(W) <= max_lds_bytes();
}

__global__ __launch_bounds__(kThreads) void ls_final_kernel(TileParams p, LsState st) {
  const int64_t npx = (int64_t)p.H * p.Wd;
  const double X = p.wide ? 1.0 : (double)p.X;  // the wide-range sums carry no 1/X
  float* out = p.dyn ? p.dyn->out : p.out;
  const int64_t out_pitch = p.dyn ? p.dyn->out_pitch : p.out_pitch;
  float* saved = p.dyn ? (p.dyn_save ? p.dyn->saved : nullptr) : p.saved;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < npx;
       i += (int64_t)gridDim.x * kThreads) {
    const int r = (int)(i / p.Wd), c = (int)(i - (int64_t)r * p.Wd);
    const double q = st.Q[i];
    const double ratio = X * st.P[i] / q;
    if (out) out[(int64_t)r * out_pitch + c] = (float)((double)p.sigma_r * ratio + (double)p.center);
    if (saved && st.DP) {
      saved[i] = (float)q;
      saved[p.saved_plane + i] = (float)ratio;
      saved[2 * p.saved_plane + i] = (float)(X * X * st.DP[i] - ratio * X * st.DQ[i]);
    }
  }
}

int64_t ls_rows_lds_bytes(int W) {
  const int RW = kLsCols + 2 * W;
  const int RWp = (RW % 4 == 2) ? RW : RW + 2;
  const int64_t npx = (int64_t)kLsRows * RWp;
  return 4 * (2 * ((npx + 3) & ~3LL) + (int64_t)kLsRows * (kLsCols + 2));
}

bool ls_supported(int W) {
  return ls_rows_lds_bytes(W) <= max_lds_bytes() &&
         (int64_t)(64 + 2 * W) * kLsColPitch * 4 <= max_lds_bytes();
}

// wide range: the F~ images and the coefficients in float64 instead of float32
// Orders per block of the streamed passes on an H x Wd image: 64 from 4 Mpx
// (the per-pixel state and the F^ image cross HBM once per block; 4096^2,
// sigma_r = 10: Gaussian W = 30 17.2 -> 15.4 -> 14.9 ms with 16 -> 32 -> 64
// orders, W = 75 20.7 -> 18.8 -> 18.1 ms), else 16, which bounds the
// row-filtered images of smaller images (a batch routes many of them to plans
// of their own).  The box strips keep their state in registers and need none;
// the box column pass of narrow supports walks at most 16 orders.
int ls_block_orders(int H, int Wd, int kernel, int W) {
  if (kernel == BF_BOX) return ls_box_strip_supported(W) ? 0 : kLsBlockSmall;
  return (int64_t)H * Wd >= (int64_t)4 << 20 ? kLsBlock : kLsBlockSmall;
}

// split: the row-filtered images pre-split (three bfloat16 planes each, the
// plain forward's split passes) instead of float32
int64_t ls_state_bytes(int H, int Wd, int W, bool save, bool wide, bool split, int nblock) {
  const int64_t pitch = ((Wd + 63) / 64) * 64;
  const int64_t img = pitch * H;
  const int64_t himg = split ? ((3 * 2 * pitch * ls_split_rows(H, W) + 255) & ~255LL) / 4 : pitch * ls_hrows(H, W);
  const int64_t npx = (int64_t)H * Wd;
  int64_t b = (wide ? 2 * img * 8 + img * 4 : 3 * img * 4) + (int64_t)nblock * himg * 4 +
              (wide ? 2 * npx * 8 + npx * 4 : 3 * npx * 4) + 2 * npx * 8;
  if (save) b += npx * 4 + 2 * npx * 8;
  return b + 256 * 32;
}

// Carve the state buffers out of one allocation.
LsState ls_layout(void* base, int H, int Wd, int W, bool save, bool wide, bool split, int nblock) {
  LsState st = {};
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
  if (wide) {
    st.Fd[0] = (double*)take(img * 8);
    st.Fd[1] = (double*)take(img * 8);
  } else {
    st.F[0] = (float*)take(img * 4);
    st.F[1] = (float*)take(img * 4);
  }
  st.Y = (float*)take(img * 4);
  if (split) {
    st.hs_plane = pitch * ls_split_rows(H, W);
    st.hs_stride = ((3 * 2 * st.hs_plane + 255) & ~255LL) / 2;  // take()'s rounding
    st.Hs0 = (uint16_t*)take(nblock * 2 * st.hs_stride);
  } else {
    st.h_stride = ((himg * 4 + 255) & ~255LL) / 4;
    st.H0 = nblock > 0 ? (float*)take(nblock * 4 * st.h_stride) : nullptr;
  }
  if (wide) {
    st.ad = (double*)take(npx * 8);
    st.apd = (double*)take(npx * 8);
  } else {
    st.a = (float*)take(npx * 4);
    st.ap = (float*)take(npx * 4);
  }
  st.z = (float*)take(npx * 4);
  st.P = (double*)take(npx * 8);
  st.Q = (double*)take(npx * 8);
  st.app = nullptr;
  st.DP = st.DQ = nullptr;
  if (save) {
    st.app = (float*)take(npx * 4);
    st.DP = (double*)take(npx * 8);
    st.DQ = (double*)take(npx * 8);
  }
  st.hbytes = split ? 0 : himg * 4;
  st.block = nblock;
  return st;
}

hipError_t launch_forward_ls(const TileParams& p, const LsState& st, bool save, hipStream_t s) {
  if (p.H <= 0 || p.Wd <= 0) return hipSuccess;
  if (p.mirror && !ls_mirror_supported(p.kt, p.W)) return hipErrorInvalidValue;
  if (save && !st.DP) return hipErrorInvalidValue;  // saved planes need the adjoint sums
  const int64_t npx = (int64_t)p.H * p.Wd;
  const int g1 = (int)std::min<int64_t>((npx + kThreads - 1) / kThreads, 4096);
  hipLaunchKernelGGL(ls_init_kernel, dim3(g1), dim3(kThreads), 0, s, p, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t rl = ls_rows_lds_bytes(p.W);
  auto rk = p.kt == BF_BOX ? ls_rows_kernel<BF_BOX> : ls_rows_kernel<BF_GAUSS>;
  e = hipFuncSetAttribute((const void*)rk, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
  if (e != hipSuccess) return e;
  const int grow = ((p.H + kLsRows - 1) / kLsRows) * ((p.Wd + kLsCols - 1) / kLsCols);
  const int tiles_x = (p.Wd + kTileCols - 1) / kTileCols;
  // box: column segments long enough that the window set-up (2W + 1 reads) is
  // amortised, short enough to give every CU several waves
  int seg_rows = 256;
  while (seg_rows > 16 && (int64_t)tiles_x * 4 * ((p.H + 4 * seg_rows - 1) / (4 * seg_rows)) < 2048) seg_rows /= 2;
  const dim3 gbox(tiles_x, (p.H + 4 * seg_rows - 1) / (4 * seg_rows));
  const int gfir8 = ((p.H + 31) / 32) * tiles_x;
  const int gfir16 = ((p.H + 63) / 64) * tiles_x;
  const size_t fl8 = (size_t)(32 + 2 * p.W) * kLsColPitch * 4;
  const size_t fl16 = (size_t)(64 + 2 * p.W) * kLsColPitch * 4;
  // box: column strips (float64 running column sums, float64 prefix-sum row windows)
  const bool box_strip = p.kt == BF_BOX && ls_box_strip_supported(p.W);
  const StripShape sh = box_strip ? ls_box_strip_shape(p.H, p.Wd, p.W, save) : StripShape{};
  if (box_strip) {
    for (int kb = sh.kb; kb >= (save || sh.kb == 32 ? 16 : 8); kb /= 2) {
      e = hipFuncSetAttribute(box_strip_kernel(sh.cpt, save, kb), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)box_strip_lds(sh.cpt, kb));
      if (e != hipSuccess) return e;
    }
  }
  // Gaussian: FIR passes on the matrix cores where the staged windows fit
  const size_t rlm = (size_t)ls_rows_mfma_lds_bytes(p.W);
  const size_t clm = (size_t)ls_cols_mfma_lds_bytes(p.W);
  const bool rows_mfma = p.kt != BF_BOX && ls_rows_mfma_fits(p.W) && rlm <= (size_t)max_lds_bytes();
  const bool cols_mfma = p.kt != BF_BOX && clm <= (size_t)max_lds_bytes();
  // split-bfloat16 passes (float32 products at about 2.3x the float32 matrix-core rate)
  const bool x3 = p.kt != BF_BOX && p.mfma_x3 && ls_x3_supported(p.W) &&
                  ls_rows_x3_lds_bytes(p.W) <= max_lds_bytes() && ls_cols_x3_lds_bytes(p.W) <= max_lds_bytes();
  if (rows_mfma) {
    e = hipFuncSetAttribute((const void*)ls_rows_mfma_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            max_lds_bytes());
    if (e != hipSuccess) return e;
  }
  if (cols_mfma) {
    e = hipFuncSetAttribute((const void*)ls_cols_mfma_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            max_lds_bytes());
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)ls_cols_mfma_kernel<true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
    if (e != hipSuccess) return e;
  }
  if (p.kt != BF_BOX) {
    auto k8 = ls_cols_fir_kernel<8, true>;
    auto k16 = ls_cols_fir_kernel<16, false>;
    e = hipFuncSetAttribute((const void*)k8, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k16, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
    if (e != hipSuccess) return e;
  }
  // pre-split row-filtered images (a plan's plain Gaussian forward): split row
  // pass and the column pass that stages the planes directly
  const bool split = st.Hs0 != nullptr;
  if (split && (save || p.mirror || !x3 || p.kt == BF_BOX)) return hipErrorInvalidValue;
  if (!box_strip && (st.block <= 0 || st.block > kLsBlock || (p.kt == BF_BOX && st.block > kLsBlockSmall)))
    return hipErrorInvalidValue;
  int src = 0;
  if (box_strip) {
    for (int n0 = 0; n0 <= p.N;) {
      const int kb = box_strip_block(sh, save, n0, p.N);
      int n0v = n0, srcv = src, segv = sh.seg_rows;
      TileParams pv = p;
      LsState sv = st;
      void* args[] = {(void*)&pv, (void*)&sv, (void*)&n0v, (void*)&srcv, (void*)&segv};
      e = hipLaunchKernel(box_strip_kernel(sh.cpt, save, kb), dim3(sh.grid), dim3(kStripThreads), args,
                          (size_t)box_strip_lds(sh.cpt, kb), s);
      if (e != hipSuccess) return e;
      src ^= 1;
      n0 += kb;
    }
  }
  // two passes per block of orders (every other path)
  for (int n0 = 0; !box_strip && n0 <= p.N; n0 += st.block) {
    const int K = std::min(st.block, p.N + 1 - n0);
    // row pass
    if (x3) {
      // split row pass always (4096^2, sigma_r = 30, ms per call, rows+cols
      // float32 / split rows / both split by the two-wave column pass: W = 30
      // 4.40 / 4.00 / 4.14, W = 51 5.82 / 4.95 / 4.78, W = 75 7.40 / 6.09 / 5.93)
      e = split ? launch_rows_x3_split(p, st, n0, K, src, grow, s) : launch_rows_x3(p, st, n0, K, src, grow, s);
    } else {
      if (rows_mfma)
        hipLaunchKernelGGL(ls_rows_mfma_kernel, dim3(grow), dim3(kThreads), (size_t)rlm, s, p, st, n0, K, src);
      else
        hipLaunchKernelGGL(rk, dim3(grow), dim3(kThreads), (size_t)rl, s, p, st, n0, K, src);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    // column pass
    if (x3) {
      // from W = 31 the column pass splits its window once per workgroup
      // (ls_cols_x3s) where its registers allow (up to 6 k-steps, plain
      // forward).  4096^2, sigma_r = 10, ms per call with the float32
      // matrix-core column pass / the split-once pass: W = 26 16.7 / 17.1,
      // W = 30 17.24 / 17.17, W = 33 17.9 / 17.3, W = 39 18.8 / 17.3.
      const bool x3s = !save && p.W >= 31 && (16 + 2 * p.W + 31) / 32 <= 6 && st.hbytes < (1LL << 31);
      if (split) {
        e = launch_cols_x3p(p, st, n0, K, n0 + K > p.N, s);  // the last block writes eq. (PbyQ) itself
      } else if (x3s) {
        e = launch_cols_x3s(p, st, n0, K, s);
      } else if (p.W >= 40) {
        e = launch_cols_x3(p, st, n0, K, save, gfir16, s);
      } else {
        if (save)
          hipLaunchKernelGGL((ls_cols_mfma_kernel<true>), dim3(gfir16), dim3(kColsThreads), clm, s, p, st, n0, K);
        else
          hipLaunchKernelGGL((ls_cols_mfma_kernel<false>), dim3(gfir16), dim3(kColsThreads), clm, s, p, st, n0, K);
        e = hipGetLastError();
      }
    } else {
      if (p.kt == BF_BOX) {
        if (save)
          hipLaunchKernelGGL((ls_cols_box_kernel<true>), gbox, dim3(kThreads), 0, s, p, st, n0, K, seg_rows);
        else
          hipLaunchKernelGGL((ls_cols_box_kernel<false>), gbox, dim3(kThreads), 0, s, p, st, n0, K, seg_rows);
      } else if (cols_mfma) {
        if (save)
          hipLaunchKernelGGL((ls_cols_mfma_kernel<true>), dim3(gfir16), dim3(kColsThreads), clm, s, p, st, n0, K);
        else
          hipLaunchKernelGGL((ls_cols_mfma_kernel<false>), dim3(gfir16), dim3(kColsThreads), clm, s, p, st, n0, K);
      } else {
        if (save)
          hipLaunchKernelGGL((ls_cols_fir_kernel<8, true>), dim3(gfir8), dim3(kThreads), fl8, s, p, st, n0, K);
        else
          hipLaunchKernelGGL((ls_cols_fir_kernel<16, false>), dim3(gfir16), dim3(kThreads), fl16, s, p, st, n0, K);
      }
      e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    src ^= 1;
  }
  if (split && !box_strip) return hipSuccess;
  hipLaunchKernelGGL(ls_final_kernel, dim3(g1), dim3(kThreads), 0, s, p, st);
  return hipGetLastError();
}

// Pieces of the streamed sequence for the volume path (bf_volume.hip): the
// lift, the row pass of one block of orders, and eq. (PbyQ).
hipError_t ls_launch_init(const TileParams& p, const LsState& st, hipStream_t s) {
  const int64_t npx = (int64_t)p.H * p.Wd;
  const int g1 = (int)std::min<int64_t>((npx + kThreads - 1) / kThreads, 4096);
  hipLaunchKernelGGL(ls_init_kernel, dim3(g1), dim3(kThreads), 0, s, p, st);
  return hipGetLastError();
}

hipError_t ls_launch_rows(const TileParams& p, const LsState& st, int n0, int K, int src, hipStream_t s) {
  const int grow = ((p.H + kLsRows - 1) / kLsRows) * ((p.Wd + kLsCols - 1) / kLsCols);
  if (p.kt != BF_BOX && p.mfma_x3 && ls_x3_supported(p.W) && ls_rows_x3_lds_bytes(p.W) <= max_lds_bytes())
    return launch_rows_x3(p, st, n0, K, src, grow, s);
  const size_t rlm = (size_t)ls_rows_mfma_lds_bytes(p.W);
  if (p.kt != BF_BOX && ls_rows_mfma_fits(p.W) && rlm <= (size_t)max_lds_bytes()) {
    hipError_t e = hipFuncSetAttribute((const void*)ls_rows_mfma_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       max_lds_bytes());
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ls_rows_mfma_kernel, dim3(grow), dim3(kThreads), rlm, s, p, st, n0, K, src);
    return hipGetLastError();
  }
  auto rk = p.kt == BF_BOX ? ls_rows_kernel<BF_BOX> : ls_rows_kernel<BF_GAUSS>;
  hipError_t e = hipFuncSetAttribute((const void*)rk, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rk, dim3(grow), dim3(kThreads), (size_t)ls_rows_lds_bytes(p.W), s, p, st, n0, K, src);
  return hipGetLastError();
}

hipError_t ls_launch_final(const TileParams& p, const LsState& st, hipStream_t s) {
  const int64_t npx = (int64_t)p.H * p.Wd;
  const int g1 = (int)std::min<int64_t>((npx + kThreads - 1) / kThreads, 4096);
  hipLaunchKernelGGL(ls_final_kernel, dim3(g1), dim3(kThreads), 0, s, p, st);
  return hipGetLastError();
}

}  // namespace bfgpa
