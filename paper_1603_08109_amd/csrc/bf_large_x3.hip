// Streamed Gaussian passes with float32 products emulated on the bfloat16
// matrix cores.  Every float32 operand is split exactly into three bfloat16
// terms, f = f_hi + f_mid + f_lo (each the round-to-nearest of what the
// previous ones leave, 8 significant bits apiece).  A product a t is then
// the six terms whose weights reach 2^-16 of it (hi hi, hi mid, mid hi,
// hi lo, mid mid, lo hi), each exact in float32 and accumulated in float32,
// which drops at most about 2^-23 of |a t|: the float32 product's own
// rounding.  v_mfma_f32_16x16x32_bf16 takes 16 cycles for a 16x16x32 block,
// against 32 for 16x16x4 in float32, so the six of them do the banded
// Toeplitz product of bf_toeplitz.h with about 2.3x fewer matrix-core cycles
// (k-steps of 32 instead of 4).
//
// Lane layout (checked on the GPU): lane l holds A[l%16][8(l/16) + i] and
// B[8(l/16) + i][l%16], i = 0..7; the result D[4(l/16) + v][l%16] sits in
// accumulator v.  The Toeplitz operand of k-step s, lane l, element i is
// tap[32 s + 8(l/16) + i - l%16] (zero outside [0, 2W]) in both passes (B of
// the row pass, A of the column pass); it is split once per workgroup into
// LDS as [s][plane][lane] groups of 8, then held in registers (up to 8
// k-steps x 3 planes x 4 VGPRs), so the only LDS reads per MFMA group are
// the data slices.
//
// Row pass: a workgroup (eight waves) owns 16 rows x 256 columns as in
// ls_rows_mfma; each order's F^_n is split into three bfloat16 planes in
// LDS (row pitch 8 mod 16 elements: the 16-byte reads of the 16 rows are
// conflict-free).  Two sets of planes: while the matrix cores multiply order
// k from one, each thread splits order k + 1 into the other, a slot pair per
// k-step; the number of k-steps is a template parameter, so one order is a
// single block of straight-line code the compiler can software-pipeline
// (operand reads of step q + 1 under the products of step q), with one
// barrier per order.
// Column pass (ls_cols_x3s, the plain forward up to 6 k-steps): tiles of 32
// columns x 128 rows; each order's window is loaded into registers while the
// previous order multiplies and split once per workgroup into one of two
// sets of three column-major bfloat16 planes in LDS, from which a lane's
// operand is one 16-byte read per plane.  Column pass with saved state or 7-8 k-steps
// (ls_cols_x3): 64 x 64 tiles, the float32 window staged by direct-to-LDS
// loads, each lane splitting its 8 rows of one column in registers.  In every
// pass a wave's blocks that read the same data slice one k-step apart share
// its reads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "bf_device.h"
#include "bf_internal.h"
#include "bf_toeplitz.h"

namespace bfgpa {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__host__ __device__ inline int x3_steps(int W) { return (16 + 2 * W + 31) / 32; }

// row pitch (bfloat16 elements) of a row-pass plane: the last slice reads
// column 239 + 32 S; 8 mod 16 keeps the 16-row reads conflict-free
__host__ __device__ inline int x3_rows_pitch(int W) {
  const int need = 240 + 32 * x3_steps(W);
  return ((need + 7) / 16) * 16 + 8;
}

// rows of a column-pass window: block pair rb, rb + 2 reads rows up to
// 16 rb + 32 S + 31 with rb <= 1
__host__ __device__ inline int x3_cols_rows(int W) { return 32 * x3_steps(W) + 48; }

constexpr int kX3RowsThreads = 512;
constexpr int kX3RowsRegs = 16;        // fp32 slots per thread in the row pass (8 pairs)
constexpr int kX3ColsThreads = 512;
constexpr int kX3MaxSteps = 8;             // k-steps of the widest support (W = 120)

// elements per bfloat16 plane of the row pass: 16 rows at x3_rows_pitch(W),
// padded so that each of a thread's slot pairs (elements below
// kX3RowsRegs * kX3RowsThreads) has a place without a bounds test
__host__ __device__ inline int x3_plane_elems(int W) {
  const int rows = kLsRows * x3_rows_pitch(W);
  return rows > kX3RowsRegs * kX3RowsThreads ? rows : kX3RowsRegs * kX3RowsThreads;
}

__device__ __forceinline__ void split3(float f, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)f;
  const float r = f - (float)h;
  m = (__bf16)r;
  l = (__bf16)(r - (float)m);
}

// split3 of two values at once, each plane's pair packed in one 32-bit word
// (first value in the low half): one packed conversion per plane, and the
// bfloat16 halves widened back by a shift or a mask.  The steps and their
// rounding are those of split3, so the pieces are the same.
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split3_pair(float f0, float f1, uint32_t& H, uint32_t& M, uint32_t& L) {
  H = __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v){f0, f1}, b2v));
  const float r0 = f0 - __uint_as_float(H << 16), r1 = f1 - __uint_as_float(H & 0xffff0000u);
  M = __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v){r0, r1}, b2v));
  const float s0 = r0 - __uint_as_float(M << 16), s1 = r1 - __uint_as_float(M & 0xffff0000u);
  L = __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v){s0, s1}, b2v));
}

// the three planes of the Toeplitz operand, [s][plane][lane] x 8, for S
// k-steps with the taps shifted down by sft rows (the window's first row is
// sft rows above the first output's)
template <int NT>
__device__ __forceinline__ void fill_toeplitz_x3(__bf16* Tb, int W, const float* __restrict__ tz, int S, int sft) {
  for (int u = threadIdx.x; u < S * 64; u += NT) {
    const int s = u >> 6, l = u & 63;
    bf8 ph, pm, pl;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int d = 32 * s + 8 * (l >> 4) + i - (l & 15) - sft;
      const float t = (d >= 0 && d <= 2 * W) ? tz[d] : 0.f;
      __bf16 h, m, lo;
      split3(t, h, m, lo);
      ph[i] = h;
      pm[i] = m;
      pl[i] = lo;
    }
    bf8* T = (bf8*)Tb;
    T[(s * 3 + 0) * 64 + l] = ph;
    T[(s * 3 + 1) * 64 + l] = pm;
    T[(s * 3 + 2) * 64 + l] = pl;
  }
}

struct X3 {
  bf8 h, m, l;
};

__device__ __forceinline__ X3 x3_table(const __bf16* Tb, int s, int lane) {
  const bf8* T = (const bf8*)Tb;
  X3 r;
  r.h = T[(s * 3 + 0) * 64 + lane];
  r.m = T[(s * 3 + 1) * 64 + lane];
  r.l = T[(s * 3 + 2) * 64 + lane];
  return r;
}

// acc += a b with both operands split (six bf16 products, smallest first)
__device__ __forceinline__ mf4 mfma_x3(const X3& a, const X3& b, mf4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, b.h, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.m, b.m, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.l, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.m, b.h, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.m, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, acc, 0, 0, 0);
  return acc;
}

// two independent sums, their six products interleaved so consecutive
// matrix-core instructions never wait on each other's result
__device__ __forceinline__ void mfma_x3_pair(const X3& a0, const X3& b0, mf4& acc0, const X3& a1, const X3& b1,
                                             mf4& acc1) {
  acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.l, b0.h, acc0, 0, 0, 0);
  acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.l, b1.h, acc1, 0, 0, 0);
  acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.m, b0.m, acc0, 0, 0, 0);
  acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.m, b1.m, acc1, 0, 0, 0);
  acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.h, b0.l, acc0, 0, 0, 0);
  acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.h, b1.l, acc1, 0, 0, 0);
  acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.m, b0.h, acc0, 0, 0, 0);
  acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.m, b1.h, acc1, 0, 0, 0);
  acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.h, b0.m, acc0, 0, 0, 0);
  acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.h, b1.m, acc1, 0, 0, 0);
  acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0.h, b0.h, acc0, 0, 0, 0);
  acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1.h, b1.h, acc1, 0, 0, 0);
}

bool ls_x3_supported(int W) {
  return kLsRows * x3_rows_pitch(W) <= kX3RowsRegs * kX3RowsThreads;  // W <= 120
}

// two sets of three bfloat16 planes, then the Toeplitz split table
int64_t ls_rows_x3_lds_bytes(int W) {
  return 2 * 2 * 3 * (int64_t)x3_plane_elems(W) + (int64_t)x3_steps(W) * 3 * 64 * 16;
}

int64_t ls_cols_x3_lds_bytes(int W) {
  // two float32 windows; the first order's Toeplitz split passes through the second
  const int64_t win = 4 * (int64_t)(x3_cols_rows(W) / 4) * (4 * 64 + 8);
  return 2 * win;
}

// slot pair jj of a thread (plane elements 2 (tid + jj 512) and + 1) into
// the three planes at P
template <typename FT>
__device__ __forceinline__ void x3_split_pair(FT f0, FT f1, __bf16* P, int plane, int jj) {
  const int q = 2 * (threadIdx.x + jj * kX3RowsThreads);
  uint32_t h, m, l;
  split3_pair((float)f0, (float)f1, h, m, l);
  *(uint32_t*)(P + q) = h;
  *(uint32_t*)(P + plane + q) = m;
  *(uint32_t*)(P + 2 * plane + q) = l;
}

// F^_n -> F^_{n+1} = F^_n y; wide range: F~_n -> F~_{n+1} = F~_n x / sqrt(n + 1)
template <bool WIDE, typename FT>
__device__ __forceinline__ void x3_advance(FT* F, const float* Y, const TileParams& p, int n) {
  if constexpr (WIDE) {
    const double g = p.isq[n + 1];
#pragma unroll
    for (int j = 0; j < kX3RowsRegs; ++j) F[j] = F[j] * (double)Y[j] * g;
  } else {
#pragma unroll
    for (int j = 0; j < kX3RowsRegs; ++j) F[j] *= Y[j];
  }
}

// Row pass for orders n0 .. n0 + K - 1 (see ls_rows_mfma_kernel for the tile
// and the F^ / y slots; here a thread owns pairs of adjacent columns).  Wave
// w takes the 16-column blocks par = w & 1 and par + 2 of column group
// w >> 1 (64 columns); they read the same slice one k-step apart.  S =
// x3_steps(W).
// WIDE: F~_n = e^{-x^2/2} x^n / sqrt(n!) in float64 (state images st.Fd),
// advanced by x / sqrt(n + 1); the matrix cores see it rounded to float32.
// SPLIT: the outputs are written pre-split (st.Hs: three bfloat16 planes,
// rows in groups of eight, image row i at row i + ls_split_top(W)); a lane's
// four consecutive rows of one column are one 8-byte store per plane.
template <int S, bool WIDE, bool SPLIT = false>
__global__ __launch_bounds__(kX3RowsThreads) void ls_rows_x3_kernel(TileParams p, LsState st, int n0, int K,
                                                                    int src) {
  using FT = typename std::conditional<WIDE, double, float>::type;
  extern __shared__ float lds[];
  const int W = p.W;
  const int RW = kLsCols + 2 * W;
  const int RWb = x3_rows_pitch(W);
  const int plane = x3_plane_elems(W);
  __bf16* Pl = (__bf16*)lds;  // two sets of 3 planes (orders k and k + 1)
  __bf16* Tb = Pl + 6 * plane;
  const int tiles_x = (p.Wd + kLsCols - 1) / kLsCols;
  const int tile = blockIdx.x;
  const int ty = tile / tiles_x, tx = tile - (tile / tiles_x) * tiles_x;
  const int r0 = ty * kLsRows, c0 = tx * kLsCols;
  const FT* Fin = (const FT*)(WIDE ? (const void*)st.Fd[src] : (const void*)st.F[src]);
  FT* Fout = (FT*)(WIDE ? (void*)st.Fd[src ^ 1] : (void*)st.F[src ^ 1]);
  fill_toeplitz_x3<kX3RowsThreads>(Tb, W, p.taps + kTapPad, x3_steps(W), 0);
  FT F[kX3RowsRegs];
  float Y[kX3RowsRegs];
#pragma unroll
  for (int j = 0; j < kX3RowsRegs; ++j) {
    const int q = 2 * (threadIdx.x + (j >> 1) * kX3RowsThreads) + (j & 1);
    const int row = q / RWb, col = q - (q / RWb) * RWb;
    const int gr = r0 + row;
    int gc = c0 - W + col;
    bool ok = row < kLsRows && col < RW && gr < p.H;
    if (p.mirror)
      gc = reflect_index(gc, p.Wd);
    else
      ok = ok && gc >= 0 && gc < p.Wd;
    const int64_t i = ok ? (int64_t)gr * st.pitch + gc : 0;
    F[j] = ok ? Fin[i] : (FT)0;
    Y[j] = ok ? st.Y[i] : 0.f;
  }
  // order n0 into the first set; F advances to order n0 + 1
#pragma unroll
  for (int jj = 0; jj < kX3RowsRegs / 2; ++jj) x3_split_pair(F[2 * jj], F[2 * jj + 1], Pl, plane, jj);
  x3_advance<WIDE>(F, Y, p, n0);
  __syncthreads();  // the table and the first set are written
  X3 T[S];  // this lane's Toeplitz operands, in registers for the whole kernel
#pragma unroll
  for (int q = 0; q < S; ++q) T[q] = x3_table(Tb, q, threadIdx.x & 63);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int cbase = 64 * (wv >> 1) + 16 * (wv & 1);  // block par; block par + 2 is 32 columns on
  const int orow = r0 + 4 * (lane >> 4);
  const int ocol = c0 + cbase + (lane & 15);
  // A reads: row l%16, columns cbase + 32 s + 8 (l/16) .. + 7
  const int abase = (lane & 15) * RWb + cbase + 8 * (lane >> 4);
  for (int k = 0; k < K; ++k) {
    if (k > 0) __syncthreads();  // order k's set is written; order k - 1's reads of the other set are done
    const __bf16* cur = Pl + (k & 1) * 3 * plane;
    __bf16* nxt = Pl + ((k + 1) & 1) * 3 * plane;
    mf4 acc[2] = {mf4{0.f, 0.f, 0.f, 0.f}, mf4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int q = 0; q <= S; ++q) {
      const int a = abase + 32 * q;
      X3 av;
      av.h = *(const bf8*)(cur + a);
      av.m = *(const bf8*)(cur + plane + a);
      av.l = *(const bf8*)(cur + 2 * plane + a);
      // block par at step q, block par + 2 at step q - 1
      if (q >= 1 && q < S)
        mfma_x3_pair(av, T[q < S ? q : 0], acc[0], av, T[q >= 1 ? q - 1 : 0], acc[1]);
      else if (q < S)
        acc[0] = mfma_x3(av, T[q], acc[0]);
      else
        acc[1] = mfma_x3(av, T[q >= 1 ? q - 1 : 0], acc[1]);
      // the next order's split under the matrix-core work (after the last
      // order it fills the idle set and is never read)
      if (q < kX3RowsRegs / 2) x3_split_pair(F[2 * q], F[2 * q + 1], nxt, plane, q);
    }
#pragma unroll
    for (int jj = S + 1; jj < kX3RowsRegs / 2; ++jj) x3_split_pair(F[2 * jj], F[2 * jj + 1], nxt, plane, jj);
    if (k + 1 < K) x3_advance<WIDE>(F, Y, p, n0 + k + 1);
    if constexpr (SPLIT) {
      // rows orow .. orow + 3 (rows past the image hold zeros: their F^ are 0)
      uint16_t* Hk = st.hs(k);
      const int R = orow + ls_split_top(W);  // a multiple of 4
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if (ocol + 32 * b < p.Wd) {
          uint32_t h0, m0, l0, h1, m1, l1;
          split3_pair(acc[b][0], acc[b][1], h0, m0, l0);
          split3_pair(acc[b][2], acc[b][3], h1, m1, l1);
          const int64_t e = ((int64_t)(R >> 3) * st.pitch + ocol + 32 * b) * 8 + (R & 7);
          *(uint2*)(Hk + e) = make_uint2(h0, h1);
          *(uint2*)(Hk + st.hs_plane + e) = make_uint2(m0, m1);
          *(uint2*)(Hk + 2 * st.hs_plane + e) = make_uint2(l0, l1);
        }
      }
    } else {
      float* Hk = st.h(k) + (int64_t)W * st.pitch;  // W zero rows above the image
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (orow + v < p.H) {
#pragma unroll
          for (int b = 0; b < 2; ++b)
            if (ocol + 32 * b < p.Wd) Hk[(int64_t)(orow + v) * st.pitch + ocol + 32 * b] = acc[b][v];
        }
      }
    }
  }
  // F holds order n0 + K
#pragma unroll
  for (int j = 0; j < kX3RowsRegs; ++j) {
    const int q = 2 * (threadIdx.x + (j >> 1) * kX3RowsThreads) + (j & 1);
    const int row = q / RWb, col = q - (q / RWb) * RWb;
    const int gr = r0 + row, gc = c0 - W + col;
    if (row < kLsRows && col >= W && col < W + kLsCols && gr < p.H && gc < p.Wd)
      Fout[(int64_t)gr * st.pitch + gc] = F[j];
  }
}

// Column pass: wave w takes the row blocks rb = w & 1 and rb + 2 of column
// block cb = w >> 1 (16 columns); they read the same window slice one k-step
// apart.  Lane pixels: accumulator v of block b at row 16 (rb + 2b) +
// 4 (l/16) + v, column 16 cb + l%16.  The window of order k + 1 is staged
// in float32 by direct-to-LDS loads (groups of 4 rows, group pitch 264
// floats so the 8-row reads of the four lane groups fall on distinct banks)
// while order k multiplies; a lane splits its 8 rows of one column into the
// three bfloat16 planes in registers.
constexpr int kX3GroupFloats = 4 * 64 + 8;

__host__ __device__ inline int64_t x3_cols_buffer_floats(int W) {
  return (int64_t)(x3_cols_rows(W) / 4) * kX3GroupFloats;
}

template <bool MIRROR>
__device__ __forceinline__ void x3_stage(const float* __restrict__ Hk, int64_t pitch, int tr0, int c0, int W, int H,
                                         int groups, float* buf) {
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  for (int g = wv; g < groups; g += kX3ColsThreads / 64) {
    int R = tr0 + 4 * g + (lane >> 4);  // padded row: image row R - W
    if (MIRROR) R = reflect_index(R - W, H) + W;
    __builtin_amdgcn_global_load_lds(Hk + (int64_t)R * pitch + c0 + (lane & 15) * 4,
                                     (__attribute__((address_space(3))) void*)(buf + g * kX3GroupFloats), 16, 0, 0);
  }
}


template <int S, bool SAVE, bool WIDE>
__global__ __launch_bounds__(kX3ColsThreads) void ls_cols_x3_kernel(TileParams p, LsState st, int n0, int K) {
  extern __shared__ float lds[];
  const int tiles_x = (p.Wd + kTileCols - 1) / kTileCols;
  const int tiles_y = (p.H + 63) / 64;
  int ty, tx;
  band_tile(xcd_remap(blockIdx.x, gridDim.x), tiles_x, tiles_y, ty, tx);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int rb = wv & 1, cb = wv >> 1;
  const int tr0 = ty * 64, c0 = tx * kTileCols;
  const int W = p.W;
  const int groups = x3_cols_rows(W) / 4;
  const int64_t bfl = x3_cols_buffer_floats(W);
  float* buf0 = lds;
  // the Toeplitz operands pass through the second buffer into registers
  fill_toeplitz_x3<kX3ColsThreads>((__bf16*)(lds + bfl), W, p.taps + kTapPad, x3_steps(W), 0);
  __syncthreads();
  X3 T[S];
#pragma unroll
  for (int q = 0; q < S; ++q) T[q] = x3_table((const __bf16*)(lds + bfl), q, lane);
  const int pr0 = tr0 + 16 * rb + 4 * (lane >> 4);
  const int pc = c0 + 16 * cb + (lane & 15);
  typename std::conditional<WIDE, WidePix<8>, LsPix<8, SAVE>>::type px;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int nr = pc < p.Wd ? max(0, min(4, p.H - (pr0 + 32 * b))) : 0;
    px.template load_part<4>(st, 4 * b, (int64_t)(pr0 + 32 * b) * p.Wd + pc, p.Wd, nr, n0 == 0);
  }
  if (p.mirror)
    x3_stage<true>(st.h(0), st.pitch, tr0, c0, W, p.H, groups, buf0);
  else
    x3_stage<false>(st.h(0), st.pitch, tr0, c0, W, p.H, groups, buf0);
  // this lane's column and first row of slice 0 (16 rb + 8 (l/16), a multiple
  // of 4: row r of a slice sits at group r / 4, offsets are compile-time)
  const int lbase = (4 * rb + 2 * (lane >> 4)) * kX3GroupFloats + 16 * cb + (lane & 15);
  for (int k = 0; k < K; ++k) {
    const int n = n0 + k;
    __syncthreads();  // order k staged (each thread waits for its loads); order k - 1 read
    float* cur = lds + (k & 1) * bfl;
    if (k + 1 < K) {
      float* nxt = lds + ((k + 1) & 1) * bfl;
      if (p.mirror)
        x3_stage<true>(st.h(k + 1), st.pitch, tr0, c0, W, p.H, groups, nxt);
      else
        x3_stage<false>(st.h(k + 1), st.pitch, tr0, c0, W, p.H, groups, nxt);
    }
    mf4 acc[2] = {mf4{0.f, 0.f, 0.f, 0.f}, mf4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int q = 0; q <= S; ++q) {
      X3 bv;
      const float* src = cur + lbase + 8 * q * kX3GroupFloats;
      uint32_t h[4], m[4], l[4];
#pragma unroll
      for (int i = 0; i < 8; i += 2)
        split3_pair(src[(i >> 2) * kX3GroupFloats + (i & 3) * 64], src[(i >> 2) * kX3GroupFloats + ((i + 1) & 3) * 64],
                    h[i / 2], m[i / 2], l[i / 2]);
      bv.h = __builtin_bit_cast(bf8, h);
      bv.m = __builtin_bit_cast(bf8, m);
      bv.l = __builtin_bit_cast(bf8, l);
      // block rb at step q, block rb + 2 at step q - 1
      if (q >= 1 && q < S)
        mfma_x3_pair(T[q < S ? q : 0], bv, acc[0], T[q >= 1 ? q - 1 : 0], bv, acc[1]);
      else if (q < S)
        acc[0] = mfma_x3(T[q], bv, acc[0]);
      else
        acc[1] = mfma_x3(T[q >= 1 ? q - 1 : 0], bv, acc[1]);
    }
    if constexpr (WIDE) {
      const double g1 = p.isq[n + 1], sn = p.sq[n];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) px.fold(4 * b + v, n, p.N, acc[b][v], g1, sn);
    } else {
      const float in1 = p.inv_tab[n + 1];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) px.fold(4 * b + v, n, p.N, acc[b][v], in1);
    }
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int nr = pc < p.Wd ? max(0, min(4, p.H - (pr0 + 32 * b))) : 0;
    px.template store_part<4>(st, 4 * b, (int64_t)(pr0 + 32 * b) * p.Wd + pc, p.Wd, nr);
  }
}

template <int S, bool WIDE, bool SPLIT>
static hipError_t rows_x3_s(const TileParams& p, const LsState& st, int n0, int K, int src, int grid, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)ls_rows_x3_kernel<S, WIDE, SPLIT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((ls_rows_x3_kernel<S, WIDE, SPLIT>), dim3(grid), dim3(kX3RowsThreads),
                     (size_t)ls_rows_x3_lds_bytes(p.W), s, p, st, n0, K, src);
  return hipGetLastError();
}

template <bool WIDE, bool SPLIT = false>
static hipError_t rows_x3_t(const TileParams& p, const LsState& st, int n0, int K, int src, int grid, hipStream_t s) {
  switch (x3_steps(p.W)) {
    case 1: return rows_x3_s<1, WIDE, SPLIT>(p, st, n0, K, src, grid, s);
    case 2: return rows_x3_s<2, WIDE, SPLIT>(p, st, n0, K, src, grid, s);
    case 3: return rows_x3_s<3, WIDE, SPLIT>(p, st, n0, K, src, grid, s);
    case 4: return rows_x3_s<4, WIDE, SPLIT>(p, st, n0, K, src, grid, s);
    case 5: return rows_x3_s<5, WIDE, SPLIT>(p, st, n0, K, src, grid, s);
    case 6: return rows_x3_s<6, WIDE, SPLIT>(p, st, n0, K, src, grid, s);
    case 7: return rows_x3_s<7, WIDE, SPLIT>(p, st, n0, K, src, grid, s);
    case 8: return rows_x3_s<8, WIDE, SPLIT>(p, st, n0, K, src, grid, s);
    default: return hipErrorInvalidValue;
  }
}

template <int S, bool SAVE, bool WIDE>
static hipError_t cols_x3_s(const TileParams& p, const LsState& st, int n0, int K, int grid, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)ls_cols_x3_kernel<S, SAVE, WIDE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((ls_cols_x3_kernel<S, SAVE, WIDE>), dim3(grid), dim3(kX3ColsThreads),
                     (size_t)ls_cols_x3_lds_bytes(p.W), s, p, st, n0, K);
  return hipGetLastError();
}

template <bool SAVE, bool WIDE>
static hipError_t cols_x3_t(const TileParams& p, const LsState& st, int n0, int K, int grid, hipStream_t s) {
  switch (x3_steps(p.W)) {
    case 1: return cols_x3_s<1, SAVE, WIDE>(p, st, n0, K, grid, s);
    case 2: return cols_x3_s<2, SAVE, WIDE>(p, st, n0, K, grid, s);
    case 3: return cols_x3_s<3, SAVE, WIDE>(p, st, n0, K, grid, s);
    case 4: return cols_x3_s<4, SAVE, WIDE>(p, st, n0, K, grid, s);
    case 5: return cols_x3_s<5, SAVE, WIDE>(p, st, n0, K, grid, s);
    case 6: return cols_x3_s<6, SAVE, WIDE>(p, st, n0, K, grid, s);
    case 7: return cols_x3_s<7, SAVE, WIDE>(p, st, n0, K, grid, s);
    case 8: return cols_x3_s<8, SAVE, WIDE>(p, st, n0, K, grid, s);
    default: return hipErrorInvalidValue;
  }
}

constexpr int kX3sCols = 32;  // columns of a split-once column-pass tile

// a lane's B operand at element offset o of the planes (8 rows of one column)
template <int RP>
__device__ __forceinline__ X3 x3s_operand(const __bf16* Pl, int o) {
  constexpr int PS = kX3sCols * RP;
  X3 r;
  r.h = *(const bf8*)(Pl + o);
  r.m = *(const bf8*)(Pl + PS + o);
  r.l = *(const bf8*)(Pl + 2 * PS + o);
  return r;
}


// Column pass, split-once form: tiles of 32 columns x 128 output rows, eight
// waves, one workgroup per compute unit.  Wave w takes column block
// cb = w >> 2 (16 columns) and the row blocks rb = (w & 1) + 4 ((w >> 1) & 1)
// and rb + 2, which read the same 32-row window slice one k-step apart, as in
// ls_cols_x3_kernel.  An order's window (R = 32 S + 112 rows of the padded
// row-filtered image) is loaded into registers, a thread owning items of 8
// consecutive rows of one column, and split ONCE into three bfloat16 planes
// in LDS, column-major: plane[column][row] with column stride RP = R + 8
// elements (8 mod 16), so the 16-byte operand reads of lanes on consecutive
// columns fall on distinct banks, and a lane's B operand (8 consecutive rows
// of one column) is one 16-byte read per plane.  Two sets of planes
// alternate between orders: one barrier per order, and each wave splits its
// share of order k + 1 into the other set between its matrix-core steps on
// order k, issuing the loads of order k + 2 as each item's registers free
// up.  The arithmetic and its order are those of ls_cols_x3, so the outputs
// are bit-identical.
constexpr int kX3sThreads = 512;
constexpr int kX3sRows = 128;

template <int S>
struct X3sGeom {
  static constexpr int R = 32 * S + 112;                                       // window rows
  static constexpr int RP = R + 8;                                             // column stride, 8 mod 16
  static constexpr int GROUPS = R / 8;                                         // items of 8 rows per column
  static constexpr int ITEMS = (GROUPS * kX3sCols + kX3sThreads - 1) / kX3sThreads;  // per thread
  static constexpr int PS = kX3sCols * RP;                                     // elements per plane
  static constexpr int BUF = 3 * PS;                                           // elements per set of planes
};

int64_t ls_cols_x3s_lds_bytes(int W) {
  const int64_t rp = 32LL * x3_steps(W) + 120;
  return 2 * 3 * kX3sCols * rp * 2;  // two sets of planes (the Toeplitz table, smaller, passes through the second)
}

// item i (8 rows of one column) of an order's window into registers; past the
// buffer (the padded rows of one row-filtered image) loads return 0
template <int S, bool MIRROR>
__device__ __forceinline__ void x3s_load_item(__amdgpu_buffer_rsrc_t rs, int pitch, int tr0, int c0, int W, int H,
                                              int i, float (&r)[8]) {
  using G = X3sGeom<S>;
  const int col = threadIdx.x & (kX3sCols - 1);
  const int g0 = threadIdx.x / kX3sCols;
  const int grp = min(g0 + (kX3sThreads / kX3sCols) * i, G::GROUPS - 1);  // idle items reload a valid group
  if (MIRROR) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int Rr = reflect_index(tr0 + 8 * grp + j - W, H) + W;  // padded row: image row Rr - W
      r[j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (Rr * pitch + c0 + col) * 4, 0, 0));
    }
  } else {
    const int vo = ((tr0 + 8 * grp) * pitch + c0 + col) * 4;
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, vo, j * pitch * 4, 0));
  }
}

template <int S>
__device__ __forceinline__ void x3s_split_item(const float (&r)[8], int i, __bf16* Pl) {
  using G = X3sGeom<S>;
  const int col = threadIdx.x & (kX3sCols - 1);
  const int grp = threadIdx.x / kX3sCols + (kX3sThreads / kX3sCols) * i;
  if (grp < G::GROUPS) {
    uint4 h, m, l;
    split3_pair(r[0], r[1], h.x, m.x, l.x);
    split3_pair(r[2], r[3], h.y, m.y, l.y);
    split3_pair(r[4], r[5], h.z, m.z, l.z);
    split3_pair(r[6], r[7], h.w, m.w, l.w);
    *(uint4*)(Pl + col * G::RP + 8 * grp) = h;
    *(uint4*)(Pl + G::PS + col * G::RP + 8 * grp) = m;
    *(uint4*)(Pl + 2 * G::PS + col * G::RP + 8 * grp) = l;
  }
}

template <int S, bool MIRROR>
__global__ __launch_bounds__(kX3sThreads) void ls_cols_x3s_kernel(TileParams p, LsState st, int n0, int K) {
  using G = X3sGeom<S>;
  extern __shared__ float lds[];
  __bf16* Pl = (__bf16*)lds;  // two sets of G::BUF elements
  const int tiles_x = (p.Wd + kX3sCols - 1) / kX3sCols;
  const int tiles_y = (p.H + kX3sRows - 1) / kX3sRows;
  int ty, tx;
  band_tile(xcd_remap(blockIdx.x, gridDim.x), tiles_x, tiles_y, ty, tx);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int cb = wv >> 2, rb = (wv & 1) + 4 * ((wv >> 1) & 1);
  const int tr0 = ty * kX3sRows, c0 = tx * kX3sCols;
  const int W = p.W;
  const int pitch = (int)st.pitch;
  auto rsrc = [&](int k) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)st.h(k), (short)0, (int)st.hbytes, 0x00020000);
  };
  float reg[G::ITEMS][8];
  {
    const __amdgpu_buffer_rsrc_t rs = rsrc(0);
#pragma unroll
    for (int i = 0; i < G::ITEMS; ++i) x3s_load_item<S, MIRROR>(rs, pitch, tr0, c0, W, p.H, i, reg[i]);
  }
  // the Toeplitz operands pass through the second set of planes into registers
  fill_toeplitz_x3<kX3sThreads>(Pl + G::BUF, W, p.taps + kTapPad, S, 0);
  __syncthreads();
  X3 T[S];
#pragma unroll
  for (int q = 0; q < S; ++q) T[q] = x3_table(Pl + G::BUF, q, lane);
#pragma unroll
  for (int i = 0; i < G::ITEMS; ++i) x3s_split_item<S>(reg[i], i, Pl);
  if (K > 1) {
    const __amdgpu_buffer_rsrc_t rs = rsrc(1);
#pragma unroll
    for (int i = 0; i < G::ITEMS; ++i) x3s_load_item<S, MIRROR>(rs, pitch, tr0, c0, W, p.H, i, reg[i]);
  }
  const int pr0 = tr0 + 16 * rb + 4 * (lane >> 4);
  const int pc = c0 + 16 * cb + (lane & 15);
  LsPix<8, false> px;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int nr = pc < p.Wd ? max(0, min(4, p.H - (pr0 + 32 * b))) : 0;
    px.template load_part<4>(st, 4 * b, (int64_t)(pr0 + 32 * b) * p.Wd + pc, p.Wd, nr, n0 == 0);
  }
  // this lane's operand: column 16 cb + l%16, rows 16 rb + 32 q + 8 (l/16) ..
  const int obase = (16 * cb + (lane & 15)) * G::RP + 16 * rb + 8 * (lane >> 4);
  for (int k = 0; k < K; ++k) {
    const int n = n0 + k;
    // order k's planes are written, and every wave has read order k - 1's (the set written next)
    __syncthreads();
    const __bf16* cur = Pl + (k & 1) * G::BUF;
    __bf16* nxt = Pl + ((k + 1) & 1) * G::BUF;
    const bool split_next = k + 1 < K;
    const bool load_next = k + 2 < K;
    const __amdgpu_buffer_rsrc_t rs = rsrc(load_next ? k + 2 : k);
    mf4 acc[2] = {mf4{0.f, 0.f, 0.f, 0.f}, mf4{0.f, 0.f, 0.f, 0.f}};
    X3 bv = x3s_operand<G::RP>(cur, obase);
#pragma unroll
    for (int q = 0; q <= S; ++q) {
      X3 bn;
      if (q < S) bn = x3s_operand<G::RP>(cur, obase + 32 * (q + 1));
      // block rb at step q, block rb + 2 at step q - 1
      if (q >= 1 && q < S)
        mfma_x3_pair(T[q < S ? q : 0], bv, acc[0], T[q >= 1 ? q - 1 : 0], bv, acc[1]);
      else if (q < S)
        acc[0] = mfma_x3(T[q], bv, acc[0]);
      else
        acc[1] = mfma_x3(T[q >= 1 ? q - 1 : 0], bv, acc[1]);
      // item q of order k + 1 into the other set, then its registers take order k + 2
      if (q < G::ITEMS) {
        if (split_next) x3s_split_item<S>(reg[q], q, nxt);
        if (load_next) x3s_load_item<S, MIRROR>(rs, pitch, tr0, c0, W, p.H, q, reg[q]);
      }
      asm volatile("" ::: "memory");
      bv = bn;
    }
    const float in1 = p.inv_tab[n + 1];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) px.fold(4 * b + v, n, p.N, acc[b][v], in1);
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int nr = pc < p.Wd ? max(0, min(4, p.H - (pr0 + 32 * b))) : 0;
    px.template store_part<4>(st, 4 * b, (int64_t)(pr0 + 32 * b) * p.Wd + pc, p.Wd, nr);
  }
}

template <int S, bool MIRROR>
static hipError_t cols_x3s_s(const TileParams& p, const LsState& st, int n0, int K, hipStream_t s) {
  static bool attr = false;
  const int64_t lb = ls_cols_x3s_lds_bytes(p.W);
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)ls_cols_x3s_kernel<S, MIRROR>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lb);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int grid = ((p.H + kX3sRows - 1) / kX3sRows) * ((p.Wd + kX3sCols - 1) / kX3sCols);
  hipLaunchKernelGGL((ls_cols_x3s_kernel<S, MIRROR>), dim3(grid), dim3(kX3sThreads), (size_t)lb, s, p, st, n0, K);
  return hipGetLastError();
}

template <bool MIRROR>
static hipError_t cols_x3s_m(const TileParams& p, const LsState& st, int n0, int K, hipStream_t s) {
  switch (x3_steps(p.W)) {
    case 1: return cols_x3s_s<1, MIRROR>(p, st, n0, K, s);
    case 2: return cols_x3s_s<2, MIRROR>(p, st, n0, K, s);
    case 3: return cols_x3s_s<3, MIRROR>(p, st, n0, K, s);
    case 4: return cols_x3s_s<4, MIRROR>(p, st, n0, K, s);
    case 5: return cols_x3s_s<5, MIRROR>(p, st, n0, K, s);
    case 6: return cols_x3s_s<6, MIRROR>(p, st, n0, K, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cols_x3s(const TileParams& p, const LsState& st, int n0, int K, hipStream_t s) {
  if (ls_cols_x3s_lds_bytes(p.W) > max_lds_bytes() || st.hbytes >= (1LL << 31)) return hipErrorInvalidValue;
  return p.mirror ? cols_x3s_m<true>(p, st, n0, K, s) : cols_x3s_m<false>(p, st, n0, K, s);
}

// Column pass on pre-split row-filtered images (the plain forward of a plan
// whose row pass writes its outputs split, st.Hs).  Tiles of 16 columns x
// 256 output rows, eight waves; wave w takes the row blocks rb = (w & 1) +
// 4 (w >> 1) and rb + 2 (16 rows each), which read the same window slice one
// k-step apart, with the matrix-core steps of ls_cols_x3s.  The window of an
// order (R = 32 S + 256 rows from the tile's first output row, in the split
// layout's row numbering) is copied straight from the planes into LDS by
// buffer-to-LDS loads while the previous order multiplies: no registers hold
// it and nothing is split here.  LDS keeps the global layout, [group of 8
// rows][16 columns][8 rows] per plane: one load of 64 lanes copies four
// groups of the tile's columns (four contiguous 256-byte runs), and a lane's
// B operand (8 rows of one column) is one 16-byte read per plane, the 16
// lanes of a group on consecutive columns (distinct banks).  The split layout
// puts image row i at row i + ls_split_top(W), sft = ls_split_top(W) - W rows
// below the window start that output row i's taps need, so the Toeplitz
// operand is shifted by sft and S = x3p_steps(W) k-steps cover 16 + 2W + sft
// rows.  Loads past the plane return zeros (the buffer's size), as do the
// zero rows above.  The taller, narrower tile re-reads fewer halo rows per
// output than 32 x 128 (1.75x against 2.4x at W = 75): 719 against 825 us per
// 16-order launch.
__host__ __device__ inline int x3p_shift(int W) { return ls_split_top(W) - W; }
__host__ __device__ inline int x3p_steps(int W) { return (16 + 2 * W + x3p_shift(W) + 31) / 32; }

constexpr int kX3pCols = 16;   // columns of a tile
constexpr int kX3pRows = 256;  // output rows of a tile (16 blocks of 16)

template <int S>
struct X3pGeom {
  static constexpr int R = 32 * S + 256;            // window rows (block 13 reads up to 16 * 13 + 32 S + 31)
  static constexpr int GROUPS = R / 8;              // groups of 8 rows, a multiple of 4
  static constexpr int PS = GROUPS * kX3pCols * 8;  // elements per plane
  static constexpr int BUF = 3 * PS;                // elements per set of planes
};

constexpr int kX3pSets = 2;  // sets of planes: order k multiplies while k + 1 arrives

int64_t ls_cols_x3p_lds_bytes(int W) {
  return kX3pSets * 3 * (32LL * x3p_steps(W) + 256) * kX3pCols * 2;  // the Toeplitz table passes through the last set
}

// With blocks of 64 orders every support; with 16 those of at least 5
// k-steps (W >= 57).  4096^2 Gaussians, ms per call (sigma_r = 10 / 30 / 50),
// 16 orders per block, split-once column pass against this pair: W = 75
// 21.7 / 5.30 / 3.16 against 20.7 / 4.80 / 2.74; at W = 30, against the
// float32 matrix-core column pass, 17.1 / 4.17 / 2.53 against 17.4 / 4.10 /
// 2.33 (the split row pass costs about as much as it saves).  With 64 orders
// per block, W = 30: 14.9 / 3.27 / 2.03 against 13.7 / 3.12 / 1.99 (and
// 14.3 / 3.17 / 1.97 for the split-once column pass).
bool ls_split_supported(int W, int nblock) {
  return ls_x3_supported(W) && x3p_steps(W) >= (nblock >= kLsBlock ? 1 : 5) && x3p_steps(W) <= kX3MaxSteps &&
         ls_cols_x3p_lds_bytes(W) <= max_lds_bytes();
}

// fin: the block holds order N, so instead of the per-pixel state the kernel
// writes eq. (PbyQ), out = sigma_r X P / Q + c (in float64, as ls_final_kernel).
template <int S>
__global__ __launch_bounds__(kX3sThreads) void ls_cols_x3p_kernel(TileParams p, LsState st, int n0, int K, int fin) {
  using G = X3pGeom<S>;
  static_assert(G::GROUPS % 4 == 0, "four groups per load");
  constexpr int NLOADS = 3 * G::GROUPS / 4;         // loads of 64 lanes per order
  constexpr int NWAVES = kX3sThreads / 64;
  extern __shared__ float lds[];
  __bf16* Pl = (__bf16*)lds;  // kX3pSets sets of G::BUF elements
  const int tiles_x = (p.Wd + kX3pCols - 1) / kX3pCols;
  const int tiles_y = (p.H + kX3pRows - 1) / kX3pRows;
  int ty, tx;
  band_tile(xcd_remap(blockIdx.x, gridDim.x), tiles_x, tiles_y, ty, tx);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: the loads' descriptors and LDS bases stay scalar
  const int rb = (wv & 1) + 4 * (wv >> 1);  // row blocks rb and rb + 2 (16 rows each)
  const int tr0 = ty * kX3pRows, c0 = tx * kX3pCols;
  const int W = p.W;
  const int64_t pitch = st.pitch;
  const int plane_bytes = (int)(st.hs_plane * 2);
  // lane offset of a load: group lane / 16 of the four, column lane % 16
  const int lvo = (int)(((int64_t)(tr0 >> 3) + (lane >> 4)) * pitch + c0 + (lane & 15)) * 16;
  // this wave's loads of an order into a set: load u = plane u / (GROUPS / 4),
  // groups 4 (u % (GROUPS / 4)) .. + 3
  auto stage = [&](int k, __bf16* set) {
    const uint16_t* Hk = st.hs(k);
    for (int u = wv; u < NLOADS; u += NWAVES) {
      const int pl = u / (G::GROUPS / 4), g0 = 4 * (u - pl * (G::GROUPS / 4));
      const __amdgpu_buffer_rsrc_t rs =
          __builtin_amdgcn_make_buffer_rsrc((void*)(Hk + pl * st.hs_plane), (short)0, plane_bytes, 0x00020000);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rs, (__attribute__((address_space(3))) void*)(set + pl * G::PS + g0 * kX3pCols * 8), 16,
          lvo + (int)(g0 * pitch * 16), 0, 0, 0);
    }
  };
  // the Toeplitz operands pass through the last set of planes into registers
  __bf16* Tset = Pl + (kX3pSets - 1) * G::BUF;
  fill_toeplitz_x3<kX3sThreads>(Tset, W, p.taps + kTapPad, S, x3p_shift(W));
  __syncthreads();
  X3 T[S];
#pragma unroll
  for (int q = 0; q < S; ++q) T[q] = x3_table(Tset, q, lane);
  stage(0, Pl);
  const int pr0 = tr0 + 16 * rb + 4 * (lane >> 4);
  const int pc = c0 + (lane & 15);
  LsPix<8, false> px;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int nr = pc < p.Wd ? max(0, min(4, p.H - (pr0 + 32 * b))) : 0;
    px.template load_part<4>(st, 4 * b, (int64_t)(pr0 + 32 * b) * p.Wd + pc, p.Wd, nr, n0 == 0);
  }
  // this lane's operand: column l%16, rows 16 rb + 32 q + 8 (l/16) .. + 7,
  // i.e. group 2 rb + 4 q + l/16
  const int obase = ((2 * rb + (lane >> 4)) * kX3pCols + (lane & 15)) * 8;
  constexpr int QSTEP = 4 * kX3pCols * 8;  // elements per k-step (four groups)
  for (int k = 0; k < K; ++k) {
    const int n = n0 + k;
    // this wave's copies of order k have landed; after the barrier every
    // wave's have, and every wave has read order k - 1's set (refilled next)
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (k + 1 < K) stage(k + 1, Pl + ((k + 1) & 1) * G::BUF);
    const __bf16* cur = Pl + (k & 1) * G::BUF;
    auto operand = [&](int o) {
      X3 r;
      r.h = *(const bf8*)(cur + o);
      r.m = *(const bf8*)(cur + G::PS + o);
      r.l = *(const bf8*)(cur + 2 * G::PS + o);
      return r;
    };
    mf4 acc[2] = {mf4{0.f, 0.f, 0.f, 0.f}, mf4{0.f, 0.f, 0.f, 0.f}};
    X3 bv = operand(obase);
#pragma unroll
    for (int q = 0; q <= S; ++q) {
      X3 bn;
      if (q < S) bn = operand(obase + QSTEP * (q + 1));
      // block rb at step q, block rb + 2 at step q - 1
      if (q >= 1 && q < S)
        mfma_x3_pair(T[q < S ? q : 0], bv, acc[0], T[q >= 1 ? q - 1 : 0], bv, acc[1]);
      else if (q < S)
        acc[0] = mfma_x3(T[q], bv, acc[0]);
      else
        acc[1] = mfma_x3(T[q >= 1 ? q - 1 : 0], bv, acc[1]);
      bv = bn;
    }
    const float in1 = p.inv_tab[n + 1];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) px.fold(4 * b + v, n, p.N, acc[b][v], in1);
  }
  if (fin) {
    float* out = p.dyn ? p.dyn->out : p.out;
    const int64_t out_pitch = p.dyn ? p.dyn->out_pitch : p.out_pitch;
    const double X = (double)p.X;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = pr0 + 32 * b + v;
        if (out && r < p.H && pc < p.Wd) {
          const double ratio = X * px.P[4 * b + v] / px.Q[4 * b + v];
          out[(int64_t)r * out_pitch + pc] = (float)((double)p.sigma_r * ratio + (double)p.center);
        }
      }
    return;
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int nr = pc < p.Wd ? max(0, min(4, p.H - (pr0 + 32 * b))) : 0;
    px.template store_part<4>(st, 4 * b, (int64_t)(pr0 + 32 * b) * p.Wd + pc, p.Wd, nr);
  }
}

template <int S>
static hipError_t cols_x3p_s(const TileParams& p, const LsState& st, int n0, int K, bool fin, hipStream_t s) {
  static bool attr = false;
  const int64_t lb = ls_cols_x3p_lds_bytes(p.W);
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)ls_cols_x3p_kernel<S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lb);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int grid = ((p.H + kX3pRows - 1) / kX3pRows) * ((p.Wd + kX3pCols - 1) / kX3pCols);
  hipLaunchKernelGGL((ls_cols_x3p_kernel<S>), dim3(grid), dim3(kX3sThreads), (size_t)lb, s, p, st, n0, K,
                     fin ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_cols_x3p(const TileParams& p, const LsState& st, int n0, int K, bool fin, hipStream_t s) {
  if (!st.Hs0 || !ls_split_supported(p.W, st.block) || (st.hs_plane + 512 * st.pitch) * 2 >= (1LL << 31) ||
      p.mirror)
    return hipErrorInvalidValue;
  switch (x3p_steps(p.W)) {
    case 1: return cols_x3p_s<1>(p, st, n0, K, fin, s);
    case 2: return cols_x3p_s<2>(p, st, n0, K, fin, s);
    case 3: return cols_x3p_s<3>(p, st, n0, K, fin, s);
    case 4: return cols_x3p_s<4>(p, st, n0, K, fin, s);
    case 5: return cols_x3p_s<5>(p, st, n0, K, fin, s);
    case 6: return cols_x3p_s<6>(p, st, n0, K, fin, s);
    case 7: return cols_x3p_s<7>(p, st, n0, K, fin, s);
    case 8: return cols_x3p_s<8>(p, st, n0, K, fin, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rows_x3_split(const TileParams& p, const LsState& st, int n0, int K, int src, int grid,
                                hipStream_t s) {
  if (!st.Hs0 || p.mirror) return hipErrorInvalidValue;
  return rows_x3_t<false, true>(p, st, n0, K, src, grid, s);
}

// one kernel per k-step count S = x3_steps(W) (W <= 120: S <= 8), the Toeplitz operands in registers
hipError_t launch_rows_x3(const TileParams& p, const LsState& st, int n0, int K, int src, int grid, hipStream_t s) {
  return rows_x3_t<false>(p, st, n0, K, src, grid, s);
}

hipError_t launch_cols_x3(const TileParams& p, const LsState& st, int n0, int K, bool save, int grid, hipStream_t s) {
  return save ? cols_x3_t<true, false>(p, st, n0, K, grid, s) : cols_x3_t<false, false>(p, st, n0, K, grid, s);
}

// Wide range (lambda = (T / sigma_r)^2 in (170, 1400]): the lift in float64
// (F~_0 = a~_0 = e^{-x^2/2}, x = (f - center) / sigma_r as in float32), the
// split passes with float64 states, and eq. (PbyQ) without the factor X.
__global__ __launch_bounds__(256) void wide_init_kernel(TileParams p, LsState st) {
  const int64_t npx = (int64_t)p.H * p.Wd;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < npx; i += (int64_t)gridDim.x * 256) {
    const int r = (int)(i / p.Wd), c = (int)(i - (int64_t)r * p.Wd);
    const float f = p.in[(int64_t)r * p.in_pitch + c];
    const float x = (f - p.center) / p.sigma_r;
    const double E = exp(-0.5 * (double)x * (double)x);
    const int64_t j = (int64_t)r * st.pitch + c;
    st.Fd[0][j] = E;
    st.Y[j] = x;
    st.ad[i] = E;  // a~_{-1} and the sums start at zero in the first block's column pass
    st.z[i] = x;
  }
}

hipError_t wide_launch_init(const TileParams& p, const LsState& st, hipStream_t s) {
  const int64_t npx = (int64_t)p.H * p.Wd;
  const int g1 = (int)std::min<int64_t>((npx + 255) / 256, 4096);
  hipLaunchKernelGGL(wide_init_kernel, dim3(g1), dim3(256), 0, s, p, st);
  return hipGetLastError();
}

hipError_t launch_rows_x3_wide(const TileParams& p, const LsState& st, int n0, int K, int src, hipStream_t s) {
  const int grow = ((p.H + kLsRows - 1) / kLsRows) * ((p.Wd + kLsCols - 1) / kLsCols);
  return rows_x3_t<true>(p, st, n0, K, src, grow, s);
}

bool ls_wide_supported(int W) {
  return ls_x3_supported(W) && ls_rows_x3_lds_bytes(W) <= max_lds_bytes() && ls_cols_x3_lds_bytes(W) <= max_lds_bytes();
}

hipError_t launch_forward_wide(const TileParams& p, const LsState& st, hipStream_t s) {
  if (p.H <= 0 || p.Wd <= 0) return hipSuccess;
  if (!p.wide || p.kt != BF_GAUSS || !ls_wide_supported(p.W) || !st.Fd[0] || !st.ad)
    return hipErrorInvalidValue;
  const int64_t npx = (int64_t)p.H * p.Wd;
  const int g1 = (int)std::min<int64_t>((npx + 255) / 256, 4096);
  hipLaunchKernelGGL(wide_init_kernel, dim3(g1), dim3(256), 0, s, p, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int grow = ((p.H + kLsRows - 1) / kLsRows) * ((p.Wd + kLsCols - 1) / kLsCols);
  const int gcols = ((p.H + 63) / 64) * ((p.Wd + kTileCols - 1) / kTileCols);
  int src = 0;
  for (int n0 = 0; n0 <= p.N; n0 += st.block) {
    const int K = std::min(st.block, p.N + 1 - n0);
    e = rows_x3_t<true>(p, st, n0, K, src, grow, s);
    if (e == hipSuccess)
      e = cols_x3_t<false, true>(p, st, n0, K, gcols, s);
    if (e != hipSuccess) return e;
    src ^= 1;
  }
  return ls_launch_final(p, st, s);
}

}  // namespace bfgpa
