// Spatial filtering on the matrix cores (the streamed passes, forward and
// adjoint).  A 1-D FIR over 16 consecutive outputs is a banded Toeplitz
// product: out[j] = sum_m x[m] tap[m - j], m = 0 .. 15 + 2W.
// v_mfma_f32_16x16x4f32 multiplies a 16x4 by a 4x16 float32 block (lane l
// holds A[l%16][l/16] and B[l/16][l%16]; the result D[4(l/16)+v][l%16] sits
// in accumulator v), so ceil((16 + 2W)/4) of them give a 16x16 block of
// outputs.  The Toeplitz operand, the same for every block, is one per-lane
// table in LDS: Tt[kk*64 + l] = tap[4kk + l/16 - l%16] (zero outside [0, 2W]).
// Along rows the staged image is the A operand and the table B; along
// columns the table is A and the staged image B.
#pragma once

#include <hip/hip_runtime.h>

#include "bf_device.h"
#include "bf_internal.h"

namespace bfgpa {

typedef float mf4 __attribute__((ext_vector_type(4)));

// k-steps of one 16x16 output block
__host__ __device__ inline int ls_kk(int W) { return (16 + 2 * W + 3) / 4; }

template <int NT>
__device__ __forceinline__ void fill_toeplitz(float* Tt, int W, const float* __restrict__ tz) {
  const int KK = ls_kk(W);
  for (int i = threadIdx.x; i < KK * 64; i += NT) {
    const int kk = i >> 6, l = i & 63;
    const int d = 4 * kk + (l >> 4) - (l & 15);
    Tt[i] = (d >= 0 && d <= 2 * W) ? tz[d] : 0.f;
  }
}

// Row products: NB blocks of 16 outputs at columns cbase + 16 bb of 16
// staged rows (row pitch `pitch`; output column c reads staged columns
// c .. c + 2W).  Operands of step kk + 1 are read from LDS while step kk's
// products run.
template <int NB>
__device__ __forceinline__ void toeplitz_rows(const float* L, int pitch, int cbase, const float* Tt, int KK,
                                              mf4 (&acc)[NB]) {
  const int lane = threadIdx.x & 63;
  const float* sa = L + (lane & 15) * pitch + (lane >> 4) + cbase;  // A[l%16][l/16]
  float tb = Tt[lane], a[NB];
#pragma unroll
  for (int bb = 0; bb < NB; ++bb) a[bb] = sa[bb * 16];
  for (int kk = 0; kk < KK; ++kk) {
    const int kn = min(kk + 1, KK - 1);
    const float tn = Tt[kn * 64 + lane];
    float an[NB];
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) an[bb] = sa[bb * 16 + 4 * kn];
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) acc[bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[bb], tb, acc[bb], 0, 0, 0);
    tb = tn;
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) a[bb] = an[bb];
  }
}

// Column products: NB blocks of 16 outputs at columns cbase + 16 bb and
// rows r0 .. r0 + 15 of a staged window S (row pitch `pitch`; output row r
// reads staged rows r .. r + 2W).
template <int NB>
__device__ __forceinline__ void toeplitz_cols(const float* S, int r0, int cbase, const float* Tt, int KK,
                                              mf4 (&acc)[NB], int pitch = 64) {
  const int lane = threadIdx.x & 63;
  const float* sb = S + (r0 + (lane >> 4)) * pitch + cbase + (lane & 15);  // B[l/16][l%16]
  float ta = Tt[lane], b[NB];
#pragma unroll
  for (int bb = 0; bb < NB; ++bb) b[bb] = sb[bb * 16];
  for (int kk = 0; kk < KK; ++kk) {
    const int kn = min(kk + 1, KK - 1);
    const float tn = Tt[kn * 64 + lane];
    float bn[NB];
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) bn[bb] = sb[4 * kn * pitch + bb * 16];
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) acc[bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ta, b[bb], acc[bb], 0, 0, 0);
    ta = tn;
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) b[bb] = bn[bb];
  }
}

// Row pitch of a staged 16 x (256 + 2W) window: the last k-step reads up to
// column 258 + 2W; twice an odd number keeps column reads conflict-free.
__host__ __device__ inline int ls_rows_pitch_mfma(int W) {
  const int need = 256 + 2 * W + 4;
  return (need % 4 == 2) ? need : need + 2;
}

// Staged rows of a 64-row column window: 64 outputs, the 2W halo and the
// last k-step's overhang, rounded to the 4 rows one wave moves at a time.
__host__ __device__ inline int ls_cols_rows(int W) { return (64 + 2 * W + 4 + 3) & ~3; }

// Copy `rows` rows x 64 columns (row pitch `pitch` floats, 16-byte aligned
// rows) into S (pitch 64) with direct-to-LDS loads: one wave instruction
// moves 4 rows (64 lanes x 16 bytes).  The caller's barrier waits for them.
template <int NT>
__device__ __forceinline__ void stage_rows_lds(const float* src, int64_t pitch, float* S, int rows) {
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const float* h = src + (int64_t)(lane >> 4) * pitch + (lane & 15) * 4;
  for (int g = wv; g < rows / 4; g += NT / 64)
    __builtin_amdgcn_global_load_lds(h + (int64_t)(4 * g) * pitch,
                                     (__attribute__((address_space(3))) void*)(S + g * 256), 16, 0, 0);
}

// As stage_rows_lds for a window of a row-filtered image laid out with W
// rows above the image (padded row R holds image row R - W), but with the
// rows outside the image taken from their reflections (mirror border).
template <int NT>
__device__ __forceinline__ void stage_rows_lds_mirror(const float* img, int64_t pitch, int R0, int c0, int W,
                                                      int H, float* S, int rows) {
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  for (int g = wv; g < rows / 4; g += NT / 64) {
    const int R = R0 + 4 * g + (lane >> 4);
    const int Rs = reflect_index(R - W, H) + W;
    __builtin_amdgcn_global_load_lds(img + (int64_t)Rs * pitch + c0 + (lane & 15) * 4,
                                     (__attribute__((address_space(3))) void*)(S + g * 256), 16, 0, 0);
  }
}

// Tile order for column passes: column bands four tiles wide, row-major
// inside a band, so the tiles resident on one XCD at a time form a tall
// block whose overlapping halos are served from its L2.
__device__ __forceinline__ void band_tile(int t, int tiles_x, int tiles_y, int& ty, int& tx) {
  constexpr int BW = 4;
  const int band = t / (BW * tiles_y);
  const int bx0 = band * BW;
  const int bw = min(BW, tiles_x - bx0);
  const int idx = t - band * BW * tiles_y;
  ty = idx / bw;
  tx = bx0 + (idx - ty * bw);
}

}  // namespace bfgpa
