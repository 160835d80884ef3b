// Internal declarations shared by the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bf_gpa.h"

namespace bfgpa {

// Threads per workgroup of every tile kernel: four wave64 waves.
constexpr int kThreads = 256;
// Output tile width: one wave's lanes span the 64 columns of a tile.
constexpr int kTileCols = 64;
// Zero padding on both sides of the tap array, so that the register-blocked
// FIR loops can index taps without bounds tests (>= largest block - 1).
constexpr int kTapPad = 16;
// Row pitch (floats) of the LDS buffer holding the first (row) pass: odd,
// so column-wise lane access and row-wise lane access are bank-conflict free.
constexpr int kHPitch = kTileCols + 1;

// Everything one tile of the fused forward / adjoint needs for one image.
struct TileParams {
  const float* in;      // device image
  float* out;           // device output (forward) or dL/din (adjoint)
  const float* gout;    // adjoint: dL/dout
  float* saved;         // forward: optional 3 planes; adjoint: the same, read
  int64_t in_pitch, out_pitch, gout_pitch;
  int64_t saved_plane;  // elements per plane (height * width)
  int H, Wd;            // image size
  int W;                // support half-width
  int N;                // order
  int kt;               // BF_BOX / BF_GAUSS
  int TY;               // tile rows (multiple of 4)
  int tiles_x;          // tiles per image row
  float sigma_r, inv_sigma_r, center;
  float inv_sigma_s3;   // 1 / sigma_s^3 (Gaussian sigma_s gradient)
  const float* s_tab;   // s_n = 1/r_n, n = 0..N+1 (s_0 = 0)
  const float* r_tab;   // r_n = M_n / M_{n-1}, n = 0..N+1 (r_0 = 0)
  const float* inv_tab; // 1/n, n = 0..N+1 (inv_0 = 0)
  const float* taps;    // kTapPad zeros, 2W+1 taps, kTapPad zeros
  const float* taps2;   // same layout, d^2 * tap (Gaussian sigma_s gradient)
};

// Kernel-shape variants (compile-time register budgets).
struct Variant {
  int opt;    // max output rows per thread (tile rows = 4 * opt)
  int mreg;   // max region pixels per thread
};

// Region (tile grown by W on every side) in LDS, in floats.
inline int region_pitch(int W) { return (kTileCols + 2 * W) | 1; }
inline int64_t region_floats(int TY, int W) {
  return (int64_t)(TY + 2 * W) * region_pitch(W);
}

// Launchers (bf_kernels.hip).  Return hipError_t.
hipError_t launch_forward(const TileParams& p, int variant, bool acc64, bool save,
                          hipStream_t s);
hipError_t launch_backward(const TileParams& p, int variant, bool sigs, double* partials,
                           double* grad_sigma, hipStream_t s);
int forward_variant_count();
Variant forward_variant(int v);
int backward_variant_count();
Variant backward_variant(int v);
int64_t forward_lds_bytes(int TY, int W);
int64_t backward_lds_bytes(int TY, int W, bool sigs);
int max_lds_bytes();

// Batch (bf_batch.hip)
struct BatchTile {
  int32_t image;
  int32_t r0, c0;
  int32_t pad;
};
hipError_t launch_batch_reset(int* counter, hipStream_t s);
hipError_t launch_batch_forward(const TileParams* d_params, const BatchTile* d_tiles,
                                int ntiles, int* counter, int grid, bool acc64,
                                hipStream_t s);
int batch_variant_mreg();
int batch_variant_opt();

// errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

// planning helpers (bf_plan.cpp)
double lambert_w0(double z);
double poisson_tail(int N, double lam);

}  // namespace bfgpa

// Plan layout (opaque to callers).
struct bf_plan {
  bf_params p;          // normalised parameters
  bf_plan_info info;
  int variant;          // forward kernel variant
  int bvariant;         // backward kernel variant
  int TY, bTY;          // forward / backward tile rows
  int device;
  float* d_const;       // tables + taps (device)
  int64_t tab_stride;   // floats per table
  float* d_work;        // recompute buffer for the adjoint (3 planes) or null
  double* d_partials;   // per-workgroup sigma-gradient partials
  int ntiles_b;         // backward tiles
};
