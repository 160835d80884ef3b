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
// Row pitch (floats) of the LDS buffer holding the row-pass output.  The
// row pass writes it with lanes on consecutive rows, each lane a run of
// adjacent columns as pairs of dword accesses at any alignment: an odd pitch
// puts every dword of the wave's access on a distinct bank.
constexpr int kHPitch = kTileCols + 1;
// The adjoint tile keeps twice an odd number (the pitches the compiler pairs
// into 64-bit accesses there; measured 7% faster than the odd ones).
constexpr int kHPitchBwd = kTileCols + 2;
// Row-pass register blocks (outputs per work item) for the box and the FIR.
constexpr int kRowSegBoxHost = 16;
constexpr int kRowSegFirHost = 8;

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
  float inv_T;          // 1 / T: y = (f - center) / T, so |y| <= 1 on [center - T, center + T]
  float X;              // T / sigma_r
  float inv_sigma_s3;   // 1 / sigma_s^3 (Gaussian sigma_s gradient)
  const float* s_tab;   // s_n = 1/r_n, n = 0..N+1 (s_0 = 0)
  const float* r_tab;   // r_n = M_n / M_{n-1}, n = 0..N+1 (r_0 = 0)
  const float* inv_tab; // 1/n, n = 0..N+1 (inv_0 = 0)
  const float* taps;    // kTapPad zeros, 2W+1 taps, kTapPad zeros
  const float* taps2;   // same layout, d^2 * tap (Gaussian sigma_s gradient)
  const float* guide;   // cross filter: the image the range kernel acts on (else null)
  int64_t guide_pitch;
  int mirror;           // 1: reflecting border (BF_FLAG_MIRROR), 0: zero extension
  const float* rg_tab;  // recursive Gaussian: recursion coefficients and scan matrices (else null)
  int mfma_x3;          // streamed Gaussian: float32 products as split-bfloat16 matrix-core products
  int wide;             // wide range (T / sigma_r above 13): float64 per-pixel states, out = sigma_r P / Q + c
  const double* isq;    // 1 / sqrt(n), n = 0 .. N+1 (isq_0 = 0)
  const double* sq;     // sqrt(n), n = 0 .. N+1
  // Launches recorded once into a graph: when set, the streamed forward's
  // lift and final pass read in / in_pitch / out / out_pitch (and, with
  // dyn_save, saved) from this device copy of the call's parameters instead
  // of the by-value fields above, and the adjoint kernels read every image
  // pointer and gsig from it (with_dyn), so one capture serves every call.
  const TileParams* dyn;
  int dyn_save;
  double* gsig;         // adjoint through dyn: {dL/d sigma_r, dL/d sigma_s} of the call (device), or null
};

// lambda = (T / sigma_r)^2 limits: exp(-x^2/2) stays a normal float32 for
// lambda <= 170 and a normal float64 for lambda <= 1400 (x up to 37.4)
constexpr double kLambdaF32 = 170.0;
constexpr double kLambdaF64 = 1400.0;

// Large-support path: orders per block and its device state.
constexpr int kLsBlock = 64;       // most orders per block of the streamed passes (row-filtered images per state)
constexpr int kLsBlockSmall = 16;  // orders per block below 4 Mpx, for the box and the volume and recursive paths
constexpr int kLsRows = 16;   // image rows per streamed row-pass workgroup
constexpr int kLsCols = 256;  // output columns per streamed row-pass workgroup
struct LsState {
  int64_t pitch;            // row pitch (floats) of the image-shaped buffers
  float* F[2];              // F^ state images (double-buffered)
  float* Y;                 // y = (f - center) / T
  float* H0;                // row-filtered images (W zero rows above and below), image k at h(k)
  int64_t h_stride;         // floats from one row-filtered image to the next
  float *a, *ap, *app, *z;  // per-pixel coefficient recursion
  double *P, *Q, *DP, *DQ;  // per-pixel sums
  int64_t hbytes;           // bytes of one row-filtered image
  int64_t tpitch;           // recursive Gaussian: row pitch of the column-major filtered images
  float* HT0;               // recursive Gaussian: the row-filtered images, column-major, image k at ht(k)
  int64_t ht_stride;
  double* Fd[2];            // wide range: F~_n = e^{-x^2/2} x^n / sqrt(n!) images (double-buffered)
  double *ad, *apd;         // wide range: per-pixel a~_n, a~_{n-1}
  uint16_t* Hs0;            // pre-split row-filtered images (ls_split_rows), or null: per image three
                            // bfloat16 planes of hs_plane elements, rows in groups of eight
                            // ([row / 8][column][row % 8], pitch columns); image k at hs(k)
  int64_t hs_stride;
  int64_t hs_plane;         // elements per plane of a pre-split image
  int block;                // orders per block: row-filtered images allocated (0: none, box strips)
  // The images of a block are equal-sized and consecutive, so base and stride
  // describe them: the struct stays small (about 200 bytes) as every streamed
  // launch takes it by value, and its pointers stay kernel-argument (global)
  // pointers to the compiler.
  __host__ __device__ float* h(int k) const { return H0 + k * h_stride; }
  __host__ __device__ float* ht(int k) const { return HT0 + k * ht_stride; }
  __host__ __device__ uint16_t* hs(int k) const { return Hs0 + k * hs_stride; }
};
static_assert(sizeof(LsState) <= 256, "every streamed launch takes the state by value");

// Rows of one row-filtered image of the streamed passes: the height padded
// to a multiple of 64, W zero rows above, and W + 40 zero rows below (a box
// window's entering row, and the overhang of a staged column window: the
// split-bfloat16 column pass stages up to 2W + 95 rows from a tile's first).
__host__ __device__ inline int64_t ls_hrows(int H, int W) { return (int64_t)((H + 63) / 64) * 64 + 2 * W + 40; }

// Rows of one pre-split row-filtered image: round_up(W, 8) zero rows above
// (image row i at row i + round_up(W, 8), so the row pass's runs of four rows
// stay inside a group of eight), the height rounded up to 16 (the row pass
// writes whole 16-row tiles; rows past the image are written as zeros).
// Reads past the last row return zeros (buffer loads with the plane's size).
__host__ __device__ inline int ls_split_top(int W) { return (W + 7) & ~7; }
__host__ __device__ inline int64_t ls_split_rows(int H, int W) { return ls_split_top(W) + (int64_t)((H + 15) / 16) * 16; }

// Streamed adjoint (supports too wide for the fused adjoint tiles): orders
// per block (kBlsBlock from 4 Mpx, kBlsBlockSmall below) and its device state.
constexpr int kBlsBlock = 32;
constexpr int kBlsBlockSmall = 8;
constexpr int kBlsPartials = 1024;  // workgroups of the final reduction pass
struct BlsState {
  int64_t pitch;               // row pitch (floats) of the image-shaped buffers
  float* A[2];                 // scaled coefficients a_m (double-buffered)
  float* B[2];                 // b_m = a_{m-1} r_m (double-buffered)
  float* R0;                   // row-filtered adjoint images with the taps, image k at r(k)
  float* R20;                  // with the d^2 taps (sigma_s gradient), image k at r2(k), or null
  int64_t r_stride;            // floats from one image to the next (equal-sized, consecutive)
  float *fc, *fp;              // F~_m and F~_{m-1} at each pixel
  double *dx, *dss;            // per-pixel sums of the image and sigma_s gradients
  int block;                   // orders per block (row-filtered images allocated per tap set)
  __host__ __device__ float* r(int k) const { return R0 + k * r_stride; }
  __host__ __device__ float* r2(int k) const { return R20 + k * r_stride; }
};
static_assert(sizeof(BlsState) <= 256, "every streamed adjoint launch takes the state by value");

// Kernel-shape variants (compile-time register budgets).
struct Variant {
  int opt;    // max output rows per thread (tile rows = 4 * opt)
  int mreg;   // max region pixels per thread
};

// Region (tile grown by W on every side) in LDS, in floats.  Row pitch is
// odd for the same reason as kHPitch (the row pass reads runs of adjacent
// columns with lanes on consecutive rows).
__host__ __device__ inline int region_pitch(int W) {
  const int rw = kTileCols + 2 * W;  // even
  return rw + 1;
}
inline int64_t region_floats(int TY, int W) {
  return (int64_t)(TY + 2 * W) * region_pitch(W);
}
// the adjoint tile's region pitch: twice an odd number, as kHPitchBwd
__host__ __device__ inline int region_pitch_bwd(int W) {
  const int rw = kTileCols + 2 * W;
  return (rw % 4 == 2) ? rw : rw + 2;
}
inline int64_t region_floats_bwd(int TY, int W) {
  return (int64_t)(TY + 2 * W) * region_pitch_bwd(W);
}

// Launchers (bf_kernels.hip).  Return hipError_t.
hipError_t launch_forward(const TileParams& p, int variant, bool acc64, bool save,
                          hipStream_t s);
// the fused forward (plain, or keeping the adjoint's state) compiled for a
// fixed support W = 1 .. 21 (bf_fused_w.hip)
bool fixed_w_available(int W, int variant);
hipError_t launch_forward_fixed_w(const TileParams& p, bool save, hipStream_t s);
// the fused adjoint tile compiled for a fixed support W = 1 .. 17 (its
// 16-row variant, the one the planner picks there; bf_fused_w_bwd.hip)
bool fixed_w_bwd_available(int W, int variant);
hipError_t launch_backward_fixed_w(const TileParams& p, bool sigs, double* partials, hipStream_t s);
hipError_t launch_backward(const TileParams& p, int variant, bool sigs, double* partials,
                           double* grad_sigma, hipStream_t s);
hipError_t launch_joint(const TileParams& p, int variant, hipStream_t s);
// Recursive Gaussian (BF_GAUSS_REC).  Table (floats): per oscillation j of
// the fit, at 8 j: a, a' (weights), Re q, Im q (pole q = rho e^{i theta});
// from 16: q_j^(8 m), m = 1 .. kRgPow, as (re, im) at 16 + 2 (kRgPow j + m - 1).
constexpr int kRgPow = 128;
constexpr int kRgTabFloats = 16 + 4 * kRgPow;
hipError_t launch_forward_rg(const TileParams& p, const LsState& st, hipStream_t s);
bool rg_supported(int H, int Wd);
int64_t rg_state_bytes(int H, int Wd);
LsState rg_layout(void* base, int H, int Wd);
void rg_table(double sigma_s, float* out);
double rg_w0(double sigma_s);

// streamed Gaussian passes with float32 emulated on the bfloat16 matrix cores (W <= 120)
bool ls_x3_supported(int W);
bool ls_wide_supported(int W);
hipError_t launch_forward_wide(const TileParams& p, const LsState& st, hipStream_t s);
// pieces of the wide-range sequence for the volume path: the float64 lift and one block's row pass
hipError_t wide_launch_init(const TileParams& p, const LsState& st, hipStream_t s);
hipError_t launch_rows_x3_wide(const TileParams& p, const LsState& st, int n0, int K, int src, hipStream_t s);
int64_t ls_rows_x3_lds_bytes(int W);
int64_t ls_cols_x3_lds_bytes(int W);
hipError_t launch_rows_x3(const TileParams& p, const LsState& st, int n0, int K, int src, int grid, hipStream_t s);
hipError_t launch_cols_x3(const TileParams& p, const LsState& st, int n0, int K, bool save, int grid, hipStream_t s);
hipError_t launch_cols_x3s(const TileParams& p, const LsState& st, int n0, int K, hipStream_t s);
int64_t ls_cols_x3s_lds_bytes(int W);
// plain forward on pre-split row-filtered images (st.Hs): the row pass writes its
// outputs split, the column pass stages the planes straight into LDS
hipError_t launch_rows_x3_split(const TileParams& p, const LsState& st, int n0, int K, int src, int grid,
                                hipStream_t s);
// fin: the block holds order N, and the pass writes eq. (PbyQ) in place of the state
hipError_t launch_cols_x3p(const TileParams& p, const LsState& st, int n0, int K, bool fin, hipStream_t s);

// pieces of the streamed sequence (an image of p.H rows)
hipError_t ls_launch_init(const TileParams& p, const LsState& st, hipStream_t s);
hipError_t ls_launch_rows(const TileParams& p, const LsState& st, int n0, int K, int src, hipStream_t s);
hipError_t ls_launch_final(const TileParams& p, const LsState& st, hipStream_t s);

// Video / volume data: D slices of Hs x Wd stacked as one image of D Hs rows.
constexpr int kVolMaxW = 32;
struct VolBufs {
  float* G[kLsBlockSmall];  // per order of a block (16 orders): the row- and column-filtered volume
};
int64_t vol_state_bytes(int D, int Hs, int Wd, int W, bool wide = false);
LsState vol_layout(void* base, int D, int Hs, int Wd, int W, VolBufs* g, bool wide = false);
hipError_t launch_forward_vol(const TileParams& p, const LsState& st, const VolBufs& g, int D, int Hs, hipStream_t s);

hipError_t launch_range(const float* in, int64_t pitch, int H, int Wd, float* mm, hipStream_t s);
int joint_variant_count();
Variant joint_variant(int v);
int64_t joint_lds_bytes(int TY, int W);
int forward_variant_count();
Variant forward_variant(int v);
int backward_variant_count();
Variant backward_variant(int v);
int64_t forward_lds_bytes(int TY, int W);
int64_t backward_lds_bytes(int TY, int W, bool sigs);
int max_lds_bytes();
// large-support path (bf_large.hip)
bool ls_supported(int W);
bool ls_box_strip_supported(int W);
// box column strips: columns per thread, output columns per strip, row-segment
// length, grid and LDS bytes on an H x Wd image
struct StripShape {
  int cpt, oc, seg_rows, grid;
  int kb;        // orders per launch (a tail block of at most 16 orders takes 16)
  int64_t lds;   // LDS bytes of the full block's kernel
};
StripShape ls_box_strip_shape(int H, int Wd, int W, bool save);
bool ls_mirror_supported(int kernel, int W);
// nblock: orders per block (row-filtered images in the state), ls_block_orders
int64_t ls_state_bytes(int H, int Wd, int W, bool save, bool wide = false, bool split = false,
                       int nblock = kLsBlockSmall);
LsState ls_layout(void* base, int H, int Wd, int W, bool save, bool wide = false, bool split = false,
                  int nblock = kLsBlockSmall);
int ls_block_orders(int H, int Wd, int kernel, int W);
bool ls_split_supported(int W, int nblock);
hipError_t launch_forward_ls(const TileParams& p, const LsState& st, bool save, hipStream_t s);
// plan-level helpers of the batch (bf_plan.cpp): the streamed forward of a
// single-image plan with the image pointers read from `dyn` (device memory)
hipError_t plan_forward_streamed_dyn(const bf_plan_t* pl, const TileParams* dyn, bool save, hipStream_t s);
// The adjoint of a single-image streamed plan with every pointer read from
// device parameters: fdyn (in, and saved as the recomputed state's
// destination; out null) for the forward recompute when `recompute`, adyn
// (in, gout, saved, out = dL/din or null, gsig or null) for the adjoint.
hipError_t plan_backward_streamed_dyn(const bf_plan_t* pl, const TileParams* fdyn, const TileParams* adyn,
                                      bool recompute, bool sigs, hipStream_t s);
// streamed adjoint (bf_large_bwd.hip)
bool bls_supported(int W, bool sigs);
int64_t bls_state_bytes(int H, int Wd, int W, bool sigs, int nblock = kBlsBlockSmall);
BlsState bls_layout(void* base, int H, int Wd, int W, bool sigs, int nblock = kBlsBlockSmall);
int bls_block_orders(int H, int Wd);
hipError_t launch_backward_ls(const TileParams& p, const BlsState& st, bool sigs, double* partials,
                              double* grad_sigma, hipStream_t s);
// out: the two sigma gradients, or (dyn set) dyn->gsig read when the kernel runs (null: nothing written)
hipError_t launch_sigma_reduce(const double* partials, int n, bool has_ss, double* out, const TileParams* dyn,
                               hipStream_t s);
// reflecting-border adjoint: extend (image by reflection, output gradient by zeros) by W on each
// side, and fold the extension's gradient back onto the image (bf_kernels.hip)
hipError_t launch_mirror_pad(const float* in, int64_t in_pitch, const float* gout, int64_t gout_pitch, int H, int Wd,
                             int W, float* fpad, float* gpad, hipStream_t s);
hipError_t launch_mirror_fold(const float* gpad, int H, int Wd, int W, float* gin, int64_t gin_pitch, hipStream_t s);

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

// Allocation-free forward (bf_noalloc.hip): the device address of the static
// table array on the current device, its capacity, and a fill of it from host
// values carried in kernel arguments.
int noalloc_capacity_floats();
hipError_t noalloc_scratch(float** out);
hipError_t noalloc_fill(float* dst, const float* h, int64_t n, hipStream_t s);

// errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

// planning helpers (bf_plan.cpp)
double lambert_w0(double z);
double poisson_tail(int N, double lam);
std::vector<double> taps1d(int kind, double sigma_s, int W);
void gpa_tables(double lam, int N, std::vector<double>& s, std::vector<double>& r, std::vector<double>& inv);
std::vector<float> const_tables(const bf_params& p, const bf_plan_info& info, int64_t* stride, int64_t* ntapr);
void bind_tables(TileParams& tp, const float* d, int64_t stride, int64_t ntapr);

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
  bool ls;              // large-support path (support too wide for the fused tiles)
  bool rec;             // recursive Gaussian (its state in d_ls / ls_state)
  bool wide;            // wide-range streamed Gaussian (its state in d_ls / ls_state)
  int depth;            // > 0: a volume plan of depth slices (its state in d_ls / ls_state, vol)
  bfgpa::VolBufs vol;
  void* d_ls;           // its device state
  bfgpa::LsState ls_state;
  bool bls;             // streamed adjoint
  void* d_bls;          // its device state
  bfgpa::BlsState bls_state;
  bf_plan* mirror_adj;  // reflecting border with BF_FLAG_GRAD: zero-border adjoint plan of the extended image
  float* d_mpad;        // its extended image, output gradient and input gradient (three planes)
  int64_t mpad_plane;   // floats per plane
};
