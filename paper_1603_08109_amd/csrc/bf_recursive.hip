// Algorithm 2 with the recursive (Deriche) Gaussian as the spatial filter:
// O(1) work per pixel and order whatever sigma_s (Sec. 1 and Sec. 3 cite
// this implementation of the Gaussian for the N+1 filterings).
//
// The 1-D filter sum_j h(|i - j|) x[j] over a whole zero-extended line is,
// per damped oscillation of the fit, a causal and an anticausal complex
// one-pole recursion (poles and weights from the host planner).  Lines are cut into chunks
// of 16 (rows) or 8 (columns) samples, one per thread:
//   1. each chunk runs both recursions from a zero state (with the true
//      neighbouring inputs), which gives its local end states;
//   2. the true states at every chunk boundary follow from a scan over the
//      chunks of the line, E_t = e_t + q^16 E_{t-1} (right to left for the
//      anticausal part), q the complex pole, with the powers q^(16 m) from
//      the host (Hillis-Steele steps by cross-lane shuffles inside a wave,
//      one LDS exchange of the waves' end states for longer lines);
//   3. each chunk reruns both recursions from its true states and adds them.
// This is the exact recursive filter of the whole line (no truncation).
//
// Per block of up to 16 orders:
//   rg_first     : a workgroup takes R image rows; F^_n for the block's orders
//                  by the power recursion in registers; each order's row
//                  filter is stored row-major;
//   rg_transpose : 64 x 64 tiles through LDS make them column-major, so
//   rg_second    : filters the transposed images along their rows (the image
//                  columns) with the same chunk scheme and folds each order
//                  into eqs. (P), (Q) of its pixels (per-pixel state
//                  column-major).
// rg_init and rg_final lift the input and form eq. (PbyQ), transposing
// through LDS tiles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>

#include "bf_device.h"
#include "bf_internal.h"

namespace bfgpa {

constexpr int kRgChunk = 16;          // samples per thread along a row (row pass)
constexpr int kRgChunk2 = 8;          // samples per thread along a column (column pass)
constexpr int kRgFirstThreads = 512;
constexpr int kRgSecondThreads = 1024;

struct RgCoef {
  float a[2], ap[2], qr[2], qi[2];
};

__device__ __forceinline__ RgCoef rg_coef(const float* __restrict__ tab) {
  RgCoef k;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    k.a[j] = tab[8 * j + 0];
    k.ap[j] = tab[8 * j + 1];
    k.qr[j] = tab[8 * j + 2];
    k.qi[j] = tab[8 * j + 3];
  }
  return k;
}

// q_j^(8 m), m = 1 .. 128, as (re, im)
__device__ __forceinline__ float2 rg_pow(const float* __restrict__ tab, int j, int m) {
  const float* z = tab + 16 + 2 * (kRgPow * j + m - 1);
  return make_float2(z[0], z[1]);
}

// e += z * s (complex, per oscillation j: components 2j, 2j+1)
__device__ __forceinline__ void cmad(float (&e)[4], int j, float2 z, float sr, float si) {
  e[2 * j] += z.x * sr - z.y * si;
  e[2 * j + 1] += z.y * sr + z.x * si;
}

// Threads of one line: Trp = Tr rounded up to a power of two (<= 64) or to a
// multiple of 64, so a line never shares a wave with another line's tail.
__host__ __device__ inline int rg_line_threads(int Tr) {
  if (Tr > 64) return (Tr + 63) & ~63;
  int p = 1;
  while (p < Tr) p <<= 1;
  return p;
}

// Per-lane transport factors of the cross-wave carries (constant per thread),
// for chunks of C samples.
struct RgLane {
  float2 in[2];   // q_j^(C (l + 1)): previous wave's end state -> after this chunk
  float2 out[2];  // q_j^(C (64 - l)): next wave's first state -> this chunk's first
};

template <int C>
__device__ __forceinline__ RgLane rg_lane(const float* __restrict__ tab, int l) {
  RgLane r;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    r.in[j] = rg_pow(tab, j, (C / 8) * (l + 1));
    r.out[j] = rg_pow(tab, j, (C / 8) * (64 - l));
  }
  return r;
}

// One chunk of a line: y[i] = sum_j h(|Ct + i - j|) x[j] over the whole line,
// xn = x[C] (the next chunk's first sample, 0 past the line).  Per
// oscillation of the fit, with q = rho e^{i theta}, the causal part is
// Re[(a - i a') w] with the complex one-pole recursion w[i] = q w[i-1] + x[i],
// the anticausal part Re[(a - i a') w'] with w'[i] = q (w'[i+1] + x[i+1]).
// (This rotation form keeps float32 rounding near 3e-7 of the output up to
// sigma_s = 100; the two-term real feedback 2 rho cos, -rho^2 of the same
// poles loses another decade through cancellation.)
// Chunk states are combined by a scan: in-wave Hillis-Steele steps through
// cross-lane shuffles, then, for lines longer than one wave (Trp > 64), the
// waves' end states through LDS (tot: 8 floats per wave of the line, one
// barrier).  Every thread of the workgroup calls it.
template <int C>
__device__ __forceinline__ void rg_filter_chunk(const float (&x)[C], float xn, float (&y)[C], int t, int Trp,
                                                const RgCoef& cf, const RgLane& ln, const float* __restrict__ tab,
                                                float* tot) {
  const int seg = min(Trp, 64);
  const int l = t & (seg - 1);

  // local states from zero: causal w after the chunk's last sample, anticausal
  // w' at its first; (re, im) per oscillation
  float e[4], b[4];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float qr = cf.qr[j], qi = cf.qi[j];
    float wr = 0.f, wi = 0.f;
#pragma unroll
    for (int i = 0; i < C; ++i) {
      const float nr = qr * wr - qi * wi + x[i];
      wi = qi * wr + qr * wi;
      wr = nr;
    }
    e[2 * j] = wr;
    e[2 * j + 1] = wi;
    wr = 0.f;
    wi = 0.f;
    float nx = xn;
#pragma unroll
    for (int i = C - 1; i >= 0; --i) {
      const float tr = wr + nx;
      wr = qr * tr - qi * wi;
      wi = qi * tr + qr * wi;
      nx = x[i];
    }
    b[2 * j] = wr;
    b[2 * j + 1] = wi;
  }

  // in-wave inclusive scans: E_t += q^(16 d) E_{t-d}, B_t += q^(16 d) B_{t+d}
  for (int d = 1; d < seg; d <<= 1) {
    float se[4], sb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      se[q] = __shfl_up(e[q], d);
      sb[q] = __shfl_down(b[q], d);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const float2 z = rg_pow(tab, j, (C / 8) * d);
      if (l >= d) cmad(e, j, z, se[2 * j], se[2 * j + 1]);
      if (l + d < seg) cmad(b, j, z, sb[2 * j], sb[2 * j + 1]);
    }
  }

  // across the waves of a line: true end state of the previous wave (ce) and
  // first state of the next (cb)
  float ce[4] = {0.f, 0.f, 0.f, 0.f}, cb[4] = {0.f, 0.f, 0.f, 0.f};
  if (Trp > 64) {
    const int nW = Trp >> 6, w = t >> 6;
    if (l == 63)
#pragma unroll
      for (int q = 0; q < 4; ++q) tot[8 * w + q] = e[q];
    if (l == 0)
#pragma unroll
      for (int q = 0; q < 4; ++q) tot[8 * w + 4 + q] = b[q];
    __syncthreads();
    for (int w2 = 0; w2 < w; ++w2) {
      float c[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) c[q] = tot[8 * w2 + q];
#pragma unroll
      for (int j = 0; j < 2; ++j) cmad(c, j, rg_pow(tab, j, 8 * C), ce[2 * j], ce[2 * j + 1]);
#pragma unroll
      for (int q = 0; q < 4; ++q) ce[q] = c[q];
    }
    for (int w2 = nW - 1; w2 > w; --w2) {
      float c[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) c[q] = tot[8 * w2 + 4 + q];
#pragma unroll
      for (int j = 0; j < 2; ++j) cmad(c, j, rg_pow(tab, j, 8 * C), cb[2 * j], cb[2 * j + 1]);
#pragma unroll
      for (int q = 0; q < 4; ++q) cb[q] = c[q];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cmad(e, j, ln.in[j], ce[2 * j], ce[2 * j + 1]);
      cmad(b, j, ln.out[j], cb[2 * j], cb[2 * j + 1]);
    }
  }
  // true states entering this chunk: E_{t-1} from the left, B_{t+1} from the right
  float ei[4], bi[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ei[q] = __shfl_up(e[q], 1);
    bi[q] = __shfl_down(b[q], 1);
    if (l == 0) ei[q] = ce[q];
    if (l == seg - 1) bi[q] = cb[q];
  }

  // both recursions from the true states
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float qr = cf.qr[j], qi = cf.qi[j], a = cf.a[j], ap = cf.ap[j];
    float wr = ei[2 * j], wi = ei[2 * j + 1];
#pragma unroll
    for (int i = 0; i < C; ++i) {
      const float nr = qr * wr - qi * wi + x[i];
      wi = qi * wr + qr * wi;
      wr = nr;
      const float u = a * wr + ap * wi;
      y[i] = j == 0 ? u : y[i] + u;
    }
    wr = bi[2 * j];
    wi = bi[2 * j + 1];
    float nx = xn;
#pragma unroll
    for (int i = C - 1; i >= 0; --i) {
      const float tr = wr + nx;
      wr = qr * tr - qi * wi;
      wi = qi * tr + qr * wi;
      nx = x[i];
      y[i] += a * wr + ap * wi;
    }
  }
}

typedef float rg_f4 __attribute__((ext_vector_type(4)));

// C floats at p (4 C-byte aligned), the first n kept, the rest zero
template <int C>
__device__ __forceinline__ void rg_load(const float* __restrict__ p, int n, float (&v)[C]) {
  const rg_f4* p4 = (const rg_f4*)p;
#pragma unroll
  for (int g = 0; g < C / 4; ++g) {
    const rg_f4 q = n > 0 ? p4[g] : rg_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < 4; ++u) v[4 * g + u] = (4 * g + u < n) ? q[u] : 0.f;
  }
}

// Row pass for orders n0 .. n0 + K - 1 of R image rows (blockDim = R * Trp,
// Tr = ceil(width / 16)); stores the row-filtered images row-major.
__global__ __launch_bounds__(kRgFirstThreads) void rg_first_kernel(TileParams p, LsState st, int K, int src, int R,
                                                                   int Tr, int Trp) {
  extern __shared__ float lds[];
  const int nW = Trp > 64 ? Trp >> 6 : 1;
  float* tot = lds;  // 2 (parity) x R x nW x 8
  const int tid = threadIdx.x;
  const int rr = tid / Trp, t = tid - (tid / Trp) * Trp;
  const int r = blockIdx.x * R + rr;
  const bool live = r < p.H && t < Tr;
  const RgCoef cf = rg_coef(p.rg_tab);
  const RgLane ln = rg_lane<kRgChunk>(p.rg_tab, t & 63);
  const float* Fin = st.F[src];
  const int c0 = kRgChunk * t;
  const int nok = live ? max(0, min(kRgChunk, p.Wd - c0)) : 0;
  const int64_t g0 = (int64_t)(live ? r : 0) * st.pitch + c0;
  float Fh[kRgChunk], Yh[kRgChunk];
  rg_load<kRgChunk>(Fin + g0, nok, Fh);
  rg_load<kRgChunk>(st.Y + g0, nok, Yh);
  // the next chunk's first sample follows the same power recursion
  const bool nxt = live && c0 + kRgChunk < p.Wd;
  float Fn = nxt ? Fin[g0 + kRgChunk] : 0.f;
  const float Yn = nxt ? st.Y[g0 + kRgChunk] : 0.f;
  for (int k = 0; k < K; ++k) {
    float y[kRgChunk];
    rg_filter_chunk<kRgChunk>(Fh, Fn, y, t, Trp, cf, ln, p.rg_tab, tot + (k & 1) * 8 * R * nW + 8 * nW * rr);
    float* Hk = st.h(k) + g0;
    if (nok == kRgChunk) {
#pragma unroll
      for (int g = 0; g < 4; ++g) ((rg_f4*)Hk)[g] = rg_f4{y[4 * g], y[4 * g + 1], y[4 * g + 2], y[4 * g + 3]};
    } else {
#pragma unroll
      for (int i = 0; i < kRgChunk; ++i)
        if (i < nok) Hk[i] = y[i];
    }
#pragma unroll
    for (int i = 0; i < kRgChunk; ++i) Fh[i] *= Yh[i];
    Fn *= Yn;
  }
  float* Fout = st.F[src ^ 1] + g0;
#pragma unroll
  for (int i = 0; i < kRgChunk; ++i)
    if (i < nok) Fout[i] = Fh[i];
}

// H[z] (row-major) -> HT[z] (column-major), 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void rg_transpose_kernel(LsState st, int H, int Wd) {
  __shared__ float T[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const float* src = st.h(blockIdx.z);
  float* dst = st.ht(blockIdx.z);
  for (int j = ty; j < 64; j += 4) {
    const int r = r0 + j, c = c0 + tx;
    if (r < H && c < Wd) T[j][tx] = src[(int64_t)r * st.pitch + c];
  }
  __syncthreads();
  for (int j = ty; j < 64; j += 4) {
    const int c = c0 + j, r = r0 + tx;
    if (r < H && c < Wd) dst[(int64_t)c * st.tpitch + r] = T[tx][j];
  }
}

// Column pass (rows of the transposed images) for orders n0 .. n0 + K - 1
// of R image columns (blockDim = R * Trp, Tr = ceil(height / 8)), folded
// into the per-pixel sums (column-major state).  Chunks of 8 samples keep
// the float64 sums of a thread's pixels within 128 VGPRs.
__global__ __launch_bounds__(kRgSecondThreads) void rg_second_kernel(TileParams p, LsState st, int n0, int K, int R,
                                                                     int Tr, int Trp) {
  constexpr int C = kRgChunk2;
  extern __shared__ float lds[];
  const int nW = Trp > 64 ? Trp >> 6 : 1;
  float* tot = lds;  // 2 (parity) x R x nW x 8
  const int tid = threadIdx.x;
  const int rr = tid / Trp, t = tid - (tid / Trp) * Trp;
  const int c = blockIdx.x * R + rr;
  const bool live = c < p.Wd && t < Tr;
  const int r0 = C * t;
  const int nok = live ? max(0, min(C, p.H - r0)) : 0;
  const bool nxt = live && r0 + C < p.H;
  const int64_t i0 = (int64_t)c * p.H + r0;
  const RgCoef cf = rg_coef(p.rg_tab);
  const RgLane ln = rg_lane<C>(p.rg_tab, t & 63);
  LsPix<C, false> px;
  px.load(st, nok > 0 ? i0 : 0, 1, nok, n0 == 0);
  const int64_t hoff = (int64_t)(live ? c : 0) * st.tpitch + r0;
  float xn[C];
  float nn = 0.f;
  rg_load<C>(st.ht(0) + hoff, nok, xn);
  if (nxt) nn = st.ht(0)[hoff + C];
  for (int k = 0; k < K; ++k) {
    float x[C], y[C];
#pragma unroll
    for (int i = 0; i < C; ++i) x[i] = xn[i];
    const float xnext = nn;
    if (k + 1 < K) {
      rg_load<C>(st.ht(k + 1) + hoff, nok, xn);
      if (nxt) nn = st.ht(k + 1)[hoff + C];
    }
    rg_filter_chunk<C>(x, xnext, y, t, Trp, cf, ln, p.rg_tab, tot + (k & 1) * 8 * R * nW + 8 * nW * rr);
    const int n = n0 + k;
    const float in1 = p.inv_tab[n + 1];
#pragma unroll
    for (int i = 0; i < C; ++i) px.fold(i, n, p.N, y[i], in1);
  }
  px.store(st, i0, 1, nok);
}

// F^_0 = e^{-x^2/2} and y (row-major), a_0, z and zero sums (column-major).
__global__ __launch_bounds__(256) void rg_init_kernel(TileParams p, LsState st) {
  __shared__ float Ta[32][33], Tz[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  for (int j = ty; j < 32; j += 8) {
    const int r = r0 + j, c = c0 + tx;
    if (r < p.H && c < p.Wd) {
      const float f = p.in[(int64_t)r * p.in_pitch + c];
      const float x = (f - p.center) / p.sigma_r;
      const float E = expf(-0.5f * x * x);
      st.F[0][(int64_t)r * st.pitch + c] = E;
      st.Y[(int64_t)r * st.pitch + c] = (f - p.center) * p.inv_T;
      Ta[j][tx] = E;
      Tz[j][tx] = x * p.X;
    }
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int c = c0 + j, r = r0 + tx;
    if (r < p.H && c < p.Wd) {
      const int64_t i = (int64_t)c * p.H + r;
      st.a[i] = Ta[tx][j];  // a_{-1} and the sums start at zero in the first block
      st.z[i] = Tz[tx][j];
    }
  }
}

// eq. (PbyQ) from the column-major sums, stored row-major.
__global__ __launch_bounds__(256) void rg_final_kernel(TileParams p, LsState st) {
  __shared__ float To[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const double X = (double)p.X;
  for (int j = ty; j < 32; j += 8) {
    const int c = c0 + j, r = r0 + tx;
    if (r < p.H && c < p.Wd) {
      const int64_t i = (int64_t)c * p.H + r;
      const double ratio = X * st.P[i] / st.Q[i];
      To[tx][j] = (float)((double)p.sigma_r * ratio + (double)p.center);
    }
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int r = r0 + j, c = c0 + tx;
    if (r < p.H && c < p.Wd) p.out[(int64_t)r * p.out_pitch + c] = To[j][tx];
  }
}

bool rg_supported(int H, int Wd) {
  return rg_line_threads((Wd + kRgChunk - 1) / kRgChunk) <= kRgFirstThreads &&
         rg_line_threads((H + kRgChunk2 - 1) / kRgChunk2) <= kRgSecondThreads;
}

int64_t rg_state_bytes(int H, int Wd) {
  const int64_t pitch = ((Wd + 63) / 64) * 64;
  const int64_t tpitch = ((H + 15) / 16) * 16;
  const int64_t npx = (int64_t)H * Wd;
  return 3 * (pitch * H * 4 + 256) + kLsBlockSmall * (pitch * H * 4 + 256) + kLsBlockSmall * ((int64_t)Wd * tpitch * 4 + 256) +
         3 * (npx * 4 + 256) + 2 * (npx * 8 + 256);
}

LsState rg_layout(void* base, int H, int Wd) {
  LsState st;
  std::memset(&st, 0, sizeof(st));
  st.block = kLsBlockSmall;
  const int64_t pitch = ((Wd + 63) / 64) * 64;
  const int64_t tpitch = ((H + 15) / 16) * 16;
  const int64_t npx = (int64_t)H * Wd;
  char* q = (char*)base;
  auto take = [&](int64_t bytes) {
    char* r = q;
    q += (bytes + 255) & ~255LL;
    return (void*)r;
  };
  st.pitch = pitch;
  st.tpitch = tpitch;
  st.F[0] = (float*)take(pitch * H * 4);
  st.F[1] = (float*)take(pitch * H * 4);
  st.Y = (float*)take(pitch * H * 4);
  st.h_stride = ((pitch * H * 4 + 255) & ~255LL) / 4;
  st.H0 = (float*)take(kLsBlockSmall * 4 * st.h_stride);
  st.ht_stride = (((int64_t)Wd * tpitch * 4 + 255) & ~255LL) / 4;
  st.HT0 = (float*)take(kLsBlockSmall * 4 * st.ht_stride);
  st.a = (float*)take(npx * 4);
  st.ap = (float*)take(npx * 4);
  st.z = (float*)take(npx * 4);
  st.P = (double*)take(npx * 8);
  st.Q = (double*)take(npx * 8);
  st.hbytes = (int64_t)Wd * tpitch * 4;
  return st;
}

// Lines per workgroup: as many as fit the thread limit, but few enough that
// the grid has about 256 workgroups or more.
static int rg_lines_per_group(int Trp, int max_threads, int lines) {
  int R = 1;
  while (2 * R * Trp <= max_threads && 2 * R * 256 <= lines) R *= 2;
  return R;
}

hipError_t launch_forward_rg(const TileParams& p, const LsState& st, hipStream_t s) {
  if (p.H <= 0 || p.Wd <= 0) return hipSuccess;
  if (!rg_supported(p.H, p.Wd) || !p.rg_tab) return hipErrorInvalidValue;
  const int Tr1 = (p.Wd + kRgChunk - 1) / kRgChunk, Trp1 = rg_line_threads(Tr1);
  const int Tr2 = (p.H + kRgChunk2 - 1) / kRgChunk2, Trp2 = rg_line_threads(Tr2);
  const int R1 = rg_lines_per_group(Trp1, kRgFirstThreads, p.H);
  const int R2 = rg_lines_per_group(Trp2, kRgSecondThreads, p.Wd);
  const int nW1 = Trp1 > 64 ? Trp1 / 64 : 1, nW2 = Trp2 > 64 ? Trp2 / 64 : 1;
  const size_t lds1 = (size_t)(16 * R1 * nW1) * 4;
  const size_t lds2 = (size_t)(16 * R2 * nW2) * 4;
  const dim3 tiles((p.Wd + 31) / 32, (p.H + 31) / 32);
  hipLaunchKernelGGL(rg_init_kernel, tiles, dim3(256), 0, s, p, st);
  int src = 0;
  for (int n0 = 0; n0 <= p.N; n0 += kLsBlockSmall) {
    const int K = std::min(kLsBlockSmall, p.N + 1 - n0);
    hipLaunchKernelGGL(rg_first_kernel, dim3((p.H + R1 - 1) / R1), dim3(R1 * Trp1), lds1, s, p, st, K, src, R1, Tr1,
                       Trp1);
    hipLaunchKernelGGL(rg_transpose_kernel, dim3((p.Wd + 63) / 64, (p.H + 63) / 64, K), dim3(256), 0, s, st, p.H,
                       p.Wd);
    hipLaunchKernelGGL(rg_second_kernel, dim3((p.Wd + R2 - 1) / R2), dim3(R2 * Trp2), lds2, s, p, st, n0, K, R2, Tr2,
                       Trp2);
    src ^= 1;
  }
  hipLaunchKernelGGL(rg_final_kernel, tiles, dim3(256), 0, s, p, st);
  return hipGetLastError();
}

}  // namespace bfgpa
