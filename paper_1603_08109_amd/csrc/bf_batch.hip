// Batched forward: many images of uneven size, each with its own sigma_s,
// sigma_r and N, in ONE persistent kernel launch.  Workgroups claim tiles
// from a device counter; the tile list is ordered by decreasing estimated
// cost (longest-processing-time first) so that the expensive tiles start
// early and the cheap ones fill the tail.  The copy of the per-call image
// pointers, the counter reset and the persistent kernel are captured once
// in a hipGraph and replayed by later calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "bf_device.h"
#include "bf_internal.h"

namespace bfgpa {

template <int OPT, int MREG, bool ACC64>
__global__ __launch_bounds__(kThreads) void gpa_batch_kernel(const TileParams* __restrict__ params,
                                                             const BatchTile* __restrict__ tiles,
                                                             int ntiles, int* counter) {
  extern __shared__ float lds[];
  __shared__ int s_idx;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= ntiles) break;  // every workgroup ends here once the list is drained
    const BatchTile bt = tiles[idx];
    const TileParams p = params[bt.image];
    if (p.kt == BF_BOX)
      forward_tile<BF_BOX, OPT, MREG, ACC64, false>(p, bt.r0, bt.c0, lds);
    else
      forward_tile<BF_GAUSS, OPT, MREG, ACC64, false>(p, bt.r0, bt.c0, lds);
  }
}

__global__ void batch_reset_kernel(int* counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

// Shapes the batch kernel is built in (opt, mreg); index = candidate variant.
static const Variant kBatchVariants[] = {{8, 20}, {8, 32}, {4, 48}, {4, 72}};
static constexpr int kNumBatchVariants = sizeof(kBatchVariants) / sizeof(kBatchVariants[0]);

template <int OPT, int MREG>
static hipError_t launch_batch_t(const TileParams* d_params, const BatchTile* d_tiles, int ntiles,
                                 int* counter, int grid, size_t lds, bool acc64, hipStream_t s) {
  if (acc64) {
    auto k = gpa_batch_kernel<OPT, MREG, true>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes() - 64);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, s, d_params, d_tiles, ntiles, counter);
  } else {
    auto k = gpa_batch_kernel<OPT, MREG, false>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes() - 64);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, s, d_params, d_tiles, ntiles, counter);
  }
  return hipGetLastError();
}

static hipError_t launch_batch_v(int v, const TileParams* d_params, const BatchTile* d_tiles,
                                 int ntiles, int* counter, int grid, size_t lds, bool acc64,
                                 hipStream_t s) {
  switch (v) {
    case 0: return launch_batch_t<8, 20>(d_params, d_tiles, ntiles, counter, grid, lds, acc64, s);
    case 1: return launch_batch_t<8, 32>(d_params, d_tiles, ntiles, counter, grid, lds, acc64, s);
    case 2: return launch_batch_t<4, 48>(d_params, d_tiles, ntiles, counter, grid, lds, acc64, s);
    default: return launch_batch_t<4, 72>(d_params, d_tiles, ntiles, counter, grid, lds, acc64, s);
  }
}

}  // namespace bfgpa

using namespace bfgpa;

// One launch shape for the whole batch.
struct BatchShape {
  int variant;                 // kBatchVariants index
  int wg_per_cu;               // persistent grid = CUs * wg_per_cu
  std::vector<int> TY;         // per-image tile rows
  std::vector<BatchTile> tiles;
  size_t lds;                  // dynamic LDS bytes
};

struct bf_batch {
  int count = 0;
  int device = 0;
  int num_cu = 256;
  bool acc64 = true;
  std::vector<bf_params> prm;
  std::vector<bf_plan_info> info;
  std::vector<int32_t> status;
  std::vector<TileParams> hp;         // per-image params (pointers patched per call)
  std::vector<BatchShape> cands;      // candidate launch shapes
  int chosen = 0;
  float* d_const = nullptr;
  TileParams* d_params = nullptr;
  BatchTile* d_tiles = nullptr;       // tiles of the chosen shape
  int ntiles = 0;
  int* d_counter = nullptr;
  TileParams* h_stage[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ev_used[2] = {false, false};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int slot = 0;
  std::string key;
};

namespace bfgpa {

static double tile_cost(const bf_params& p, const bf_plan_info& inf, int TY) {
  const double region = (double)(TY + 2 * p.W) * (kTileCols + 2 * p.W);
  const double fr = p.kernel == BF_BOX ? 3.0 : (2.0 * p.W + 1.0);
  const double per_n = 3.0 * region + fr * (TY + 2 * p.W) * kTileCols + fr * TY * kTileCols +
                       6.0 * TY * kTileCols;
  return (inf.N + 1.0) * per_n;
}

static bool build_shape(bf_batch* b, int v, int wg_per_cu, BatchShape* out) {
  const Variant vv = kBatchVariants[v];
  out->variant = v;
  out->wg_per_cu = wg_per_cu;
  out->TY.assign(b->count, 0);
  out->tiles.clear();
  int64_t lds = 0;
  std::vector<std::pair<double, BatchTile>> list;
  for (int i = 0; i < b->count; ++i) {
    if (b->status[i] < 0) continue;
    const bf_params& p = b->prm[i];
    const int TY = 4 * vv.opt;
    if (region_floats(TY, p.W) > (int64_t)kThreads * vv.mreg) return false;
    if (forward_lds_bytes(TY, p.W) > max_lds_bytes() - 64) return false;
    out->TY[i] = TY;
    lds = std::max(lds, forward_lds_bytes(TY, p.W));
    const double c = tile_cost(p, b->info[i], TY);
    for (int r0 = 0; r0 < p.height; r0 += TY)
      for (int c0 = 0; c0 < p.width; c0 += kTileCols) list.push_back({c, BatchTile{i, r0, c0, 0}});
  }
  std::stable_sort(list.begin(), list.end(),
                   [](const std::pair<double, BatchTile>& a, const std::pair<double, BatchTile>& b2) {
                     return a.first > b2.first;
                   });
  for (auto& e : list) out->tiles.push_back(e.second);
  out->lds = (size_t)lds;
  return true;
}

static std::string batch_key(const bf_batch* b) {
  // shape summary: count, total pixels, sum of N, max W, kernel mix
  int64_t px = 0, sn = 0;
  int maxw = 0, nbox = 0;
  for (int i = 0; i < b->count; ++i) {
    px += (int64_t)b->prm[i].height * b->prm[i].width;
    sn += b->info[i].N;
    maxw = std::max(maxw, b->prm[i].W);
    nbox += b->prm[i].kernel == BF_BOX;
  }
  std::ostringstream os;
  os << "gfx950/batch/" << b->count << "/" << px << "/" << sn << "/" << maxw << "/" << nbox << "/"
     << (b->acc64 ? 64 : 32);
  return os.str();
}

static int cache_lookup(const std::string& key) {
  const char* path = std::getenv("BF_TUNE_CACHE");
  if (!path || !*path) return -1;
  std::ifstream in(path);
  std::string k;
  int v;
  int found = -1;
  while (in >> k >> v)
    if (k == key) found = v;
  return found;
}

static void cache_store(const std::string& key, int v) {
  const char* path = std::getenv("BF_TUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream out(path, std::ios::app);
  out << key << " " << v << "\n";
}

static void destroy_graphs(bf_batch* b) {
  for (int k = 0; k < 2; ++k) {
    if (b->gexec[k]) hipGraphExecDestroy(b->gexec[k]);
    b->gexec[k] = nullptr;
  }
}

static int select_shape(bf_batch* b, int c) {
  const BatchShape& sh = b->cands[c];
  if (b->d_tiles) hipFree(b->d_tiles);
  b->d_tiles = nullptr;
  b->ntiles = (int)sh.tiles.size();
  if (b->ntiles > 0) {
    if (hipMalloc(&b->d_tiles, sh.tiles.size() * sizeof(BatchTile)) != hipSuccess)
      return fail(BF_ENOMEM, "hipMalloc batch tiles failed");
    if (hipMemcpy(b->d_tiles, sh.tiles.data(), sh.tiles.size() * sizeof(BatchTile),
                  hipMemcpyHostToDevice) != hipSuccess)
      return fail(BF_EHIP, "hipMemcpy batch tiles failed");
  }
  for (int i = 0; i < b->count; ++i) {
    b->hp[i].TY = sh.TY[i];
    b->hp[i].tiles_x = (b->prm[i].width + kTileCols - 1) / kTileCols;
  }
  destroy_graphs(b);
  b->chosen = c;
  return BF_OK;
}

// Fill the staging slot with this call's pointers (waiting until the
// slot's previous copy has been consumed).
static int stage(bf_batch* b, int k, const float* const* in, const int64_t* in_pitch,
                 float* const* out, const int64_t* out_pitch) {
  if (b->ev_used[k]) {
    if (hipEventSynchronize(b->ev[k]) != hipSuccess) return fail(BF_EHIP, "hipEventSynchronize");
  }
  for (int i = 0; i < b->count; ++i) {
    TileParams t = b->hp[i];
    if (b->status[i] >= 0) {
      if (!in[i] || !out[i]) return fail(BF_EINVAL, "NULL image pointer in batch");
      if (in_pitch[i] < b->prm[i].width || out_pitch[i] < b->prm[i].width)
        return fail(BF_EINVAL, "pitch smaller than width in batch");
      t.in = in[i];
      t.out = out[i];
      t.in_pitch = in_pitch[i];
      t.out_pitch = out_pitch[i];
    }
    b->h_stage[k][i] = t;
  }
  return BF_OK;
}

static int run_direct(bf_batch* b, int k, hipStream_t s, int grid) {
  const BatchShape& sh = b->cands[b->chosen];
  if (hipMemcpyAsync(b->d_params, b->h_stage[k], b->count * sizeof(TileParams), hipMemcpyHostToDevice,
                     s) != hipSuccess)
    return fail(BF_EHIP, "hipMemcpyAsync batch params");
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, b->d_counter);
  hipError_t e = launch_batch_v(sh.variant, b->d_params, b->d_tiles, b->ntiles, b->d_counter, grid,
                                sh.lds, b->acc64, s);
  if (e != hipSuccess) return fail(BF_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
  return BF_OK;
}

static int grid_of(const bf_batch* b) {
  const BatchShape& sh = b->cands[b->chosen];
  int g = b->num_cu * sh.wg_per_cu;
  return std::max(1, std::min(g, std::max(1, b->ntiles)));
}

}  // namespace bfgpa

extern "C" {

int bf_batch_plan(int32_t count, const bf_params* per_image, bf_batch_t** out) {
  if (!out) return fail(BF_EINVAL, "out is NULL");
  *out = nullptr;
  if (count <= 0 || !per_image) return fail(BF_EINVAL, "count must be > 0 with a parameter array");
  bf_batch* b = new (std::nothrow) bf_batch();
  if (!b) return fail(BF_ENOMEM, "host allocation failed");
  b->count = count;
  hipGetDevice(&b->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, b->device) == hipSuccess && prop.multiProcessorCount > 0)
    b->num_cu = prop.multiProcessorCount;
  b->acc64 = (per_image[0].flags & BF_FLAG_FP32_ACCUM) == 0;
  b->prm.resize(count);
  b->info.resize(count);
  b->status.assign(count, BF_OK);
  b->hp.resize(count);
  int warn = BF_OK;
  // per-image order and tables
  std::vector<std::vector<float>> tabs(count);
  std::vector<int64_t> offs(count, 0);
  int64_t total = 0;
  for (int i = 0; i < count; ++i) {
    bf_params pi = per_image[i];
    pi.flags &= ~BF_FLAG_GRAD;
    int st = bf_order(&pi, &b->info[i]);
    b->status[i] = st;
    if (st < 0) continue;
    if (st > 0) warn = st;
    // normalised copy (bf_order normalises internally; redo the defaults here)
    if (pi.kernel == BF_GAUSS && pi.W <= 0) pi.W = b->info[i].W;
    if (pi.T == 0.0) pi.T = 127.5;
    if (std::isnan(pi.center)) pi.center = pi.T;
    b->prm[i] = pi;
    if (((pi.flags & BF_FLAG_FP32_ACCUM) == 0) != b->acc64) {
      delete b;
      return fail(BF_EINVAL, "all images of a batch must use the same accumulation precision");
    }
    // tables: s, r, inv (N+2), taps (padded)
    const int N = b->info[i].N, W = pi.W;
    const double lam = b->info[i].lambda, X = std::sqrt(lam);
    auto logM = [&](int n) -> double {
      if (n == 0) return 0.0;
      if ((double)n <= lam) return 0.5 * n * (std::log((double)n) - 1.0);
      return -0.5 * lam + n * std::log(X);
    };
    const int64_t stride = ((N + 2 + 63) / 64) * 64;
    const int64_t ntap = ((2 * W + 1 + 2 * kTapPad + 63) / 64) * 64;
    std::vector<float>& h = tabs[i];
    h.assign(3 * stride + ntap, 0.0f);
    for (int n = 1; n <= N + 1; ++n) {
      const double r = std::exp(logM(n) - logM(n - 1));
      h[n] = (float)(1.0 / r);
      h[stride + n] = (float)r;
      h[2 * stride + n] = (float)(1.0 / n);
    }
    for (int a = -W; a <= W; ++a)
      h[3 * stride + kTapPad + a + W] =
          pi.kernel == BF_BOX ? 1.0f : (float)std::exp(-(double)a * a / (2.0 * pi.sigma_s * pi.sigma_s));
    offs[i] = total;
    total += (int64_t)h.size();
    TileParams& t = b->hp[i];
    std::memset(&t, 0, sizeof(t));
    t.H = pi.height;
    t.Wd = pi.width;
    t.W = W;
    t.N = N;
    t.kt = pi.kernel;
    t.sigma_r = (float)pi.sigma_r;
    t.inv_sigma_r = (float)(1.0 / pi.sigma_r);
    t.center = (float)pi.center;
    t.inv_T = (float)(1.0 / pi.T);
    t.X = (float)(pi.T / pi.sigma_r);
    (void)stride;
  }
  if (hipMalloc(&b->d_const, std::max<int64_t>(total, 1) * sizeof(float)) != hipSuccess) {
    delete b;
    return fail(BF_ENOMEM, "hipMalloc batch tables failed");
  }
  for (int i = 0; i < count; ++i) {
    if (b->status[i] < 0) continue;
    hipMemcpy(b->d_const + offs[i], tabs[i].data(), tabs[i].size() * sizeof(float), hipMemcpyHostToDevice);
    const int N = b->info[i].N;
    const int64_t stride = ((N + 2 + 63) / 64) * 64;
    TileParams& t = b->hp[i];
    t.s_tab = b->d_const + offs[i];
    t.r_tab = t.s_tab + stride;
    t.inv_tab = t.s_tab + 2 * stride;
    t.taps = t.s_tab + 3 * stride;
    t.taps2 = t.taps;
  }
  // candidate launch shapes
  for (int v = 0; v < kNumBatchVariants; ++v)
    for (int wg : {1, 2, 4}) {
      BatchShape sh;
      if (build_shape(b, v, wg, &sh)) b->cands.push_back(std::move(sh));
    }
  if (b->cands.empty()) {
    hipFree(b->d_const);
    delete b;
    return fail(BF_EUNSUPPORTED, "a batch image's support W is too large for the batch kernel");
  }
  if (hipMalloc(&b->d_params, count * sizeof(TileParams)) != hipSuccess ||
      hipMalloc(&b->d_counter, sizeof(int)) != hipSuccess) {
    hipFree(b->d_const);
    delete b;
    return fail(BF_ENOMEM, "hipMalloc batch buffers failed");
  }
  for (int k = 0; k < 2; ++k) {
    if (hipHostMalloc((void**)&b->h_stage[k], count * sizeof(TileParams), hipHostMallocDefault) != hipSuccess)
      return fail(BF_ENOMEM, "hipHostMalloc staging failed");
    hipEventCreateWithFlags(&b->ev[k], hipEventDisableTiming);
  }
  b->key = batch_key(b);
  // default shape: cached choice, else the first candidate with 2 workgroups per CU
  int c = cache_lookup(b->key);
  if (c < 0 || c >= (int)b->cands.size()) {
    c = 0;
    for (int i = 0; i < (int)b->cands.size(); ++i)
      if (b->cands[i].wg_per_cu == 2) { c = i; break; }
  }
  int st = select_shape(b, c);
  if (st < 0) return st;
  *out = b;
  return warn;
}

int bf_batch_status(const bf_batch_t* b, int32_t* per_image_status, int32_t* per_image_N) {
  if (!b) return fail(BF_EINVAL, "NULL batch");
  for (int i = 0; i < b->count; ++i) {
    if (per_image_status) per_image_status[i] = b->status[i];
    if (per_image_N) per_image_N[i] = b->status[i] >= 0 ? b->info[i].N : 0;
  }
  return BF_OK;
}

int bf_batch_forward(bf_batch_t* b, const float* const* in, const int64_t* in_pitch,
                     float* const* out, const int64_t* out_pitch, void* stream) {
  if (!b || !in || !out || !in_pitch || !out_pitch) return fail(BF_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const int k = b->slot;
  b->slot ^= 1;
  int st = stage(b, k, in, in_pitch, out, out_pitch);
  if (st < 0) return st;
  if (!b->gexec[k]) {
    // capture: params copy from this slot, counter reset, persistent kernel
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
      return fail(BF_EHIP, "hipStreamCreate");
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      int rs = run_direct(b, k, cap, grid_of(b));
      e = hipStreamEndCapture(cap, &graph);
      if (rs < 0) {
        if (graph) hipGraphDestroy(graph);
        hipStreamDestroy(cap);
        return rs;
      }
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec[k], graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    hipStreamDestroy(cap);
    if (e != hipSuccess) return fail(BF_EHIP, std::string("batch graph capture: ") + hipGetErrorString(e));
  }
  hipError_t e = hipGraphLaunch(b->gexec[k], s);
  if (e != hipSuccess) return fail(BF_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  hipEventRecord(b->ev[k], s);
  b->ev_used[k] = true;
  return BF_OK;
}

int bf_batch_tune(bf_batch_t* b, const float* const* in, const int64_t* in_pitch, float* const* out,
                  const int64_t* out_pitch, void* stream, int32_t* chosen) {
  if (!b || !in || !out || !in_pitch || !out_pitch) return fail(BF_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  float best = 1e30f;
  int bestc = b->chosen;
  for (int c = 0; c < (int)b->cands.size(); ++c) {
    int st = select_shape(b, c);
    if (st < 0) return st;
    const int k = b->slot;
    b->slot ^= 1;
    st = stage(b, k, in, in_pitch, out, out_pitch);
    if (st < 0) return st;
    // one warm-up, then three timed launches (direct, not graphed)
    run_direct(b, k, s, grid_of(b));
    hipEventRecord(e0, s);
    for (int rep = 0; rep < 3; ++rep) run_direct(b, k, s, grid_of(b));
    hipEventRecord(e1, s);
    hipEventRecord(b->ev[k], s);
    b->ev_used[k] = true;
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      bestc = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  int st = select_shape(b, bestc);
  if (st < 0) return st;
  cache_store(b->key, bestc);
  if (chosen) *chosen = bestc;
  return BF_OK;
}

int bf_batch_destroy(bf_batch_t* b) {
  if (!b) return BF_OK;
  for (int k = 0; k < 2; ++k)
    if (b->ev_used[k]) hipEventSynchronize(b->ev[k]);
  destroy_graphs(b);
  for (int k = 0; k < 2; ++k) {
    if (b->ev[k]) hipEventDestroy(b->ev[k]);
    if (b->h_stage[k]) hipHostFree(b->h_stage[k]);
  }
  if (b->d_const) hipFree(b->d_const);
  if (b->d_params) hipFree(b->d_params);
  if (b->d_tiles) hipFree(b->d_tiles);
  if (b->d_counter) hipFree(b->d_counter);
  delete b;
  return BF_OK;
}

}  // extern "C"
