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

template <int OPT, int MREG, bool ACC64, bool SAVE>
__global__ __launch_bounds__(kThreads, (OPT * MREG <= 256 ? 2 : 1)) void gpa_batch_kernel(const TileParams* __restrict__ params,
                                                             const BatchTile* __restrict__ tiles,
                                                             int ntiles, int* counter) {
  extern __shared__ float lds[];
  __shared__ int s_idx;
  for (;;) {
    // The barrier in front of the claim keeps the compiler from merging this
    // thread-0 branch with one at the end of the previous tile across the
    // loop latch (which would leave the claim outside the loop that holds
    // the barriers).  The claimed index is made wave-uniform, so the exit
    // test and the tile's parameters are scalar.
    __syncthreads();
    if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
    __syncthreads();
    const int idx = __builtin_amdgcn_readfirstlane(s_idx);
    if (idx >= ntiles) break;  // every workgroup ends here once the list is drained
    const BatchTile bt = tiles[idx];
    const TileParams p = params[__builtin_amdgcn_readfirstlane(bt.image)];
    if (p.kt == BF_BOX)
      forward_tile<BF_BOX, OPT, MREG, ACC64, SAVE>(p, bt.r0, bt.c0, lds);
    else
      forward_tile<BF_GAUSS, OPT, MREG, ACC64, SAVE>(p, bt.r0, bt.c0, lds);
  }
}

// Batched adjoint: the same persistent scheme over adjoint tiles.  Each
// tile writes its two sigma-gradient sums to its own slot (BatchTile::pad),
// so the per-image sums below run in a fixed order.
template <int OPT, int MREG>
__global__ __launch_bounds__(kThreads) void gpa_batch_backward_kernel(const TileParams* __restrict__ params,
                                                                      const BatchTile* __restrict__ tiles,
                                                                      int ntiles, int* counter,
                                                                      double* partials) {
  extern __shared__ float lds[];
  __shared__ double red[2 * kThreads];
  __shared__ int s_idx;
  for (;;) {
    // as in gpa_batch_kernel: barrier before the claim, wave-uniform index
    __syncthreads();
    if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
    __syncthreads();
    const int idx = __builtin_amdgcn_readfirstlane(s_idx);
    if (idx >= ntiles) break;  // every workgroup ends here once the list is drained
    const BatchTile bt = tiles[idx];
    const TileParams p = params[__builtin_amdgcn_readfirstlane(bt.image)];
    double* part = partials + 2 * (int64_t)__builtin_amdgcn_readfirstlane(bt.pad);
    if (p.kt == BF_BOX)
      backward_tile<BF_BOX, OPT, MREG, false>(p, bt.r0, bt.c0, lds, red, part);
    else
      backward_tile<BF_GAUSS, OPT, MREG, true>(p, bt.r0, bt.c0, lds, red, part);
  }
}

// Per-image sums of the adjoint tiles' partials (one workgroup per image;
// n < 0 marks an image whose gradients are produced elsewhere).
struct BatchRed {
  int32_t off, n, has_ss, pad;
};

__global__ __launch_bounds__(kThreads) void batch_sigma_reduce_kernel(const double* partials,
                                                                      const BatchRed* info, const TileParams* gp) {
  __shared__ double red[2][kThreads];
  const BatchRed bi = info[blockIdx.x];
  double* out = gp[blockIdx.x].gsig;  // this call's destination of image blockIdx.x (or null)
  if (bi.n < 0 || !out) return;       // uniform per workgroup
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < bi.n; i += kThreads) {
    a += partials[2 * (int64_t)(bi.off + i)];
    b += partials[2 * (int64_t)(bi.off + i) + 1];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0][0];
    out[1] = bi.has_ss ? red[1][0] : __builtin_nan("");
  }
}

__global__ void batch_reset_kernel(int* counter) {
  if (threadIdx.x < 2) counter[threadIdx.x] = 0;
}

// Shapes the batch kernel is built in (opt, mreg); index = candidate variant.
static const Variant kBatchVariants[] = {{8, 20}, {8, 32}, {4, 48}, {4, 72}};
static constexpr int kNumBatchVariants = sizeof(kBatchVariants) / sizeof(kBatchVariants[0]);

template <int OPT, int MREG, bool ACC64, bool SAVE>
static hipError_t launch_batch_k(const TileParams* d_params, const BatchTile* d_tiles, int ntiles,
                                 int* counter, int grid, size_t lds, hipStream_t s) {
  auto k = gpa_batch_kernel<OPT, MREG, ACC64, SAVE>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     max_lds_bytes() - 64);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, s, d_params, d_tiles, ntiles, counter);
  return hipGetLastError();
}

template <int OPT, int MREG>
static hipError_t launch_batch_t(const TileParams* d_params, const BatchTile* d_tiles, int ntiles,
                                 int* counter, int grid, size_t lds, bool acc64, bool save, hipStream_t s) {
  if (acc64)
    return save ? launch_batch_k<OPT, MREG, true, true>(d_params, d_tiles, ntiles, counter, grid, lds, s)
                : launch_batch_k<OPT, MREG, true, false>(d_params, d_tiles, ntiles, counter, grid, lds, s);
  return save ? launch_batch_k<OPT, MREG, false, true>(d_params, d_tiles, ntiles, counter, grid, lds, s)
              : launch_batch_k<OPT, MREG, false, false>(d_params, d_tiles, ntiles, counter, grid, lds, s);
}

static hipError_t launch_batch_v(int v, const TileParams* d_params, const BatchTile* d_tiles,
                                 int ntiles, int* counter, int grid, size_t lds, bool acc64, bool save,
                                 hipStream_t s) {
  switch (v) {
    case 0: return launch_batch_t<8, 20>(d_params, d_tiles, ntiles, counter, grid, lds, acc64, save, s);
    case 1: return launch_batch_t<8, 32>(d_params, d_tiles, ntiles, counter, grid, lds, acc64, save, s);
    case 2: return launch_batch_t<4, 48>(d_params, d_tiles, ntiles, counter, grid, lds, acc64, save, s);
    default: return launch_batch_t<4, 72>(d_params, d_tiles, ntiles, counter, grid, lds, acc64, save, s);
  }
}

// Adjoint tile shapes: the single-image adjoint's variants (backward_variant).
template <int OPT, int MREG>
static hipError_t launch_batch_bwd_t(const TileParams* d_params, const BatchTile* d_tiles, int ntiles,
                                     int* counter, double* partials, int grid, size_t lds, hipStream_t s) {
  auto k = gpa_batch_backward_kernel<OPT, MREG>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     max_lds_bytes() - 2 * kThreads * 8 - 64);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, s, d_params, d_tiles, ntiles, counter, partials);
  return hipGetLastError();
}

static hipError_t launch_batch_bwd(int v, const TileParams* d_params, const BatchTile* d_tiles, int ntiles,
                                   int* counter, double* partials, int grid, size_t lds, hipStream_t s) {
  const Variant vv = backward_variant(v);
  if (vv.opt == 4 && vv.mreg == 20)
    return launch_batch_bwd_t<4, 20>(d_params, d_tiles, ntiles, counter, partials, grid, lds, s);
  if (vv.opt == 8 && vv.mreg == 24)
    return launch_batch_bwd_t<8, 24>(d_params, d_tiles, ntiles, counter, partials, grid, lds, s);
  if (vv.opt == 4 && vv.mreg == 32)
    return launch_batch_bwd_t<4, 32>(d_params, d_tiles, ntiles, counter, partials, grid, lds, s);
  return hipErrorInvalidValue;
}

}  // namespace bfgpa

using namespace bfgpa;

// One launch shape for the whole batch.
struct BatchShape {
  int variant;                 // kBatchVariants index
  int wg_per_cu;               // persistent grid = CUs * wg_per_cu
  std::vector<int> TY;         // per-image tile rows (0: the image runs a streamed plan of its own)
  std::vector<BatchTile> tiles;  // the persistent launch's tiles, cost-ordered
  size_t lds;                  // dynamic LDS bytes (the largest need of the persistent images)
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
  BatchTile* d_ftiles = nullptr;      // the chosen shape's tiles (images not on a plan of their own)
  int nftiles = 0;
  int64_t graph_launches = 0;         // hipGraphLaunch calls made by bf_batch_forward
  int64_t direct_launches = 0;        // launch sequences bf_batch_forward issued outside its graph
  int64_t own_bytes = 0;              // device bytes of the batch's own buffers
  std::vector<bf_plan_t*> fplans;     // images whose plain forward runs the streamed passes of a plan of their own
  static constexpr int kAux = 4;      // side streams for those images, concurrent with the persistent launch
  std::vector<int> aux_imgs[kAux];    // images per side stream (longest first, least-loaded stream)
  hipStream_t aux[kAux] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kAux] = {};
  int* d_counter = nullptr;
  TileParams* h_stage[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ev_used[2] = {false, false};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int slot = 0;
  std::string key;
  // adjoint (planned when an image asks for BF_FLAG_GRAD)
  bool grad = false;
  int bvariant = -1;                  // adjoint tile variant of the fused images
  size_t blds = 0;                    // its dynamic LDS bytes
  std::vector<int> bTY;               // per-image adjoint tile rows (0: streamed adjoint)
  std::vector<int> streamed;          // images on the streamed adjoint
  BatchTile* d_btiles = nullptr;      // adjoint tiles, cost-ordered
  int nbtiles = 0;
  double* d_bpartials = nullptr;      // two sums per adjoint tile
  BatchRed* d_bred = nullptr;         // per-image partial ranges
  float* d_saved = nullptr;           // forward state (3 planes per image)
  std::vector<int64_t> saved_off;
  TileParams* d_bparams = nullptr;    // forward-with-state params, then adjoint params
  TileParams* h_bstage = nullptr;     // pinned staging of d_bparams
  hipEvent_t bev = nullptr;
  bool bev_used = false;
  hipGraphExec_t bgexec[4] = {};      // captured adjoints: [saved given | 2 * sigma gradients asked]
  int64_t bgraph_launches = 0;        // hipGraphLaunch calls made by the batch adjoint
  int64_t bdirect_launches = 0;       // adjoint sequences issued outside a graph
  void* d_bls = nullptr;              // streamed adjoint state, reused image by image
  double* d_bls_partials = nullptr;
  std::vector<int> mirrored;          // images with the reflecting border: adjoint through their own plan
  std::vector<bool> own_adj;          // images whose adjoint runs on their own streamed plan (fplans)
  std::vector<bf_plan_t*> mplans;     // those plans (per image, null elsewhere)
};

namespace bfgpa {

static double tile_cost(const bf_params& p, const bf_plan_info& inf, int TY) {
  const double region = (double)(TY + 2 * p.W) * (kTileCols + 2 * p.W);
  const double fr = p.kernel == BF_BOX ? 3.0 : (2.0 * p.W + 1.0);
  const double per_n = 3.0 * region + fr * (TY + 2 * p.W) * kTileCols + fr * TY * kTileCols +
                       6.0 * TY * kTileCols;
  return (inf.N + 1.0) * per_n;
}

// A launch shape of the persistent kernel over the images that run no
// streamed plan of their own: every such image must fit the variant's
// register and LDS budget; the images on their own plans are left out of the
// fit test and of the LDS size.
static bool build_shape(bf_batch* b, int v, int wg_per_cu, BatchShape* out) {
  const Variant vv = kBatchVariants[v];
  out->variant = v;
  out->wg_per_cu = wg_per_cu;
  out->TY.assign(b->count, 0);
  out->tiles.clear();
  int64_t lds = 0;
  std::vector<std::pair<double, BatchTile>> list;
  for (int i = 0; i < b->count; ++i) {
    if (b->status[i] < 0 || b->fplans[i]) continue;
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
  for (int k = 0; k < 4; ++k) {
    if (b->bgexec[k]) hipGraphExecDestroy(b->bgexec[k]);
    b->bgexec[k] = nullptr;
  }
}

static int select_shape(bf_batch* b, int c) {
  const BatchShape& sh = b->cands[c];
  if (b->d_ftiles) hipFree(b->d_ftiles);
  b->d_ftiles = nullptr;
  b->nftiles = (int)sh.tiles.size();
  if (!sh.tiles.empty()) {
    if (hipMalloc(&b->d_ftiles, sh.tiles.size() * sizeof(BatchTile)) != hipSuccess)
      return fail(BF_ENOMEM, "hipMalloc batch tiles failed");
    if (hipMemcpy(b->d_ftiles, sh.tiles.data(), sh.tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice) !=
        hipSuccess)
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

// The tiles of images without a plan of their own; save: the staged params
// carry per-image saved planes, written as well.
static int run_direct(bf_batch* b, int k, hipStream_t s, int grid, bool save = false) {
  const BatchShape& sh = b->cands[b->chosen];
  if (hipMemcpyAsync(b->d_params, b->h_stage[k], b->count * sizeof(TileParams), hipMemcpyHostToDevice,
                     s) != hipSuccess)
    return fail(BF_EHIP, "hipMemcpyAsync batch params");
  if (b->nftiles == 0) return BF_OK;
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, b->d_counter);
  hipError_t e = launch_batch_v(sh.variant, b->d_params, b->d_ftiles, b->nftiles, b->d_counter, grid, sh.lds,
                                b->acc64, save, s);
  if (e != hipSuccess) return fail(BF_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
  return BF_OK;
}

// Side streams: fork them from `s` (they start after the work queued on `s` so far) and join
// them back into it (work queued on `s` afterwards waits for theirs).
static void fork_side(bf_batch* b, hipStream_t s) {
  hipEventRecord(b->fork_ev, s);
  for (int j = 0; j < bf_batch::kAux; ++j) hipStreamWaitEvent(b->aux[j], b->fork_ev, 0);
}

static void join_side(bf_batch* b, hipStream_t s) {
  for (int j = 0; j < bf_batch::kAux; ++j) {
    hipEventRecord(b->join_ev[j], b->aux[j]);
    hipStreamWaitEvent(s, b->join_ev[j], 0);
  }
}

// Adjoint planning: images whose support fits the fused adjoint tiles get
// adjoint tiles in one persistent work list (the shape that fits the most
// images); the others run the streamed adjoint one after another on a
// shared state buffer.  The forward state the adjoint reads (3 planes per
// image) is recomputed by the batch forward kernel at each call.  Images with
// the reflecting border run the adjoint of their own plan (bf_backward on the
// image extended by reflection) one after another.
static int plan_batch_adjoint(bf_batch* b) {
  const int count = b->count;
  b->mplans.assign(count, nullptr);
  for (int i = 0; i < count; ++i) {
    if (b->status[i] < 0 || !b->hp[i].mirror) continue;
    bf_params q = b->prm[i];
    q.flags |= BF_FLAG_GRAD;
    const int st = bf_plan(&q, &b->mplans[i]);
    if (st < 0) return st;
    if (b->mplans[i]->info.N != b->info[i].N || b->mplans[i]->info.W != b->prm[i].W)
      return fail(BF_EINVAL, "batch mirror adjoint: order or support differs from the batch plan");
    b->mirrored.push_back(i);
  }
  b->own_adj.assign(count, false);
  for (int i = 0; i < count; ++i)
    b->own_adj[i] = b->status[i] >= 0 && b->fplans[i] && !b->mplans[i];
  int best = -1, best_n = -1;
  for (int v = 0; v < backward_variant_count(); ++v) {
    const Variant vv = backward_variant(v);
    int n = 0;
    for (int i = 0; i < count; ++i) {
      if (b->status[i] < 0 || b->mplans[i] || b->own_adj[i]) continue;
      const int TY = 4 * vv.opt, W = b->prm[i].W;
      const bool sigs = b->prm[i].kernel == BF_GAUSS;
      if (region_floats_bwd(TY, W) <= (int64_t)kThreads * vv.mreg &&
          backward_lds_bytes(TY, W, sigs) + 2 * kThreads * 8 + 64 <= max_lds_bytes())
        ++n;
    }
    if (n > best_n) {
      best_n = n;
      best = v;
    }
  }
  b->bvariant = best;
  const Variant vv = backward_variant(best);
  b->bTY.assign(count, 0);
  std::vector<std::pair<double, BatchTile>> list;
  std::vector<BatchRed> red(count, BatchRed{0, -1, 0, 0});
  int slots = 0;
  int64_t lds = 0, bls_bytes = 0, saved = 0;
  b->saved_off.assign(count, 0);
  for (int i = 0; i < count; ++i) {
    if (b->status[i] < 0) continue;
    const bf_params& p = b->prm[i];
    const bool sigs = p.kernel == BF_GAUSS;
    b->saved_off[i] = saved;
    saved += 3 * (int64_t)p.height * p.width;
    if (b->mplans[i] || b->own_adj[i]) continue;
    const int TY = 4 * vv.opt;
    if (region_floats_bwd(TY, p.W) <= (int64_t)kThreads * vv.mreg &&
        backward_lds_bytes(TY, p.W, sigs) + 2 * kThreads * 8 + 64 <= max_lds_bytes()) {
      b->bTY[i] = TY;
      lds = std::max(lds, backward_lds_bytes(TY, p.W, sigs));
      const double c = 2.5 * tile_cost(p, b->info[i], TY);
      red[i] = BatchRed{slots, 0, sigs ? 1 : 0, 0};
      for (int r0 = 0; r0 < p.height; r0 += TY)
        for (int c0 = 0; c0 < p.width; c0 += kTileCols) {
          list.push_back({c, BatchTile{i, r0, c0, slots++}});
          red[i].n++;
        }
    } else {
      if (!bls_supported(p.W, sigs)) return fail(BF_EUNSUPPORTED, "a batch image's support W is too large for the adjoint");
      b->streamed.push_back(i);
      bls_bytes = std::max(bls_bytes, bls_state_bytes(p.height, p.width, p.W, sigs));
    }
  }
  std::stable_sort(list.begin(), list.end(),
                   [](const std::pair<double, BatchTile>& a, const std::pair<double, BatchTile>& c) {
                     return a.first > c.first;
                   });
  std::vector<BatchTile> tiles;
  for (auto& e : list) tiles.push_back(e.second);
  b->nbtiles = (int)tiles.size();
  b->blds = (size_t)lds;
  auto dev_alloc = [&](void** ptr, size_t bytes) {
    b->own_bytes += (int64_t)std::max<size_t>(bytes, 16);
    return hipMalloc(ptr, std::max<size_t>(bytes, 16)) == hipSuccess;
  };
  if (!dev_alloc((void**)&b->d_btiles, tiles.size() * sizeof(BatchTile)) ||
      !dev_alloc((void**)&b->d_bpartials, 2 * (size_t)slots * sizeof(double)) ||
      !dev_alloc((void**)&b->d_bred, count * sizeof(BatchRed)) ||
      !dev_alloc((void**)&b->d_saved, (size_t)saved * sizeof(float)) ||
      !dev_alloc((void**)&b->d_bparams, 2 * (size_t)count * sizeof(TileParams)) ||
      !dev_alloc((void**)&b->d_bls_partials, 2 * (size_t)kBlsPartials * sizeof(double)))
    return fail(BF_ENOMEM, "hipMalloc batch adjoint buffers failed");
  if (bls_bytes > 0 && !dev_alloc(&b->d_bls, (size_t)bls_bytes))
    return fail(BF_ENOMEM, "hipMalloc batch streamed adjoint state failed");
  if (!tiles.empty() && hipMemcpy(b->d_btiles, tiles.data(), tiles.size() * sizeof(BatchTile),
                                  hipMemcpyHostToDevice) != hipSuccess)
    return fail(BF_EHIP, "hipMemcpy batch adjoint tiles failed");
  if (hipMemcpy(b->d_bred, red.data(), count * sizeof(BatchRed), hipMemcpyHostToDevice) != hipSuccess)
    return fail(BF_EHIP, "hipMemcpy batch reduction table failed");
  if (hipHostMalloc((void**)&b->h_bstage, 2 * (size_t)count * sizeof(TileParams), hipHostMallocDefault) !=
      hipSuccess)
    return fail(BF_ENOMEM, "hipHostMalloc batch adjoint staging failed");
  if (hipEventCreateWithFlags(&b->bev, hipEventDisableTiming) != hipSuccess)
    return fail(BF_EHIP, "hipEventCreate failed");
  return BF_OK;
}

static int grid_of(const bf_batch* b) {
  const BatchShape& sh = b->cands[b->chosen];
  int g = b->num_cu * sh.wg_per_cu;
  return std::max(1, std::min(g, std::max(1, b->nftiles)));
}

// The whole plain forward on `s`: the copy of this call's parameters from
// staging slot k, the fork of the side streams, the persistent launch, each
// routed image's streamed plan on its side stream (reading its image
// pointers from the copied parameters), and the join.  Recorded once into
// the slot's graph, so that one hipGraphLaunch replays all of it.
static int record_forward(bf_batch* b, int k, hipStream_t s) {
  const bool side = b->fork_ev != nullptr;
  if (side) {
    // the copy comes first, so the side streams fork after it
    if (hipMemcpyAsync(b->d_params, b->h_stage[k], b->count * sizeof(TileParams), hipMemcpyHostToDevice, s) !=
        hipSuccess)
      return fail(BF_EHIP, "hipMemcpyAsync batch params");
    fork_side(b, s);
    int st = BF_OK;
    for (int j = 0; j < bf_batch::kAux; ++j)
      for (int i : b->aux_imgs[j]) {
        if (st < 0) break;
        const hipError_t e = plan_forward_streamed_dyn(b->fplans[i], b->d_params + i, false, b->aux[j]);
        if (e != hipSuccess) st = fail(BF_EHIP, std::string("batch streamed image: ") + hipGetErrorString(e));
      }
    if (st >= 0 && b->nftiles > 0) {
      hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, b->d_counter);
      const BatchShape& sh = b->cands[b->chosen];
      const hipError_t e = launch_batch_v(sh.variant, b->d_params, b->d_ftiles, b->nftiles, b->d_counter,
                                          grid_of(b), sh.lds, b->acc64, false, s);
      if (e != hipSuccess) st = fail(BF_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
    }
    join_side(b, s);  // joined even after an error, so the capture ends with every stream rejoined
    return st;
  }
  return run_direct(b, k, s, grid_of(b));
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
  std::vector<int64_t> strides(count, 0), ntaps(count, 0);
  for (int i = 0; i < count; ++i) {
    bf_params pi = per_image[i];
    if (pi.flags & BF_FLAG_GRAD) b->grad = true;
    pi.flags &= ~(BF_FLAG_GRAD | BF_FLAG_STREAMED);
    int st = (pi.flags & BF_FLAG_JOINT)  ? fail(BF_EUNSUPPORTED, "the batch runs the plain filter only")
             : pi.kernel == BF_GAUSS_REC ? fail(BF_EUNSUPPORTED, "the batch has no recursive Gaussian")
                                         : bf_order(&pi, &b->info[i]);
    if (st >= 0 && b->info[i].lambda > kLambdaF32)
      st = fail(BF_EUNSUPPORTED, "the batch runs float32 ranges only: need T/sigma_r <= 13");
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
    tabs[i] = const_tables(pi, b->info[i], &strides[i], &ntaps[i]);
    offs[i] = total;
    total += (int64_t)tabs[i].size();
    TileParams& t = b->hp[i];
    std::memset(&t, 0, sizeof(t));
    t.H = pi.height;
    t.Wd = pi.width;
    t.W = pi.W;
    t.N = b->info[i].N;
    t.kt = pi.kernel;
    t.sigma_r = (float)pi.sigma_r;
    t.inv_sigma_r = (float)(1.0 / pi.sigma_r);
    t.center = (float)pi.center;
    t.inv_T = (float)(1.0 / pi.T);
    t.X = (float)(pi.T / pi.sigma_r);
    t.inv_sigma_s3 = pi.kernel == BF_GAUSS ? (float)(1.0 / (pi.sigma_s * pi.sigma_s * pi.sigma_s)) : 0.0f;
    t.saved_plane = (int64_t)pi.height * pi.width;
    t.mirror = (pi.flags & BF_FLAG_MIRROR) ? 1 : 0;
  }
  b->own_bytes += std::max<int64_t>(total, 1) * (int64_t)sizeof(float) + count * (int64_t)sizeof(TileParams) + 8;
  if (hipMalloc(&b->d_const, std::max<int64_t>(total, 1) * sizeof(float)) != hipSuccess) {
    delete b;
    return fail(BF_ENOMEM, "hipMalloc batch tables failed");
  }
  for (int i = 0; i < count; ++i) {
    if (b->status[i] < 0) continue;
    hipMemcpy(b->d_const + offs[i], tabs[i].data(), tabs[i].size() * sizeof(float), hipMemcpyHostToDevice);
    bind_tables(b->hp[i], b->d_const + offs[i], strides[i], ntaps[i]);
  }
  // images whose own plan takes the streamed passes (the per-image engine rule) run them
  b->fplans.assign(count, nullptr);
  for (int i = 0; i < count; ++i) {
    if (b->status[i] < 0 || b->info[i].path != BF_PATH_STREAMED) continue;
    bf_params q = b->prm[i];
    if (b->grad && !(q.flags & BF_FLAG_MIRROR)) q.flags |= BF_FLAG_GRAD;  // its adjoint runs on it too
    const int st = bf_plan(&q, &b->fplans[i]);
    if (st < 0) {
      bf_batch_destroy(b);
      return st;
    }
  }
  {
    // spread them over the side streams, largest cost first, each to the least-loaded stream
    std::vector<std::pair<double, int>> cost;
    for (int i = 0; i < count; ++i)
      if (b->fplans[i]) cost.push_back({(double)b->prm[i].height * b->prm[i].width * (b->info[i].N + 1), i});
    std::stable_sort(cost.begin(), cost.end(),
                     [](const std::pair<double, int>& x, const std::pair<double, int>& y) { return x.first > y.first; });
    double load[bf_batch::kAux] = {};
    for (const auto& c : cost) {
      const int j = (int)(std::min_element(load, load + bf_batch::kAux) - load);
      load[j] += c.first;
      b->aux_imgs[j].push_back(c.second);
    }
    if (!cost.empty()) {
      bool ok = hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) == hipSuccess;
      for (int j = 0; ok && j < bf_batch::kAux; ++j)
        ok = hipStreamCreateWithFlags(&b->aux[j], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&b->join_ev[j], hipEventDisableTiming) == hipSuccess;
      if (!ok) {
        bf_batch_destroy(b);
        return fail(BF_EHIP, "batch side streams");
      }
    }
  }
  // candidate launch shapes
  for (int v = 0; v < kNumBatchVariants; ++v)
    for (int wg : {1, 2, 4}) {
      BatchShape sh;
      if (build_shape(b, v, wg, &sh)) b->cands.push_back(std::move(sh));
    }
  if (b->cands.empty()) {
    bf_batch_destroy(b);
    return fail(BF_EUNSUPPORTED, "a batch image's support W is too large for the batch kernel");
  }
  if (hipMalloc(&b->d_params, count * sizeof(TileParams)) != hipSuccess ||
      hipMalloc(&b->d_counter, 2 * sizeof(int)) != hipSuccess) {
    bf_batch_destroy(b);
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
  if (b->grad) {
    st = plan_batch_adjoint(b);
    if (st < 0) {
      bf_batch_destroy(b);
      return st;
    }
  }
  *out = b;
  return warn;
}

int bf_batch_get_info(const bf_batch_t* b, bf_batch_info* out) {
  if (!b || !out) return fail(BF_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  for (int i = 0; i < b->count; ++i) {
    if (b->status[i] < 0) continue;
    if (b->fplans[i])
      out->images_streamed++;
    else
      out->images_persistent++;
  }
  out->persistent_lds_bytes = (int64_t)b->cands[b->chosen].lds;
  out->workspace_bytes = b->own_bytes + (int64_t)b->nftiles * (int64_t)sizeof(BatchTile);
  for (const bf_plan_t* pl : b->fplans)
    if (pl) out->workspace_bytes += pl->info.workspace_bytes;
  for (const bf_plan_t* pl : b->mplans)
    if (pl) out->workspace_bytes += pl->info.workspace_bytes;
  out->forward_graph_launches = b->graph_launches;
  out->forward_direct_launches = b->direct_launches;
  out->backward_graph_launches = b->bgraph_launches;
  out->backward_direct_launches = b->bdirect_launches;
  return BF_OK;
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
    // capture the whole forward (parameter copy, side-stream fork, persistent
    // launch, the routed images' streamed plans, join) from this slot
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
      return fail(BF_EHIP, "hipStreamCreate");
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
    int rs = BF_OK;
    if (e == hipSuccess) {
      rs = record_forward(b, k, cap);
      const hipError_t e2 = hipStreamEndCapture(cap, &graph);
      if (e == hipSuccess) e = e2;
    }
    if (rs >= 0 && e == hipSuccess) e = hipGraphInstantiate(&b->gexec[k], graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    hipStreamDestroy(cap);
    if (rs < 0) return rs;
    if (e != hipSuccess) {
      b->gexec[k] = nullptr;
      return fail(BF_EHIP, std::string("batch graph capture: ") + hipGetErrorString(e));
    }
  }
  hipError_t e = hipGraphLaunch(b->gexec[k], s);
  if (e != hipSuccess) return fail(BF_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  b->graph_launches++;
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

int bf_batch_forward_saved(bf_batch_t* b, const float* const* in, const int64_t* in_pitch,
                           float* const* out, const int64_t* out_pitch, float* const* saved, void* stream) {
  if (!b || !in || !out || !in_pitch || !out_pitch || !saved) return fail(BF_EINVAL, "NULL argument");
  if (!b->grad) return fail(BF_EINVAL, "saved state needs a batch planned with BF_FLAG_GRAD");
  hipStream_t s = (hipStream_t)stream;
  const int k = b->slot;
  b->slot ^= 1;
  int st = stage(b, k, in, in_pitch, out, out_pitch);
  if (st < 0) return st;
  for (int i = 0; i < b->count; ++i) {
    if (b->status[i] < 0) continue;
    if (!saved[i]) return fail(BF_EINVAL, "NULL saved pointer in batch");
    b->h_stage[k][i].saved = saved[i];
  }
  // images on their own streamed plans run it on the side streams (keeping their state there
  // unless their adjoint is the mirror plan's, which recomputes)
  const bool side = b->fork_ev != nullptr;
  if (side) fork_side(b, s);
  st = run_direct(b, k, s, grid_of(b), true);
  if (st < 0) return st;
  int fst = BF_OK;
  if (side) {
    for (int j = 0; j < bf_batch::kAux; ++j)
      for (int i : b->aux_imgs[j])
        if (fst >= 0)
          fst = bf_forward(b->fplans[i], in[i], in_pitch[i], out[i], out_pitch[i], b->own_adj[i] ? saved[i] : nullptr,
                           b->aux[j]);
    join_side(b, s);
  }
  hipEventRecord(b->ev[k], s);
  b->ev_used[k] = true;
  return fst < 0 ? fst : BF_OK;
}

}  // extern "C"

// The adjoint's launches from the staged parameters (h_bstage, copied to
// the device here): the forward state of the persistent images (unless
// saved), their adjoint tiles as one persistent launch and the sigma
// reductions on `s`, and the images on streamed plans of their own on the
// side streams, forked after the copy and joined back into `s`.  Every
// launch reads its image pointers from the device copy, so the batch records
// this once per (saved, sigma) combination into a graph.
static int record_backward(bf_batch* b, bool have_saved, bool sig, hipStream_t s) {
  const int n = b->count;
  const BatchShape& sh = b->cands[b->chosen];
  if (hipMemcpyAsync(b->d_bparams, b->h_bstage, 2 * (size_t)n * sizeof(TileParams), hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return fail(BF_EHIP, "hipMemcpyAsync batch adjoint params");
  const bool side = b->fork_ev != nullptr;
  if (side) fork_side(b, s);
  int st = BF_OK;
  // images on their own streamed plans: their whole adjoint on the side streams, the state
  // recomputed into the batch's planes of that image unless saved
  if (side)
    for (int j = 0; j < bf_batch::kAux; ++j)
      for (int i : b->aux_imgs[j]) {
        if (!b->own_adj[i] || st < 0) continue;
        const hipError_t e = plan_backward_streamed_dyn(b->fplans[i], b->d_bparams + i, b->d_bparams + n + i,
                                                        !have_saved, sig, b->aux[j]);
        if (e != hipSuccess) st = fail(BF_EHIP, std::string("batch streamed-plan adjoint: ") + hipGetErrorString(e));
      }
  if (st >= 0) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, b->d_counter);
    hipError_t e = hipSuccess;
    if (!have_saved && b->nftiles > 0) {
      e = launch_batch_v(sh.variant, b->d_bparams, b->d_ftiles, b->nftiles, b->d_counter, grid_of(b), sh.lds,
                         b->acc64, true, s);
      if (e != hipSuccess) st = fail(BF_EHIP, std::string("batch forward-state launch: ") + hipGetErrorString(e));
    }
    if (st >= 0 && b->nbtiles > 0) {
      const int grid = std::max(1, std::min(2 * b->num_cu, b->nbtiles));
      e = launch_batch_bwd(b->bvariant, b->d_bparams + n, b->d_btiles, b->nbtiles, b->d_counter + 1,
                           b->d_bpartials, grid, b->blds, s);
      if (e != hipSuccess) st = fail(BF_EHIP, std::string("batch adjoint launch: ") + hipGetErrorString(e));
    }
    if (st >= 0 && sig) {
      hipLaunchKernelGGL(batch_sigma_reduce_kernel, dim3(n), dim3(kThreads), 0, s, (const double*)b->d_bpartials,
                         (const BatchRed*)b->d_bred, (const TileParams*)(b->d_bparams + n));
      e = hipGetLastError();
      if (e != hipSuccess) st = fail(BF_EHIP, std::string("batch sigma reduction: ") + hipGetErrorString(e));
    }
  }
  if (side) join_side(b, s);  // joined even after an error, so a capture ends with every stream rejoined
  return st;
}

// saved: NULL (recompute the forward state into the batch workspace) or the
// per-image planes bf_batch_forward_saved wrote
static int batch_backward(bf_batch_t* b, const float* const* in, const int64_t* in_pitch,
                          const float* const* grad_out, const int64_t* gout_pitch, const float* const* saved,
                          float* const* grad_in, const int64_t* gin_pitch, double* grad_sigma, void* stream) {
  if (!b || !in || !in_pitch || !grad_out || !gout_pitch) return fail(BF_EINVAL, "NULL argument");
  if (!b->grad) return fail(BF_EINVAL, "batch was planned without BF_FLAG_GRAD");
  if (grad_in && !gin_pitch) return fail(BF_EINVAL, "grad_in without gin_pitch");
  hipStream_t s = (hipStream_t)stream;
  if (b->bev_used && hipEventSynchronize(b->bev) != hipSuccess) return fail(BF_EHIP, "hipEventSynchronize");
  const int n = b->count;
  for (int i = 0; i < n; ++i) {
    TileParams f = b->hp[i];  // forward with state
    TileParams g = b->hp[i];  // adjoint
    f.dyn = g.dyn = nullptr;
    f.gsig = g.gsig = nullptr;
    if (b->status[i] >= 0) {
      const int Wd = b->prm[i].width;
      if (!in[i] || !grad_out[i]) return fail(BF_EINVAL, "NULL image pointer in batch");
      if (in_pitch[i] < Wd || gout_pitch[i] < Wd || (grad_in && grad_in[i] && gin_pitch[i] < Wd))
        return fail(BF_EINVAL, "pitch smaller than width in batch");
      f.in = g.in = in[i];
      f.in_pitch = g.in_pitch = in_pitch[i];
      f.out = nullptr;
      f.out_pitch = 0;
      if (saved && !saved[i]) return fail(BF_EINVAL, "NULL saved pointer in batch");
      f.saved = g.saved = saved ? const_cast<float*>(saved[i]) : b->d_saved + b->saved_off[i];
      g.gout = grad_out[i];
      g.gout_pitch = gout_pitch[i];
      g.out = grad_in ? grad_in[i] : nullptr;
      g.out_pitch = (grad_in && grad_in[i]) ? gin_pitch[i] : 0;
      g.TY = b->bTY[i];
      g.gsig = grad_sigma ? grad_sigma + 2 * i : nullptr;
    }
    b->h_bstage[i] = f;
    b->h_bstage[n + i] = g;
  }
  const bool have_saved = saved != nullptr, sig = grad_sigma != nullptr;
  // images on the shared streamed-adjoint state (its clear is a memset) and
  // images with the reflecting border (their own plan's padding launches
  // take host pointers) keep the call issued launch by launch
  if (b->streamed.empty() && b->mirrored.empty()) {
    const int key = (have_saved ? 1 : 0) | (sig ? 2 : 0);
    if (!b->bgexec[key]) {
      hipStream_t cap;
      if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
        return fail(BF_EHIP, "hipStreamCreate");
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
      int rs = BF_OK;
      if (e == hipSuccess) {
        rs = record_backward(b, have_saved, sig, cap);
        const hipError_t e2 = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = e2;
      }
      if (rs >= 0 && e == hipSuccess) e = hipGraphInstantiate(&b->bgexec[key], graph, nullptr, nullptr, 0);
      if (graph) hipGraphDestroy(graph);
      hipStreamDestroy(cap);
      if (rs < 0) return rs;
      if (e != hipSuccess) {
        b->bgexec[key] = nullptr;
        return fail(BF_EHIP, std::string("batch adjoint graph capture: ") + hipGetErrorString(e));
      }
    }
    const hipError_t e = hipGraphLaunch(b->bgexec[key], s);
    if (e != hipSuccess) return fail(BF_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    b->bgraph_launches++;
    hipEventRecord(b->bev, s);
    b->bev_used = true;
    return BF_OK;
  }
  int st = record_backward(b, have_saved, sig, s);
  b->bdirect_launches++;
  hipError_t e = hipSuccess;
  for (int i : b->streamed) {
    if (st < 0) break;
    const bf_params& p = b->prm[i];
    const bool sigs = p.kernel == BF_GAUSS && sig;
    const bool gauss = p.kernel == BF_GAUSS;
    // the zero rows of this image's layout must be zero: clear the shared state
    e = hipMemsetAsync(b->d_bls, 0, (size_t)bls_state_bytes(p.height, p.width, p.W, gauss), s);
    if (e != hipSuccess) {
      st = fail(BF_EHIP, "hipMemsetAsync streamed adjoint state");
      break;
    }
    const BlsState bst = bls_layout(b->d_bls, p.height, p.width, p.W, gauss);
    e = launch_backward_ls(b->h_bstage[n + i], bst, sigs, b->d_bls_partials, b->h_bstage[n + i].gsig, s);
    if (e != hipSuccess) st = fail(BF_EHIP, std::string("batch streamed adjoint: ") + hipGetErrorString(e));
  }
  for (int i : b->mirrored) {
    if (st < 0) break;
    // recomputes its own state (the batch's saved planes of this image go unread)
    st = bf_backward(b->mplans[i], in[i], in_pitch[i], grad_out[i], gout_pitch[i], nullptr,
                     grad_in ? grad_in[i] : nullptr, grad_in ? gin_pitch[i] : 0,
                     grad_sigma ? grad_sigma + 2 * i : nullptr, stream);
  }
  hipEventRecord(b->bev, s);
  b->bev_used = true;
  return st < 0 ? st : BF_OK;
}

extern "C" {

int bf_batch_backward(bf_batch_t* b, const float* const* in, const int64_t* in_pitch,
                      const float* const* grad_out, const int64_t* gout_pitch, float* const* grad_in,
                      const int64_t* gin_pitch, double* grad_sigma, void* stream) {
  return batch_backward(b, in, in_pitch, grad_out, gout_pitch, nullptr, grad_in, gin_pitch, grad_sigma, stream);
}

int bf_batch_backward_saved(bf_batch_t* b, const float* const* in, const int64_t* in_pitch,
                            const float* const* grad_out, const int64_t* gout_pitch, const float* const* saved,
                            float* const* grad_in, const int64_t* gin_pitch, double* grad_sigma, void* stream) {
  if (!saved) return fail(BF_EINVAL, "NULL saved array");
  return batch_backward(b, in, in_pitch, grad_out, gout_pitch, saved, grad_in, gin_pitch, grad_sigma, stream);
}

int bf_batch_destroy(bf_batch_t* b) {
  if (!b) return BF_OK;
  for (int k = 0; k < 2; ++k)
    if (b->ev_used[k]) hipEventSynchronize(b->ev[k]);
  if (b->bev_used) hipEventSynchronize(b->bev);
  if (b->bev) hipEventDestroy(b->bev);
  if (b->h_bstage) hipHostFree(b->h_bstage);
  for (void* ptr : {(void*)b->d_btiles, (void*)b->d_bpartials, (void*)b->d_bred, (void*)b->d_saved,
                    (void*)b->d_bparams, b->d_bls, (void*)b->d_bls_partials})
    if (ptr) hipFree(ptr);
  destroy_graphs(b);
  for (int k = 0; k < 2; ++k) {
    if (b->ev[k]) hipEventDestroy(b->ev[k]);
    if (b->h_stage[k]) hipHostFree(b->h_stage[k]);
  }
  if (b->d_const) hipFree(b->d_const);
  if (b->d_params) hipFree(b->d_params);
  if (b->d_counter) hipFree(b->d_counter);
  if (b->d_ftiles) hipFree(b->d_ftiles);
  for (int j = 0; j < bf_batch::kAux; ++j) {
    if (b->aux[j]) {
      hipStreamSynchronize(b->aux[j]);
      hipStreamDestroy(b->aux[j]);
    }
    if (b->join_ev[j]) hipEventDestroy(b->join_ev[j]);
  }
  if (b->fork_ev) hipEventDestroy(b->fork_ev);
  for (bf_plan_t* pl : b->mplans)
    if (pl) bf_destroy(pl);
  for (bf_plan_t* pl : b->fplans)
    if (pl) bf_destroy(pl);
  delete b;
  return BF_OK;
}

}  // extern "C"
