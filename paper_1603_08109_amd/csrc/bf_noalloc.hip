// Static device memory for the allocation-free forward (bf_forward_noalloc).
//
// bf_plan keeps the constant tables of a filter (the range-safe scale factors
// s_n, r_n, the reciprocals 1/n and the padded spatial taps) in device memory
// it allocates.  The allocation-free forward keeps them in one file-scope
// array instead, `scratch`, of kNoAllocFloats floats (64 KiB).  Each device
// the library runs on holds its own copy until the process ends.  In host code
// the array's name is only a host-side stand-in, so its device address is
// taken once per device with hipGetSymbolAddress and only that address is
// ever handed to kernels.
//
// The tables reach the array through small fill kernels whose arguments carry
// the values by value: no host staging buffer has to outlive the call, and no
// copy or set routine of the runtime is involved.  Every call on one device
// shares the array and leaves the last call's tables in it, so calls that
// overlap on one device (different streams, or threads) race; calls in order
// on one stream do not.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "bf_internal.h"

namespace bfgpa {

constexpr int kNoAllocFloats = 16384;
static __device__ __align__(256) float scratch[kNoAllocFloats];

// floats carried by one fill launch (3.5 KiB of kernel arguments)
constexpr int kFillChunk = 896;
struct FillChunk {
  int32_t offset;
  int32_t count;
  float v[kFillChunk];
};

__global__ __launch_bounds__(kThreads) void noalloc_fill_kernel(FillChunk c, float* dst) {
  for (int i = threadIdx.x; i < c.count; i += kThreads) dst[c.offset + i] = c.v[i];
}

int noalloc_capacity_floats() { return kNoAllocFloats; }

// Device address of `scratch` on the current device, looked up on the first
// call on that device and kept.
hipError_t noalloc_scratch(float** out) {
  static std::mutex mu;
  static float* addr[64] = {nullptr};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = static_cast<float*>(p);
  }
  *out = addr[dev];
  return hipSuccess;
}

// Write n floats of host memory h to dst (inside the scratch array) on stream s.
hipError_t noalloc_fill(float* dst, const float* h, int64_t n, hipStream_t s) {
  if (n < 0 || n > kNoAllocFloats) return hipErrorInvalidValue;
  for (int64_t o = 0; o < n; o += kFillChunk) {
    FillChunk c;
    c.offset = (int32_t)o;
    c.count = (int32_t)(n - o < kFillChunk ? n - o : kFillChunk);
    for (int i = 0; i < c.count; ++i) c.v[i] = h[o + i];
    for (int i = c.count; i < kFillChunk; ++i) c.v[i] = 0.0f;
    hipLaunchKernelGGL(noalloc_fill_kernel, dim3(1), dim3(kThreads), 0, s, c, dst);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace bfgpa
