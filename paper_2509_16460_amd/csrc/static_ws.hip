// Static device scratch of the allocation-free J build (pwdf_build_j_noalloc).
//
// The per-call workspaces of a J build (D(L) / J(L) blocks, transform
// coefficients, moment and partial-row arrays, rho, V, energy partials, folded
// J, the FP32-MFMA operands) normally live in the context's own allocations.
// For callers that cannot allocate at all, they can instead be carved out of
// this file-scope array, which every device the library is loaded on holds for
// the life of the process.  Its host-side name is only a stand-in: the device
// address is looked up once per device with hipGetSymbolAddress and that
// address is what the kernels receive.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "kernels.h"

namespace pwdf {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(int device, void **ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!addr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

// Zero fill of n floats (a kernel rather than a memset node, so that the call
// can be captured into a graph).
__global__ __launch_bounds__(256) void k_zero_f32(float *__restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace pwdf
