// Small utility kernels of the apply sequences: zero fill (used instead of a runtime
// memset so that an apply can be captured into a HIP graph) and the per-channel
// completion stamps of the batched sweep.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "wf_internal.h"

namespace wf {

namespace {

__global__ void __launch_bounds__(256) k_fill_zero(float4* p, int64_t n4) {
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z;
}

__global__ void __launch_bounds__(256) k_fill_zero_tail(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// Device wall clock (constant rate, hipDeviceAttributeWallClockRate kHz) into *dst.  The
// stamp kernel is ordered after the previous work of its stream like any other kernel.
__global__ void __launch_bounds__(64) k_stamp(unsigned long long* dst) {
  if (threadIdx.x == 0) dst[0] = wall_clock64();
}

// out[i] += in_b[i] for the extra accumulators of a split channel (complex or real
// FP32 values, counted in floats).
__global__ void __launch_bounds__(256) k_add_into(float* out, const float* in, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] += in[i];
}

}  // namespace

hipError_t launch_fill_zero(void* p, int64_t nfloats, hipStream_t s) {
  if (nfloats <= 0) return hipSuccess;
  const int64_t n4 = ((uintptr_t)p % 16 == 0) ? nfloats / 4 : 0;
  if (n4 > 0) {
    const int64_t nb = std::min<int64_t>((n4 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)nb), dim3(256), 0, s, (float4*)p, n4);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t rest = nfloats - 4 * n4;
  if (rest > 0) {
    const int64_t nb = (rest + 255) / 256;
    hipLaunchKernelGGL(k_fill_zero_tail, dim3((unsigned)nb), dim3(256), 0, s,
                       (float*)p + 4 * n4, rest);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_stamp(unsigned long long* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, dst);
  return hipGetLastError();
}

hipError_t launch_add_into(float* out, const float* in, int64_t nfloats, hipStream_t s) {
  if (nfloats <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((nfloats + 255) / 256, 8192);
  hipLaunchKernelGGL(k_add_into, dim3((unsigned)nb), dim3(256), 0, s, out, in, nfloats);
  return hipGetLastError();
}

}  // namespace wf
