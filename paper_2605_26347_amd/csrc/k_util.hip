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

// out[idx[i]] = 0: the forward values of flagged (discarded) visibilities.
__global__ void __launch_bounds__(256) k_scatter_zero(float2* out, const int32_t* idx,
                                                      int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[idx[i]] = make_float2(0.f, 0.f);
}

}  // namespace

hipError_t launch_scatter_zero(float2* out, const int32_t* idx, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_scatter_zero, dim3((unsigned)nb), dim3(256), 0, s, out, idx, n);
  return hipGetLastError();
}

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

// ------------------------------------------------------------------ forward-backward
// (Sect. 2, eq. 4) elementwise steps and reductions of the FB driver.

namespace wf {

namespace {

// x <- max(x + gamma (dirty - hx) - t, 0): gradient step of 1/2 ||Phi x - y||^2 followed
// by the prox of t ||x||_1 under positivity.
__global__ __launch_bounds__(256) void k_fb_step(float* __restrict__ x,
                                                 const float* __restrict__ dirty,
                                                 const float* __restrict__ hx, float gamma,
                                                 float t, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = fmaxf(x[i] + gamma * (dirty[i] - hx[i]) - t, 0.f);
}

// *out += sum a[i] b[i] (out cleared by the caller); block sums in LDS, one atomic each.
__global__ __launch_bounds__(256) void k_dot(const float* __restrict__ a,
                                             const float* __restrict__ b, int64_t n,
                                             float* __restrict__ out) {
  __shared__ float part[256];
  float s = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s += a[i] * b[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, part[0]);
}

// dst = src / sqrt(*nrm2)
__global__ __launch_bounds__(256) void k_normalize(float* __restrict__ dst,
                                                   const float* __restrict__ src, int64_t n,
                                                   const float* __restrict__ nrm2) {
  const float s = rsqrtf(fmaxf(*nrm2, 1e-30f));
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i] * s;
}

__global__ __launch_bounds__(256) void k_fill_value(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(256) void k_real_part(const float2* __restrict__ src,
                                                   float* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i].x;
}

unsigned blocks_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}

}  // namespace

hipError_t launch_fb_step(float* x, const float* dirty, const float* hx, float gamma, float t,
                          int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fb_step, dim3(blocks_for(n)), dim3(256), 0, s, x, dirty, hx, gamma, t, n);
  return hipGetLastError();
}

hipError_t launch_dot(const float* a, const float* b, int64_t n, float* out, hipStream_t s) {
  hipError_t e = launch_fill_zero(out, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dot, dim3(blocks_for(n)), dim3(256), 0, s, a, b, n, out);
  return hipGetLastError();
}

hipError_t launch_normalize(float* dst, const float* src, int64_t n, const float* nrm2,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_normalize, dim3(blocks_for(n)), dim3(256), 0, s, dst, src, n, nrm2);
  return hipGetLastError();
}

hipError_t launch_fill_value(float* p, int64_t n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_value, dim3(blocks_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_real_part(const float2* src, float* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_real_part, dim3(blocks_for(n)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace wf
