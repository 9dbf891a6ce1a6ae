// Briggs robust data weighting (the density-aware weighting named in Sect. 2; formula
// from D. S. Briggs' 1995 thesis): gridded density of the natural weights over the
// image's Fourier cells, two global sums, then one weight per sample.  FP64 arithmetic;
// the density and the sums use FP64 atomics in global memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "wf_internal.h"

namespace wf {

namespace {

// Flat index iv * nx + iu of (u, v): floor(u / du + 1/2) modulo nx, likewise v.
__device__ __forceinline__ int64_t uv_cell(double u, double v, double du, double dv, int nx,
                                           int ny) {
  const int64_t iu = (int64_t)floor(u / du + 0.5);
  const int64_t iv = (int64_t)floor(v / dv + 0.5);
  const int64_t mu = ((iu % nx) + nx) % nx, mv = ((iv % ny) + ny) % ny;
  return mv * nx + mu;
}

__device__ __forceinline__ double nat_weight(const float* w, const uint8_t* flags, int64_t k) {
  if (flags && flags[k]) return 0.0;
  return w ? (double)w[k] : 1.0;
}

// W[cell(u, v)] += w and W[cell(-u, -v)] += w for every sample (the conjugate sample of a
// real image).
__global__ __launch_bounds__(256) void k_density(const double* __restrict__ uvw, int64_t n,
                                                 double scale, double du, double dv, int nx,
                                                 int ny, const float* __restrict__ w,
                                                 const uint8_t* __restrict__ flags,
                                                 double* __restrict__ W) {
#pragma clang fp contract(off)
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double wk = nat_weight(w, flags, k);
    if (wk == 0.0) continue;
    const double u = uvw[3 * k] * scale, v = uvw[3 * k + 1] * scale;
    atomicAdd(W + uv_cell(u, v, du, dv, nx, ny), wk);
    atomicAdd(W + uv_cell(-u, -v, du, dv, nx, ny), wk);
  }
}

// sums[0] += sum_k w_k W[cell(k)], sums[1] += sum_k w_k (one atomic pair per workgroup).
__global__ __launch_bounds__(256) void k_briggs_sums(const double* __restrict__ uvw, int64_t n,
                                                     double scale, double du, double dv, int nx,
                                                     int ny, const float* __restrict__ w,
                                                     const uint8_t* __restrict__ flags,
                                                     const double* __restrict__ W,
                                                     double* __restrict__ sums) {
#pragma clang fp contract(off)
  __shared__ double red[2][256];
  double a = 0.0, b = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double wk = nat_weight(w, flags, k);
    if (wk == 0.0) continue;
    const double u = uvw[3 * k] * scale, v = uvw[3 * k + 1] * scale;
    a += wk * W[uv_cell(u, v, du, dv, nx, ny)];
    b += wk;
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(sums, red[0][0]);
    atomicAdd(sums + 1, red[1][0]);
  }
}

// out_k = sqrt(w_k / (1 + W[cell(k)] f2)), zero for flagged or zero-weight samples.
__global__ __launch_bounds__(256) void k_briggs_out(const double* __restrict__ uvw, int64_t n,
                                                    double scale, double du, double dv, int nx,
                                                    int ny, const float* __restrict__ w,
                                                    const uint8_t* __restrict__ flags,
                                                    const double* __restrict__ W, double f2,
                                                    float* __restrict__ out) {
#pragma clang fp contract(off)
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double wk = nat_weight(w, flags, k);
    if (wk == 0.0) {
      out[k] = 0.f;
      continue;
    }
    const double u = uvw[3 * k] * scale, v = uvw[3 * k + 1] * scale;
    out[k] = (float)sqrt(wk / (1.0 + W[uv_cell(u, v, du, dv, nx, ny)] * f2));
  }
}

// As k_briggs_out with f^2 = a2 sums[1] / sums[0] formed on the device from the sums
// k_briggs_sums wrote (same operations, in the same order, as the host form), so that
// nothing waits on the host between the passes; all zero when either sum is not positive.
__global__ __launch_bounds__(256) void k_briggs_out_dev(const double* __restrict__ uvw,
                                                        int64_t n, double scale, double du,
                                                        double dv, int nx, int ny,
                                                        const float* __restrict__ w,
                                                        const uint8_t* __restrict__ flags,
                                                        const double* __restrict__ W,
                                                        const double* __restrict__ sums,
                                                        double a2, float* __restrict__ out) {
#pragma clang fp contract(off)
  const double s0 = sums[0], s1 = sums[1];
  const bool ok = s0 > 0 && s1 > 0;
  const double f2 = ok ? a2 * s1 / s0 : 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double wk = nat_weight(w, flags, k);
    if (!ok || wk == 0.0) {
      out[k] = 0.f;
      continue;
    }
    const double u = uvw[3 * k] * scale, v = uvw[3 * k + 1] * scale;
    out[k] = (float)sqrt(wk / (1.0 + W[uv_cell(u, v, du, dv, nx, ny)] * f2));
  }
}

unsigned blocks_for(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 8192); }

}  // namespace

// Device memory of the allocation-free entry point (wf_briggs_weights_noalloc): the
// density over at most WF_BRIGGS_NOALLOC_MAX_CELLS Fourier cells, then the two sums.
// Static device memory: every device the library runs on holds its own copy until the
// process ends.  Host code reaches it only through the address hipGetSymbolAddress
// returns for the current device (the symbol's name is a host-side stand-in).
static __device__ __align__(256) double scratch[WF_BRIGGS_NOALLOC_MAX_CELLS + 2];

hipError_t briggs_scratch(double** out) {
  constexpr int MAXDEV = 64;
  static std::mutex mu;
  static double* ptr[MAXDEV] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptr[dev] = static_cast<double*>(p);
  }
  *out = ptr[dev];
  return hipSuccess;
}

hipError_t launch_briggs_out_dev(const double* uvw, int64_t n, double scale, double du,
                                 double dv, int nx, int ny, const float* w,
                                 const uint8_t* flags, const double* W, const double* sums,
                                 double a2, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_briggs_out_dev, dim3(blocks_for(n)), dim3(256), 0, s, uvw, n, scale,
                     du, dv, nx, ny, w, flags, W, sums, a2, out);
  return hipGetLastError();
}

hipError_t launch_density(const double* uvw, int64_t n, double scale, double du, double dv,
                          int nx, int ny, const float* w, const uint8_t* flags, double* W,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_density, dim3(blocks_for(n)), dim3(256), 0, s, uvw, n, scale, du, dv,
                     nx, ny, w, flags, W);
  return hipGetLastError();
}

hipError_t launch_briggs_sums(const double* uvw, int64_t n, double scale, double du,
                              double dv, int nx, int ny, const float* w,
                              const uint8_t* flags, const double* W, double* sums,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_briggs_sums, dim3(std::min(blocks_for(n), 1024u)), dim3(256), 0, s, uvw,
                     n, scale, du, dv, nx, ny, w, flags, W, sums);
  return hipGetLastError();
}

hipError_t launch_briggs_out(const double* uvw, int64_t n, double scale, double du, double dv,
                             int nx, int ny, const float* w, const uint8_t* flags,
                             const double* W, double f2, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_briggs_out, dim3(blocks_for(n)), dim3(256), 0, s, uvw, n, scale, du, dv,
                     nx, ny, w, flags, W, f2, out);
  return hipGetLastError();
}

}  // namespace wf
