// Sparse products with the de-gridding matrix G_p (Sect. 3.2, eq. 6) and its adjoint
// (Sect. 3.3, eq. 8).
//
// Rows are sorted by (bin, grid tile, patch side) and cut into work items; a
// workgroup owns one work item and a wavefront processes one row at a time with its
// 64 lanes spread over the row's T x T patch (T <= 37 -> at most 22 taps per lane).
//   fused G^dag G : y_k = sum_q g_k[q] X[q] (gather from the grid, wave reduction),
//                   then conj(g_k) y_k is added into an LDS window of the tile plus
//                   its halo (LDS atomics); G is read from HBM once.  The window is
//                   flushed with global atomics into Y, skipping untouched cells.
//   de-gridding   : the gather half, y written to the caller's visibility order.
//   gridding      : the scatter half, y read from the caller's visibility order.
// Values are stored as complex FP32, FP16 or BF16; all arithmetic is FP32.
#include <hip/hip_fp16.h>

#include "fft_lds.h"
#include "wf_internal.h"

namespace wf {

constexpr int GWAVES = 8;          // wavefronts per workgroup
constexpr int GNT = GWAVES * 64;
constexpr int MAXK = 22;           // ceil(37*37 / 64)

template <int STORE>
__device__ __forceinline__ float2 load_val(const void* __restrict__ vals, int64_t i) {
  if constexpr (STORE == WF_STORE_F32) {
    return reinterpret_cast<const float2*>(vals)[i];
  } else if constexpr (STORE == WF_STORE_F16) {
    const __half2 h = reinterpret_cast<const __half2*>(vals)[i];
    return __half22float2(h);
  } else {
    const uint32_t b = reinterpret_cast<const uint32_t*>(vals)[i];
    return make_float2(__uint_as_float(b << 16), __uint_as_float(b & 0xffff0000u));
  }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Gather y = sum_t g[t] X[cell(t)] over one row; keeps the row's values and LDS
// window indices in registers for a following scatter.
template <int STORE>
__device__ __forceinline__ float2 row_gather(const void* __restrict__ vals, int64_t vb, int T,
                                             int lu0, int lv0, int u0, int v0, int Kx, int Ky,
                                             const float2* __restrict__ X, float2 (&g)[MAXK],
                                             int (&li)[MAXK], int W, int lane, bool need_x) {
  const int TT = T * T;
  const float invT = 1.0f / (float)T;
  float sx = 0.f, sy = 0.f;
#pragma unroll
  for (int k = 0; k < MAXK; ++k) li[k] = -1;
#pragma unroll
  for (int k = 0; k < MAXK; ++k) {
    if (64 * k >= TT) break;  // wave-uniform
    const int t = lane + 64 * k;
    if (t < TT) {
      const int a = (int)(((float)t + 0.5f) * invT);
      const int b = t - a * T;
      g[k] = load_val<STORE>(vals, vb + t);
      li[k] = (lv0 + a) * W + (lu0 + b);
      if (need_x) {
        const int gu = (u0 + lu0 + b) & (Kx - 1);
        const int gv = (v0 + lv0 + a) & (Ky - 1);
        const float2 x = X[strip_index(gv, gu, Ky)];
        sx += g[k].x * x.x - g[k].y * x.y;
        sy += g[k].x * x.y + g[k].y * x.x;
      }
    }
  }
  return make_float2(sx, sy);
}

__device__ __forceinline__ void window_flush(const float2* acc, int W, int u0, int v0, int Kx,
                                             int Ky, float2* __restrict__ Y) {
  for (int c = threadIdx.x; c < W * W; c += GNT) {
    const float2 v = acc[c];
    if (v.x != 0.f || v.y != 0.f) {
      const int a = c / W, b = c - a * W;
      const int gu = (u0 + b) & (Kx - 1);
      const int gv = (v0 + a) & (Ky - 1);
      float2* p = Y + strip_index(gv, gu, Ky);
      unsafeAtomicAdd(&p->x, v.x);
      unsafeAtomicAdd(&p->y, v.y);
    }
  }
}

template <int STORE>
__global__ __launch_bounds__(GNT) void k_gtg(const WorkItem* __restrict__ wis,
                                             const uint32_t* __restrict__ meta,
                                             const uint32_t* __restrict__ voff,
                                             const void* __restrict__ vals,
                                             const float2* __restrict__ X,
                                             float2* __restrict__ Y, int Kx, int Ky, int W) {
  extern __shared__ float2 acc[];
  const WorkItem wi = wis[xcd_remap(blockIdx.x, gridDim.x)];
  for (int c = threadIdx.x; c < W * W; c += GNT) acc[c] = make_float2(0.f, 0.f);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* accf = reinterpret_cast<float*>(acc);
  for (int r = wave; r < wi.nrows; r += GWAVES) {
    const int row = wi.row0 + r;
    const uint32_t m = meta[row];
    const int lu0 = m & 0xff, lv0 = (m >> 8) & 0xff, T = (m >> 16) & 0xff;
    const int64_t vb = wi.voff + voff[row];
    float2 g[MAXK];
    int li[MAXK];
    float2 s = row_gather<STORE>(vals, vb, T, lu0, lv0, wi.u0, wi.v0, Kx, Ky, X, g, li, W,
                                 lane, true);
    s.x = wave_sum(s.x);
    s.y = wave_sum(s.y);
#pragma unroll
    for (int k = 0; k < MAXK; ++k) {
      if (64 * k >= T * T) break;  // wave-uniform
      if (li[k] >= 0) {
        // conj(g) * y
        const float rx = g[k].x * s.x + g[k].y * s.y;
        const float ry = g[k].x * s.y - g[k].y * s.x;
        atomicAdd(accf + 2 * li[k], rx);
        atomicAdd(accf + 2 * li[k] + 1, ry);
      }
    }
  }
  __syncthreads();
  window_flush(acc, W, wi.u0, wi.v0, Kx, Ky, Y);
}

template <int STORE>
__global__ __launch_bounds__(GNT) void k_degrid(const WorkItem* __restrict__ wis,
                                                const uint32_t* __restrict__ meta,
                                                const uint32_t* __restrict__ voff,
                                                const int32_t* __restrict__ perm,
                                                const void* __restrict__ vals,
                                                const float2* __restrict__ X,
                                                float2* __restrict__ vis, int Kx, int Ky) {
  const WorkItem wi = wis[xcd_remap(blockIdx.x, gridDim.x)];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = wave; r < wi.nrows; r += GWAVES) {
    const int row = wi.row0 + r;
    const uint32_t m = meta[row];
    const int lu0 = m & 0xff, lv0 = (m >> 8) & 0xff, T = (m >> 16) & 0xff;
    const int64_t vb = wi.voff + voff[row];
    float2 g[MAXK];
    int li[MAXK];
    float2 s = row_gather<STORE>(vals, vb, T, lu0, lv0, wi.u0, wi.v0, Kx, Ky, X, g, li, 256,
                                 lane, true);
    s.x = wave_sum(s.x);
    s.y = wave_sum(s.y);
    if (lane == 0) vis[perm[row]] = s;
  }
}

template <int STORE>
__global__ __launch_bounds__(GNT) void k_grid(const WorkItem* __restrict__ wis,
                                              const uint32_t* __restrict__ meta,
                                              const uint32_t* __restrict__ voff,
                                              const int32_t* __restrict__ perm,
                                              const void* __restrict__ vals,
                                              const float2* __restrict__ vis,
                                              float2* __restrict__ Y, int Kx, int Ky, int W) {
  extern __shared__ float2 acc[];
  const WorkItem wi = wis[xcd_remap(blockIdx.x, gridDim.x)];
  for (int c = threadIdx.x; c < W * W; c += GNT) acc[c] = make_float2(0.f, 0.f);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* accf = reinterpret_cast<float*>(acc);
  for (int r = wave; r < wi.nrows; r += GWAVES) {
    const int row = wi.row0 + r;
    const uint32_t m = meta[row];
    const int lu0 = m & 0xff, lv0 = (m >> 8) & 0xff, T = (m >> 16) & 0xff;
    const int64_t vb = wi.voff + voff[row];
    const float2 s = vis[perm[row]];
    float2 g[MAXK];
    int li[MAXK];
    row_gather<STORE>(vals, vb, T, lu0, lv0, wi.u0, wi.v0, Kx, Ky, nullptr, g, li, W, lane,
                      false);
#pragma unroll
    for (int k = 0; k < MAXK; ++k) {
      if (64 * k >= T * T) break;  // wave-uniform
      if (li[k] >= 0) {
        const float rx = g[k].x * s.x + g[k].y * s.y;
        const float ry = g[k].x * s.y - g[k].y * s.x;
        atomicAdd(accf + 2 * li[k], rx);
        atomicAdd(accf + 2 * li[k] + 1, ry);
      }
    }
  }
  __syncthreads();
  window_flush(acc, W, wi.u0, wi.v0, Kx, Ky, Y);
}

// ------------------------------------------------------------------ launchers

template <typename K>
static hipError_t set_lds(K kern, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_gtg(const WorkItem* wi, int nwi, const uint32_t* meta, const uint32_t* voff,
                      const void* vals, wf_store store, const float2* X, float2* Y, int Kx,
                      int Ky, int win, hipStream_t s) {
  if (nwi <= 0) return hipSuccess;
  const size_t lds = (size_t)win * win * sizeof(float2);
  hipError_t e;
  switch (store) {
    case WF_STORE_F32:
      if ((e = set_lds(k_gtg<WF_STORE_F32>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_gtg<WF_STORE_F32>, dim3(nwi), dim3(GNT), lds, s, wi, meta, voff,
                         vals, X, Y, Kx, Ky, win);
      break;
    case WF_STORE_F16:
      if ((e = set_lds(k_gtg<WF_STORE_F16>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_gtg<WF_STORE_F16>, dim3(nwi), dim3(GNT), lds, s, wi, meta, voff,
                         vals, X, Y, Kx, Ky, win);
      break;
    default:
      if ((e = set_lds(k_gtg<WF_STORE_BF16>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_gtg<WF_STORE_BF16>, dim3(nwi), dim3(GNT), lds, s, wi, meta, voff,
                         vals, X, Y, Kx, Ky, win);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_degrid(const WorkItem* wi, int nwi, const uint32_t* meta,
                         const uint32_t* voff, const int32_t* perm, const void* vals,
                         wf_store store, const float2* X, float2* vis, int Kx, int Ky,
                         hipStream_t s) {
  if (nwi <= 0) return hipSuccess;
  switch (store) {
    case WF_STORE_F32:
      hipLaunchKernelGGL(k_degrid<WF_STORE_F32>, dim3(nwi), dim3(GNT), 0, s, wi, meta, voff,
                         perm, vals, X, vis, Kx, Ky);
      break;
    case WF_STORE_F16:
      hipLaunchKernelGGL(k_degrid<WF_STORE_F16>, dim3(nwi), dim3(GNT), 0, s, wi, meta, voff,
                         perm, vals, X, vis, Kx, Ky);
      break;
    default:
      hipLaunchKernelGGL(k_degrid<WF_STORE_BF16>, dim3(nwi), dim3(GNT), 0, s, wi, meta, voff,
                         perm, vals, X, vis, Kx, Ky);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_grid(const WorkItem* wi, int nwi, const uint32_t* meta, const uint32_t* voff,
                       const int32_t* perm, const void* vals, wf_store store,
                       const float2* vis, float2* Y, int Kx, int Ky, int win, hipStream_t s) {
  if (nwi <= 0) return hipSuccess;
  const size_t lds = (size_t)win * win * sizeof(float2);
  hipError_t e;
  switch (store) {
    case WF_STORE_F32:
      if ((e = set_lds(k_grid<WF_STORE_F32>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_grid<WF_STORE_F32>, dim3(nwi), dim3(GNT), lds, s, wi, meta, voff,
                         perm, vals, vis, Y, Kx, Ky, win);
      break;
    case WF_STORE_F16:
      if ((e = set_lds(k_grid<WF_STORE_F16>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_grid<WF_STORE_F16>, dim3(nwi), dim3(GNT), lds, s, wi, meta, voff,
                         perm, vals, vis, Y, Kx, Ky, win);
      break;
    default:
      if ((e = set_lds(k_grid<WF_STORE_BF16>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_grid<WF_STORE_BF16>, dim3(nwi), dim3(GNT), lds, s, wi, meta, voff,
                         perm, vals, vis, Y, Kx, Ky, win);
      break;
  }
  return hipGetLastError();
}

}  // namespace wf
