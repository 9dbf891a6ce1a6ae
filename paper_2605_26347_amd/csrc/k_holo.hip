// Holographic matrix H_p = G_p^dag G_p (Sect. 3.3) and its product X'_p = H_p X_p, the
// alternative to the fused G^dag G when many visibilities share each grid cell.
//
// Storage: for every active grid tile of a bin (32 x 32 output cells), a dense stencil
// of side D = 2 Tmax - 1 (Tmax = the largest patch side of the rows that reach the
// tile): value [d][c] multiplies X at cell c + d - (D - 1) / 2 (both axes) and adds into
// output cell c.  H_p[q, q'] is non-zero only when one row's patch holds both q and q',
// so |q' - q| < Tmax on both axes and the stencil holds every entry of the tile's rows of
// H_p (entries no patch connects stay zero).  Layout [tile][d][c]: a workgroup streams
// its tile's stencil with consecutive threads on consecutive cells.
//
// Build: rows of one bin, in their work items; rows with the same patch word (origin
// and side) form a run whose pair products are summed before they are added, with
// global atomics, into the stencil of each output cell.
#include <hip/hip_fp16.h>

#include <mutex>
#include <vector>

#include "wf_internal.h"

namespace wf {

namespace {

__global__ __launch_bounds__(256) void k_hbuild(const WorkItem* __restrict__ wi,
                                                const uint32_t* __restrict__ meta,
                                                const uint32_t* __restrict__ voff,
                                                const float2* __restrict__ g, int64_t vbase,
                                                const int32_t* __restrict__ slot_of_tile,
                                                const HTile* __restrict__ ht, int tiles_x,
                                                int tsh, int Kx, int Ky,
                                                float* __restrict__ h) {
  const WorkItem w = wi[blockIdx.x];
  const int tile = 1 << tsh;
  const int rend = w.row0 + w.nrows;
  int r = w.row0;
  while (r < rend) {
    const uint32_t m = meta[r];
    int r1 = r + 1;
    while (r1 < rend && meta[r1] == m) ++r1;
    const int lu0 = (int)(m & 0xff), lv0 = (int)((m >> 8) & 0xff), T = (int)((m >> 16) & 0xff);
    const int TT = T * T;
    const int64_t npair = (int64_t)TT * TT;
    for (int64_t i = threadIdx.x; i < npair; i += blockDim.x) {
      const int a = (int)(i / TT), b = (int)(i - (int64_t)a * TT);
      float re = 0.f, im = 0.f;
      for (int k = r; k < r1; ++k) {
        const int64_t base = w.voff + (int64_t)voff[k] - vbase;
        const float2 ga = g[base + a], gb = g[base + b];
        re += ga.x * gb.x + ga.y * gb.y;     // conj(g[a]) g[b]
        im += ga.x * gb.y - ga.y * gb.x;
      }
      const int av = a / T, au = a - av * T, bv = b / T, bu = b - bv * T;
      const int qu = (w.u0 + lu0 + au) & (Kx - 1);
      const int qv = (w.v0 + lv0 + av) & (Ky - 1);
      const int sl = slot_of_tile[(qv >> tsh) * tiles_x + (qu >> tsh)];
      if (sl < 0) continue;   // cannot happen: the tile set covers every patch
      const HTile t = ht[sl];
      const int R = (t.D - 1) / 2;
      const int64_t di = (int64_t)(bv - av + R) * t.D + (bu - au + R);
      const int cell = ((qv & (tile - 1)) << tsh) + (qu & (tile - 1));
      float* dst = h + 2 * (t.voff + di * tile * tile + cell);
      atomicAdd(dst, re);
      atomicAdd(dst + 1, im);
    }
    r = r1;
  }
}

// FP32 stencils -> packed FP16 / BF16 pairs (round to nearest even); *overflow counts
// values beyond the FP16 range.
__global__ __launch_bounds__(256) void k_hpack(const float2* __restrict__ src,
                                               uint32_t* __restrict__ dst, int64_t n,
                                               int store, int* __restrict__ overflow) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float2 v = src[i];
    uint32_t out;
    if (store == WF_STORE_F16) {
      if (fabsf(v.x) > 65504.f || fabsf(v.y) > 65504.f) atomicAdd(overflow, 1);
      const __half2 hv = __floats2half2_rn(v.x, v.y);
      __builtin_memcpy(&out, &hv, 4);
    } else {
      auto bf = [](float f) -> uint32_t {
        const uint32_t b = __float_as_uint(f);
        return (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
      };
      out = bf(v.x) | (bf(v.y) << 16);
    }
    dst[i] = out;
  }
}

// Four consecutive stencil values (cells c .. c + 3 of one offset) as FP32 pairs.
template <int STORE>
__device__ __forceinline__ void hval4(const void* __restrict__ v, int64_t i, float2 (&h)[4]) {
  if constexpr (STORE == WF_STORE_F32) {
    const float4* p = reinterpret_cast<const float4*>(reinterpret_cast<const float2*>(v) + i);
    const float4 a = p[0], b = p[1];
    h[0] = make_float2(a.x, a.y);
    h[1] = make_float2(a.z, a.w);
    h[2] = make_float2(b.x, b.y);
    h[3] = make_float2(b.z, b.w);
  } else {
    const uint4 r = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint32_t*>(v) + i);
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (STORE == WF_STORE_F16) {
        __half2 hv;
        __builtin_memcpy(&hv, &w[j], 4);
        h[j] = __half22float2(hv);
      } else {
        h[j] = make_float2(__uint_as_float(w[j] << 16), __uint_as_float(w[j] & 0xffff0000u));
      }
    }
  }
}

// Y += H X over the active tiles of one bin; one workgroup per tile, the X window
// (tile + 2R cells per side, wrapped on the periodic grid) staged in LDS as two planes.
// Thread t owns the four consecutive cells 4t .. 4t + 3 of the tile (one vector load of
// stencil values per offset).  tile * tile == 4 * 256.
template <int STORE>
__global__ __launch_bounds__(256) void k_happly(const HTile* __restrict__ ht,
                                                const void* __restrict__ hv,
                                                const float2* __restrict__ X,
                                                float2* __restrict__ Y, int tiles_x, int tsh,
                                                int Kx, int Ky) {
  extern __shared__ float xw[];
  const HTile t = ht[blockIdx.x];
  const int tile = 1 << tsh, ncell = tile * tile;
  const int tu = t.tile % tiles_x, tv = t.tile / tiles_x;
  const int R = (t.D - 1) / 2, W = tile + 2 * R;
  float* xr = xw;
  float* xi = xw + W * W;
  const int u0 = tu * tile - R, v0 = tv * tile - R;
  for (int i = threadIdx.x; i < W * W; i += blockDim.x) {
    const int wv = i / W, wu = i - wv * W;
    const float2 x = X[strip_index((v0 + wv) & (Ky - 1), (u0 + wu) & (Kx - 1), Ky)];
    xr[i] = x.x;
    xi[i] = x.y;
  }
  __syncthreads();
  const int c0 = 4 * threadIdx.x;
  const int cv = c0 >> tsh, cu = c0 & (tile - 1);
  float ar[4] = {0.f, 0.f, 0.f, 0.f}, ai[4] = {0.f, 0.f, 0.f, 0.f};
  for (int dv = 0; dv < t.D; ++dv) {
    const float* rr = xr + (cv + dv) * W + cu;
    const float* ri = xi + (cv + dv) * W + cu;
    const int64_t rowbase = t.voff + (int64_t)dv * t.D * ncell + c0;
    for (int du = 0; du < t.D; ++du) {
      float2 h[4];
      hval4<STORE>(hv, rowbase + (int64_t)du * ncell, h);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float x0 = rr[du + j], x1 = ri[du + j];
        ar[j] += h[j].x * x0 - h[j].y * x1;
        ai[j] += h[j].x * x1 + h[j].y * x0;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float2* p = Y + strip_index(tv * tile + cv, tu * tile + cu + j, Ky);
    const float2 y = *p;
    *p = make_float2(y.x + ar[j], y.y + ai[j]);
  }
}

template <typename K>
hipError_t lds_limit(K kern, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  static std::mutex mu;
  static std::vector<std::pair<const void*, size_t>> done;
  const void* k = reinterpret_cast<const void*>(kern);
  std::lock_guard<std::mutex> lock(mu);
  for (auto& d : done)
    if (d.first == k && d.second >= bytes) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) done.push_back({k, bytes});
  return e;
}

}  // namespace

hipError_t launch_hbuild(const WorkItem* wi, int nwi, const uint32_t* meta, const uint32_t* voff,
                         const float2* g, int64_t vbase, const int32_t* slot_of_tile,
                         const HTile* ht, int tiles_x, int tsh, int Kx, int Ky, float* h,
                         hipStream_t s) {
  if (nwi <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hbuild, dim3(nwi), dim3(256), 0, s, wi, meta, voff, g, vbase,
                     slot_of_tile, ht, tiles_x, tsh, Kx, Ky, h);
  return hipGetLastError();
}

hipError_t launch_hpack(const float2* src, uint32_t* dst, int64_t n, wf_store store,
                        int* overflow, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_hpack, dim3((unsigned)nb), dim3(256), 0, s, src, dst, n, (int)store,
                     overflow);
  return hipGetLastError();
}

hipError_t launch_happly(const HTile* ht, int ntiles, int Dmax, const void* hv, wf_store store,
                         const float2* X, float2* Y, int tiles_x, int tsh, int Kx, int Ky,
                         hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const int W = (1 << tsh) + (Dmax - 1);
  const size_t lds = 2 * sizeof(float) * (size_t)W * W;
  hipError_t e;
  switch (store) {
    case WF_STORE_F32:
      if ((e = lds_limit(k_happly<WF_STORE_F32>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_happly<WF_STORE_F32>, dim3(ntiles), dim3(256), lds, s, ht, hv, X, Y,
                         tiles_x, tsh, Kx, Ky);
      break;
    case WF_STORE_F16:
      if ((e = lds_limit(k_happly<WF_STORE_F16>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_happly<WF_STORE_F16>, dim3(ntiles), dim3(256), lds, s, ht, hv, X, Y,
                         tiles_x, tsh, Kx, Ky);
      break;
    default:
      if ((e = lds_limit(k_happly<WF_STORE_BF16>, lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_happly<WF_STORE_BF16>, dim3(ntiles), dim3(256), lds, s, ht, hv, X, Y,
                         tiles_x, tsh, Kx, Ky);
      break;
  }
  return hipGetLastError();
}

}  // namespace wf
