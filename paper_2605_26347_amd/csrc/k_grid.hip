// Sparse products with the de-gridding matrix G_p (Sect. 3.2, eq. 6) and its adjoint
// (Sect. 3.3, eq. 8).
//
// Rows are sorted by (bin, grid tile, patch side, patch origin) and cut into work
// items that hold one patch-size class; a workgroup owns one work item and each of its
// wavefronts walks a contiguous segment of the item's rows, its 64 lanes spread over a
// register patch (MK slots per lane).  Consecutive rows with the same patch origin and
// side form a "run" (visibilities falling in one grid cell); consecutive runs with the
// same side and patch row whose origins lie a few columns apart form a merge group that
// shares one register patch of T x (T + span) cells (the span fills the class's spare
// slots), each row's taps mapped in at its column offset.  Per group
//   * the grid values X of the group's patch are gathered once,
//   * conj(g_k) y_k is accumulated in registers over the group and added into the LDS
//     window of the tile (plus halo) once,
// and the stored values of G are streamed from HBM exactly once.  A row's sum
// y_k = sum_t g_k[t] X[t] is reduced across the wavefront with DPP within each
// 16-lane row and four readlanes, which leaves y_k wave-uniform.  At the end the
// window is added into Y with global atomics (untouched cells skipped).
//   fused G^dag G : gather + reduce + accumulate (Phi^dag Phi);
//   de-gridding   : gather + reduce, y written to the caller's visibility order (Phi);
//   gridding      : y read from the caller's order, accumulate (Phi^dag).
// Values are stored as complex FP32, FP16 or BF16; all arithmetic is FP32.
#include <hip/hip_fp16.h>

#include "fft_lds.h"
#include "wf_internal.h"

namespace wf {

constexpr int GWAVES = 8;          // wavefronts per workgroup
constexpr int GNT = GWAVES * 64;

// Stored values are loaded in their raw form (float2, or one 32-bit word holding two
// 16-bit halves) and widened to FP32 only where they are used, so that the loads of a
// row can all be in flight together.
template <int STORE>
struct RawT {
  using type = uint32_t;
};
template <>
struct RawT<WF_STORE_F32> {
  using type = float2;
};

template <int STORE>
__device__ __forceinline__ typename RawT<STORE>::type load_raw(const void* __restrict__ vals,
                                                               int64_t i) {
  if constexpr (STORE == WF_STORE_F32) {
    return reinterpret_cast<const float2*>(vals)[i];
  } else {
    return reinterpret_cast<const uint32_t*>(vals)[i];
  }
}

template <int STORE>
__device__ __forceinline__ float2 widen(typename RawT<STORE>::type r) {
  if constexpr (STORE == WF_STORE_F32) {
    return r;
  } else if constexpr (STORE == WF_STORE_F16) {
    __half2 h;
    __builtin_memcpy(&h, &r, 4);
    return __half22float2(h);
  } else {
    return make_float2(__uint_as_float(r << 16), __uint_as_float(r & 0xffff0000u));
  }
}

// Sum over the wavefront, returned wave-uniform: DPP butterflies inside each row of 16
// lanes (quad xor 1, quad xor 2, half-row mirror, row mirror), then the four row sums.
__device__ __forceinline__ float wave_sum_uniform(float v) {
  v += __builtin_amdgcn_update_dpp(0.f, v, 0xb1, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x4e, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x141, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x140, 0xf, 0xf, false);
  const int b = __float_as_int(v);
  return (__int_as_float(__builtin_amdgcn_readlane(b, 0)) +
          __int_as_float(__builtin_amdgcn_readlane(b, 16))) +
         (__int_as_float(__builtin_amdgcn_readlane(b, 32)) +
          __int_as_float(__builtin_amdgcn_readlane(b, 48)));
}

// A merge group: runs of patch side T in one patch row whose origins lie within `span`
// columns of the first run's origin lu0 share a register patch of T x Wx cells,
// Wx = T + span, slot t <-> (t / Wx, t % Wx).  A row's word carries lu0 | lv0 << 8 |
// T << 16 | du << 24, du being its column offset from the group's origin.
struct RunGeom {
  int T, Wx, TT, lu0, lv0;
};

// Group key of a row word: its origin moved back by du (no borrow: lu0 >= du).  Without
// merging (de-gridding, which has no scatter to save) every run is its own group.
template <bool MERGE>
__device__ __forceinline__ uint32_t group_key(uint32_t m) {
  return MERGE ? (m & 0x00ffffffu) - (m >> 24) : (m & 0x00ffffffu);
}

template <int MK, bool MERGE>
__device__ __forceinline__ RunGeom decode(uint32_t gkey) {
  RunGeom r;
  r.lu0 = gkey & 0xff;
  r.lv0 = (gkey >> 8) & 0xff;
  r.T = (gkey >> 16) & 0xff;
  r.Wx = r.T + (MERGE ? group_span(r.T, MK) : 0);
  r.TT = r.T * r.Wx;
  return r;
}


// Patch coordinates (a = row, b = column) of tap t; exact for t < 2^13, T <= 64.
__device__ __forceinline__ void tap_ab(int t, int T, float invT, int& a, int& b) {
  a = (int)(((float)t + 0.5f) * invT);
  b = t - a * T;
}

// Slots of a row with patch side T and column offset du in its group's register patch:
// bit k set when slot lane + 64 k holds one of the row's taps; tap[k] its index in the
// row's stored values (0 for the other slots, an in-bounds dummy).
template <int MK, bool MERGE>
__device__ __forceinline__ uint32_t row_slots(uint32_t m, int lane, int (&tap)[MK]) {
  const int T = (int)((m >> 16) & 0xff), du = MERGE ? (int)(m >> 24) : 0;
  const int Wx = T + (MERGE ? group_span(T, MK) : 0);
  const float invW = 1.0f / (float)Wx;
  uint32_t valid = 0;
#pragma unroll
  for (int k = 0; k < MK; ++k) {
    const int t = lane + 64 * k;
    int a, b;
    tap_ab(t, Wx, invW, a, b);
    const int bb = b - du;
    const bool ok = t < T * Wx && bb >= 0 && bb < T;
    tap[k] = ok ? a * T + bb : 0;
    valid |= ok ? (1u << k) : 0u;
  }
  return valid;
}

// Load the grid values of a group's register patch (one per lane and slot).
template <int MK>
__device__ __forceinline__ void load_patch_x(const RunGeom& r, int u0, int v0, int Kx, int Ky,
                                             const float2* __restrict__ X, int lane,
                                             float2 (&xr)[MK]) {
  const float invW = 1.0f / (float)r.Wx;
  // branch-free: lanes past the patch read its last cell and zero the value
#pragma unroll
  for (int k = 0; k < MK; ++k) {
    const int t = lane + 64 * k;
    const int tc = t < r.TT ? t : r.TT - 1;
    int a, b;
    tap_ab(tc, r.Wx, invW, a, b);
    const int gu = (u0 + r.lu0 + b) & (Kx - 1);
    const int gv = (v0 + r.lv0 + a) & (Ky - 1);
    xr[k] = X[strip_index(gv, gu, Ky)];
  }
#pragma unroll
  for (int k = 0; k < MK; ++k)
    if (lane + 64 * k >= r.TT) xr[k] = make_float2(0.f, 0.f);
}

// Add a group's register accumulator into the LDS window: the columns its runs covered,
// b < bend = T + largest offset (inside the window: that run's patch is).  The window is
// stored as two planes (real parts, then imaginary parts) so that the consecutive cells
// of a patch row fall in consecutive banks.
template <int MK>
__device__ __forceinline__ void scatter_run(const RunGeom& r, int bend, int W, int lane,
                                            const float2 (&ac)[MK], float* accf) {
  const float invW = 1.0f / (float)r.Wx;
  float* acci = accf + W * W;
#pragma unroll
  for (int k = 0; k < MK; ++k) {
    const int t = lane + 64 * k;
    int a, b;
    tap_ab(t < r.TT ? t : 0, r.Wx, invW, a, b);
    if (t < r.TT && b < bend) {
      const int li = (r.lv0 + a) * W + (r.lu0 + b);
      atomicAdd(accf + li, ac[k].x);
      atomicAdd(acci + li, ac[k].y);
    }
  }
}

// The work item's bounding box of patch cells in its window (packed by the host as
// origin u, origin v, width, height, 8 bits each): only these cells are cleared and
// flushed, which matters when an item holds few rows.
struct Box {
  int u0, v0, w, h;
};
__device__ __forceinline__ Box box_of(int32_t packed) {
  const uint32_t b = (uint32_t)packed;
  return Box{(int)(b & 0xff), (int)((b >> 8) & 0xff), (int)((b >> 16) & 0xff), (int)(b >> 24)};
}

__device__ __forceinline__ void window_zero(float* accf, int W, const Box& bx) {
  const int n = bx.w * bx.h;
  for (int c = threadIdx.x; c < n; c += GNT) {
    const int a = c / bx.w, b = c - a * bx.w;
    const int o = (bx.v0 + a) * W + bx.u0 + b;
    accf[o] = 0.f;
    accf[W * W + o] = 0.f;
  }
}
__device__ __forceinline__ void window_flush(const float* accf, int W, const Box& bx, int u0,
                                             int v0, int Kx, int Ky, float2* __restrict__ Y) {
  const int n = bx.w * bx.h;
  for (int c = threadIdx.x; c < n; c += GNT) {
    const int a = c / bx.w, b = c - a * bx.w;
    const int o = (bx.v0 + a) * W + bx.u0 + b;
    const float2 v = make_float2(accf[o], accf[W * W + o]);
    if (v.x != 0.f || v.y != 0.f) {
      const int gu = (u0 + bx.u0 + b) & (Kx - 1);
      const int gv = (v0 + bx.v0 + a) & (Ky - 1);
      float2* p = Y + strip_index(gv, gu, Ky);
      unsafeAtomicAdd(&p->x, v.x);
      unsafeAtomicAdd(&p->y, v.y);
    }
  }
}

// MODE 0: fused G^dag G; 1: de-gridding; 2: gridding.
template <int STORE, int MK, int MODE>
__global__ __launch_bounds__(GNT) void k_rows(const WorkItem* __restrict__ wis,
                                              const uint32_t* __restrict__ meta,
                                              const uint32_t* __restrict__ voff,
                                              const int32_t* __restrict__ perm,
                                              const void* __restrict__ vals,
                                              const float2* __restrict__ X,
                                              float2* __restrict__ Y,
                                              float2* __restrict__ vis, int Kx, int Ky,
                                              int W) {
  extern __shared__ float accf[];
  // Items are ordered largest first and dealt round-robin over the XCDs by the hardware,
  // which spreads the dense uv core (many items) evenly and schedules longest first.
  const WorkItem wi = wis[blockIdx.x];
  constexpr bool GATHER = MODE != 2;
  constexpr bool SCATTER = MODE != 1;
  constexpr bool MERGE = SCATTER;   // merge groups save scatter work only
  const Box bx = box_of(wi.box);
  if constexpr (SCATTER) {
    window_zero(accf, W, bx);
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int seg = (wi.nrows + GWAVES - 1) / GWAVES;
  const int r0 = wave * seg;
  const int r1 = min(wi.nrows, r0 + seg);
  float2 xr[MK], ac[MK];
  RunGeom rg{};
  uint32_t cur = 0xffffffffu;
  using Raw = typename RawT<STORE>::type;
  if (r0 >= r1) {
    if constexpr (SCATTER) {
      __syncthreads();
      window_flush(accf, W, bx, wi.u0, wi.v0, Kx, Ky, Y);
    }
    return;
  }
  // Software pipeline, D rows deep.  The metadata of the wavefront's whole segment (at
  // most 128 rows: items hold at most 1024 rows) sits in two VGPRs, lane i holding rows
  // r0 + i and r0 + 64 + i, and is read back with readlane, so the loop never waits on
  // the LDS/scalar counter that the window atomics use.  Value offsets are the running
  // sum of T^2 inside the item; the values of row r + D are requested (after a new run's
  // grid values) before row r is reduced.
  constexpr int D = MK <= 4 ? 4 : (MK <= 7 ? 2 : 1);
  const int nseg = r1 - r0;
  const uint32_t* __restrict__ mrow = meta + wi.row0 + r0;
  const uint32_t mv0 = mrow[min(lane, nseg - 1)];
  const uint32_t mv1 = mrow[min(64 + lane, nseg - 1)];
  auto meta_of = [&](int r) -> uint32_t {
    const int i = r - r0;
    return (uint32_t)__builtin_amdgcn_readlane((int)(i < 64 ? mv0 : mv1), i & 63);
  };
  // gridding: the segment's visibilities are fetched once, like its metadata (lane i
  // holds rows r0 + i and r0 + 64 + i), so that no row waits on its own y
  float2 yv0 = make_float2(0.f, 0.f), yv1 = make_float2(0.f, 0.f);
  if constexpr (MODE == 2) {
    yv0 = vis[perm[wi.row0 + r0 + min(lane, nseg - 1)]];
    yv1 = vis[perm[wi.row0 + r0 + min(64 + lane, nseg - 1)]];
  }
  Raw buf[D][MK];
  uint32_t mb[D], vm[D];                              // row word, slots holding its taps
  int rp = r0;                                        // next row to request
  int64_t vbp = wi.voff + (int64_t)voff[wi.row0 + r0];  // its value offset
  uint32_t mp = meta_of(r0);                          // its metadata
#pragma unroll
  for (int d = 0; d < D; ++d) {
    mb[d] = 0u;
    vm[d] = 0u;
    if (rp < r1) {
      const int Tn = (int)((mp >> 16) & 0xff);
      int tap[MK];
      vm[d] = row_slots<MK, MERGE>(mp, lane, tap);
#pragma unroll
      for (int k = 0; k < MK; ++k) buf[d][k] = load_raw<STORE>(vals, vbp + tap[k]);
      mb[d] = mp;
      vbp += (int64_t)Tn * Tn;
      ++rp;
      mp = rp < r1 ? meta_of(rp) : 0u;
    }
  }
  int dmax = 0;   // largest column offset of the current group's rows
  for (int rb = r0; rb < r1; rb += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int r = rb + d;
      if (r >= r1) break;
      const int row = wi.row0 + r;
      const uint32_t m = mb[d];
      const uint32_t valid = vm[d];
      Raw graw[MK];
#pragma unroll
      for (int k = 0; k < MK; ++k) graw[k] = buf[d][k];
      const uint32_t gk = group_key<MERGE>(m);
      const int du = MERGE ? (int)(m >> 24) : 0;
      if (gk != cur) {
        if constexpr (SCATTER) {
          if (cur != 0xffffffffu) scatter_run<MK>(rg, rg.T + dmax, W, lane, ac, accf);
        }
        cur = gk;
        rg = decode<MK, MERGE>(gk);
        dmax = du;
        if constexpr (GATHER) load_patch_x<MK>(rg, wi.u0, wi.v0, Kx, Ky, X, lane, xr);
#pragma unroll
        for (int k = 0; k < MK; ++k) ac[k] = make_float2(0.f, 0.f);
      } else {
        dmax = du > dmax ? du : dmax;
      }
      if (rp < r1) {  // request row rp = r + D (branch-free, in-bounds loads)
        const int Tn = (int)((mp >> 16) & 0xff);
        int tap[MK];
        vm[d] = row_slots<MK, MERGE>(mp, lane, tap);
#pragma unroll
        for (int k = 0; k < MK; ++k) buf[d][k] = load_raw<STORE>(vals, vbp + tap[k]);
        mb[d] = mp;
        vbp += (int64_t)Tn * Tn;
        ++rp;
        mp = rp < r1 ? meta_of(rp) : 0u;
      }
      // slots outside the row's own patch read an in-bounds dummy and are zeroed: they add
      // nothing to y and nothing to the group's accumulator
      float2 g[MK];
#pragma unroll
      for (int k = 0; k < MK; ++k)
        g[k] = ((valid >> k) & 1u) ? widen<STORE>(graw[k]) : make_float2(0.f, 0.f);
      float yx, yy;
      if constexpr (GATHER) {
        float sx = 0.f, sy = 0.f;
#pragma unroll
        for (int k = 0; k < MK; ++k) {
          sx += g[k].x * xr[k].x - g[k].y * xr[k].y;
          sy += g[k].x * xr[k].y + g[k].y * xr[k].x;
        }
        yx = wave_sum_uniform(sx);
        yy = wave_sum_uniform(sy);
        if constexpr (MODE == 1) {
          if (lane == 0) vis[perm[row]] = make_float2(yx, yy);
        }
      } else {
        const int i = r - r0;
        const float2 yv = i < 64 ? yv0 : yv1;
        yx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(yv.x), i & 63));
        yy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(yv.y), i & 63));
      }
      if constexpr (SCATTER) {
#pragma unroll
        for (int k = 0; k < MK; ++k) {  // += conj(g) y
          ac[k].x += g[k].x * yx + g[k].y * yy;
          ac[k].y += g[k].x * yy - g[k].y * yx;
        }
      }
    }
  }
  if constexpr (SCATTER) {
    if (cur != 0xffffffffu) scatter_run<MK>(rg, rg.T + dmax, W, lane, ac, accf);
    __syncthreads();
    window_flush(accf, W, bx, wi.u0, wi.v0, Kx, Ky, Y);
  }
}

// ------------------------------------------------------------------ launchers

template <typename K>
static hipError_t set_lds(K kern, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int STORE, int MK, int MODE>
static hipError_t launch_one(const WorkItem* wi, int nwi, const uint32_t* meta,
                             const uint32_t* voff, const int32_t* perm, const void* vals,
                             const float2* X, float2* Y, float2* vis, int Kx, int Ky, int win,
                             hipStream_t s) {
  const size_t lds = MODE == 1 ? 0 : (size_t)win * win * sizeof(float2);
  hipError_t e = set_lds(k_rows<STORE, MK, MODE>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_rows<STORE, MK, MODE>), dim3(nwi), dim3(GNT), lds, s, wi, meta, voff,
                     perm, vals, X, Y, vis, Kx, Ky, win);
  return hipGetLastError();
}

template <int STORE, int MODE>
static hipError_t launch_cls(int cls, const WorkItem* wi, int nwi, const uint32_t* meta,
                             const uint32_t* voff, const int32_t* perm, const void* vals,
                             const float2* X, float2* Y, float2* vis, int Kx, int Ky, int win,
                             hipStream_t s) {
#define WF_ONE(MK) \
  launch_one<STORE, MK, MODE>(wi, nwi, meta, voff, perm, vals, X, Y, vis, Kx, Ky, win, s)
  switch (cls) {
    case 0: return WF_ONE(2);
    case 1: return WF_ONE(4);
    case 2: return WF_ONE(7);
    case 3: return WF_ONE(12);
    case 4: return WF_ONE(16);
    default: return WF_ONE(22);
  }
#undef WF_ONE
}

template <int MODE>
static hipError_t launch_mode(int cls, const WorkItem* wi, int nwi, const uint32_t* meta,
                              const uint32_t* voff, const int32_t* perm, const void* vals,
                              wf_store store, const float2* X, float2* Y, float2* vis, int Kx,
                              int Ky, int win, hipStream_t s) {
  if (nwi <= 0) return hipSuccess;
  switch (store) {
    case WF_STORE_F32:
      return launch_cls<WF_STORE_F32, MODE>(cls, wi, nwi, meta, voff, perm, vals, X, Y, vis,
                                            Kx, Ky, win, s);
    case WF_STORE_F16:
      return launch_cls<WF_STORE_F16, MODE>(cls, wi, nwi, meta, voff, perm, vals, X, Y, vis,
                                            Kx, Ky, win, s);
    default:
      return launch_cls<WF_STORE_BF16, MODE>(cls, wi, nwi, meta, voff, perm, vals, X, Y, vis,
                                             Kx, Ky, win, s);
  }
}

hipError_t launch_gtg(int cls, const WorkItem* wi, int nwi, const uint32_t* meta,
                      const uint32_t* voff, const void* vals, wf_store store, const float2* X,
                      float2* Y, int Kx, int Ky, int win, hipStream_t s) {
  return launch_mode<0>(cls, wi, nwi, meta, voff, nullptr, vals, store, X, Y, nullptr, Kx, Ky,
                        win, s);
}

hipError_t launch_degrid(int cls, const WorkItem* wi, int nwi, const uint32_t* meta,
                         const uint32_t* voff, const int32_t* perm, const void* vals,
                         wf_store store, const float2* X, float2* vis, int Kx, int Ky,
                         hipStream_t s) {
  return launch_mode<1>(cls, wi, nwi, meta, voff, perm, vals, store, X, nullptr, vis, Kx, Ky,
                        0, s);
}

hipError_t launch_grid(int cls, const WorkItem* wi, int nwi, const uint32_t* meta,
                       const uint32_t* voff, const int32_t* perm, const void* vals,
                       wf_store store, const float2* vis, float2* Y, int Kx, int Ky, int win,
                       hipStream_t s) {
  return launch_mode<2>(cls, wi, nwi, meta, voff, perm, vals, store, nullptr, Y,
                        const_cast<float2*>(vis), Kx, Ky, win, s);
}

}  // namespace wf
