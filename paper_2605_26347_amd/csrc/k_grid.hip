// Sparse products with the de-gridding matrix G_p (Sect. 3.2, eq. 6) and its adjoint
// (Sect. 3.3, eq. 8).
//
// Rows are sorted by (bin, grid tile, patch side, patch origin) and cut into work
// items that hold one patch-size class; a workgroup owns one work item and each of its
// wavefronts walks a contiguous segment of the item's rows.  The 64 lanes of a
// wavefront hold a row's T x T patch in MK slots each, slot k of lane l being tap
// t = l + 64 k of the row (patch row t / T, column t % T): a row's stored values are
// read as they lie in memory, one coalesced pass, with no per-row index arithmetic.
// The values are read through a buffer resource sized to the row, so that the slots
// past its T^2 taps read zero from the hardware's range check instead of being masked.
// Consecutive rows with the same patch origin and side form a "run" (visibilities
// falling in one grid cell).  Per run
//   * the grid values X of the run's patch are gathered once,
//   * conj(g_k) y_k is accumulated in registers over the run and added into the LDS
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

#include <algorithm>

#include "fft_lds.h"
#include "wf_internal.h"

namespace wf {

constexpr int GWAVES = 8;          // wavefronts per workgroup
constexpr int GNT = GWAVES * 64;

// Word 3 of a raw (untyped, unswizzled) buffer resource on CDNA: 32-bit data format,
// so that a load whose byte offset lies at or past the resource's size returns zero.
constexpr int RSRC_WORD3 = 0x00020000;

// Stored values are loaded in their raw form (two 32-bit words for FP32, one word
// holding two 16-bit halves otherwise) and widened to FP32 only where they are used,
// so that the loads of a row can all be in flight together.
template <int STORE>
struct RawT {
  using type = uint32_t;
};
template <>
struct RawT<WF_STORE_F32> {
  using type = uint2;
};

template <int STORE>
constexpr int value_bytes() {
  return STORE == WF_STORE_F32 ? 8 : 4;
}

template <int STORE>
__device__ __forceinline__ typename RawT<STORE>::type load_tap(__amdgpu_buffer_rsrc_t r,
                                                               int byte_off) {
  if constexpr (STORE == WF_STORE_F32) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
    return make_uint2(v[0], v[1]);
  } else {
    return __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0);
  }
}

template <int STORE>
__device__ __forceinline__ float2 widen(typename RawT<STORE>::type r) {
  if constexpr (STORE == WF_STORE_F32) {
    return make_float2(__uint_as_float(r.x), __uint_as_float(r.y));
  } else if constexpr (STORE == WF_STORE_F16) {
    __half2 h;
    __builtin_memcpy(&h, &r, 4);
    return __half22float2(h);
  } else {
    return make_float2(__uint_as_float(r << 16), __uint_as_float(r & 0xffff0000u));
  }
}

// Sum over the wavefront, returned wave-uniform: DPP butterflies inside each row of 16
// lanes (quad xor 1, quad xor 2, half-row mirror, row mirror) leave every lane with its
// row's sum; broadcasting lane 15 into row 1 (and 47 into row 3), then lane 31 into rows
// 2 and 3, leaves the total in lane 63, which is read into a scalar register.
__device__ __forceinline__ float wave_sum_uniform(float v) {
  v += __builtin_amdgcn_update_dpp(0.f, v, 0xb1, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x4e, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x141, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x140, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x142, 0xa, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0.f, v, 0x143, 0xc, 0xf, false);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// A row's word: window-local patch origin lu0 | lv0 << 8 | patch side T << 16.
struct Run {
  int T, TT, lu0, lv0;
};
__device__ __forceinline__ Run decode(uint32_t m) {
  Run r;
  r.lu0 = m & 0xff;
  r.lv0 = (m >> 8) & 0xff;
  r.T = (m >> 16) & 0xff;
  r.TT = r.T * r.T;
  return r;
}

// Patch coordinates (a = row, b = column) of tap t, invT ~ 1/T to within 2 ulp: exact for
// t < 2^13, T <= 64, since (t + 1/2)/T stays at least 1/(2T) away from an integer.
__device__ __forceinline__ void tap_ab(int t, int T, float invT, int& a, int& b) {
  a = (int)(((float)t + 0.5f) * invT);
  b = t - a * T;
}

// Buffer resource over the T^2 stored values of one row starting at value index vi.
template <int STORE>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* vals, int64_t vi,
                                                           int TT) {
  const char* p = reinterpret_cast<const char*>(vals) + vi * value_bytes<STORE>();
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(p), (short)0,
                                           TT * value_bytes<STORE>(), RSRC_WORD3);
}

// Load the grid values of a run's patch (one per lane and slot).  Slots past the patch
// read its first cell: their stored value is zero, so they add nothing.
template <int MK>
__device__ __forceinline__ void load_patch_x(const Run& r, int u0, int v0, int Kx, int Ky,
                                             const float2* __restrict__ X, int lane,
                                             float2 (&xr)[MK]) {
  const float invT = __builtin_amdgcn_rcpf((float)r.T);
#pragma unroll
  for (int k = 0; k < MK; ++k) {
    const int t = lane + 64 * k;
    int a, b;
    tap_ab(t < r.TT ? t : 0, r.T, invT, a, b);
    const int gu = (u0 + r.lu0 + b) & (Kx - 1);
    const int gv = (v0 + r.lv0 + a) & (Ky - 1);
    xr[k] = X[strip_index(gv, gu, Ky)];
  }
}

// The work item's bounding box of patch cells in its window (packed by the host as
// origin u, origin v, width, height, 8 bits each).  The LDS accumulator holds exactly
// this box, as two planes of FP64 (real parts, then imaginary parts): LDS float atomics
// in FP64 issue an order of magnitude faster than in FP32 on CDNA4, and the wider sums
// cost no precision.  Only these cells are cleared and flushed.
struct Box {
  int u0, v0, w, h;
};
__device__ __forceinline__ Box box_of(int32_t packed) {
  const uint32_t b = (uint32_t)packed;
  return Box{(int)(b & 0xff), (int)((b >> 8) & 0xff), (int)((b >> 16) & 0xff), (int)(b >> 24)};
}

// Add a run's register accumulator into the box accumulator.
template <int MK>
__device__ __forceinline__ void scatter_run(const Run& r, const Box& bx, int lane,
                                            const float2 (&ac)[MK], double* acc) {
  const float invT = __builtin_amdgcn_rcpf((float)r.T);
  double* acci = acc + bx.w * bx.h;
  const int base = (r.lv0 - bx.v0) * bx.w + (r.lu0 - bx.u0);
#pragma unroll
  for (int k = 0; k < MK; ++k) {
    const int t = lane + 64 * k;
    if (t < r.TT) {
      int a, b;
      tap_ab(t, r.T, invT, a, b);
      const int li = base + a * bx.w + b;
      atomicAdd(acc + li, (double)ac[k].x);
      atomicAdd(acci + li, (double)ac[k].y);
    }
  }
}

__device__ __forceinline__ void window_zero(double* acc, const Box& bx) {
  const int n = bx.w * bx.h;
  for (int c = threadIdx.x; c < 2 * n; c += GNT) acc[c] = 0.0;
}
__device__ __forceinline__ void window_flush(const double* acc, const Box& bx, int u0, int v0,
                                             int Kx, int Ky, float2* __restrict__ Y) {
  const int n = bx.w * bx.h;
  for (int c = threadIdx.x; c < n; c += GNT) {
    const float2 v = make_float2((float)acc[c], (float)acc[n + c]);
    if (v.x != 0.f || v.y != 0.f) {
      const int a = c / bx.w, b = c - a * bx.w;
      const int gu = (u0 + bx.u0 + b) & (Kx - 1);
      const int gv = (v0 + bx.v0 + a) & (Ky - 1);
      float2* p = Y + strip_index(gv, gu, Ky);
      unsafeAtomicAdd(&p->x, v.x);
      unsafeAtomicAdd(&p->y, v.y);
    }
  }
}

// One work item on one workgroup.  MODE 0: fused G^dag G; 1: de-gridding; 2: gridding.
// Every thread passes the same two barriers (scattering modes), whatever its rows.
template <int STORE, int MK, int MODE>
__device__ __forceinline__ void row_item(const WorkItem& wi, const uint32_t* __restrict__ meta,
                                         const uint32_t* __restrict__ voff,
                                         const int32_t* __restrict__ perm,
                                         const void* __restrict__ vals,
                                         const float2* __restrict__ X, float2* __restrict__ Y,
                                         float2* __restrict__ vis, int Kx, int Ky,
                                         double* acc) {
  constexpr bool GATHER = MODE != 2;
  constexpr bool SCATTER = MODE != 1;
  constexpr int VB = value_bytes<STORE>();
  const Box bx = box_of(wi.box);
  if constexpr (SCATTER) {
    window_zero(acc, bx);
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int seg = (wi.nrows + GWAVES - 1) / GWAVES;
  const int r0 = wave * seg;
  const int r1 = min(wi.nrows, r0 + seg);
  float2 xr[MK], ac[MK];
  Run rg{};
  uint32_t cur = 0xffffffffu;
  using Raw = typename RawT<STORE>::type;
  if (r0 >= r1) {
    if constexpr (SCATTER) {
      __syncthreads();
      window_flush(acc, bx, wi.u0, wi.v0, Kx, Ky, Y);
    }
    return;
  }
  // Software pipeline, D rows deep.  The metadata of the wavefront's whole segment (at
  // most 128 rows: items hold at most 1024 rows) sits in two VGPRs, lane i holding rows
  // r0 + i and r0 + 64 + i, and is read back with readlane, so the loop never waits on
  // the LDS/scalar counter that the window atomics use.  Value offsets are the running
  // sum of T^2 inside the item; the values of row r + D are requested (after a new run's
  // grid values) before row r is reduced.
  constexpr int D = MK <= 4 ? 4 : (MK <= 16 || STORE != WF_STORE_F32 ? 2 : 1);
  // the next run's grid values are gathered while the current run is reduced (one run
  // ahead), where registers allow
  constexpr bool PREFETCH = GATHER && (MK <= 12 || (MK <= 16 && STORE != WF_STORE_F32));
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
  float2 xn[PREFETCH ? MK : 1];                       // grid values of the next run
  uint32_t nm = 0xffffffffu;                          // ... and its row word
  uint32_t mb[D];                                     // row words of the rows in flight
  int rp = r0;                                        // next row to request
  int64_t vbp = wi.voff + (int64_t)voff[wi.row0 + r0];  // its first value
  uint32_t mp = meta_of(r0);                          // its word
  auto request = [&](int d) {
    const int Tn = (int)((mp >> 16) & 0xff);
    const __amdgpu_buffer_rsrc_t rs = row_rsrc<STORE>(vals, vbp, Tn * Tn);
#pragma unroll
    for (int k = 0; k < MK; ++k) buf[d][k] = load_tap<STORE>(rs, (lane + 64 * k) * VB);
    mb[d] = mp;
    vbp += (int64_t)Tn * Tn;
    ++rp;
    mp = rp < r1 ? meta_of(rp) : 0u;
  };
#pragma unroll
  for (int d = 0; d < D; ++d) {
    mb[d] = 0u;
    if (rp < r1) request(d);
  }
  for (int rb = r0; rb < r1; rb += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int r = rb + d;
      if (r >= r1) break;
      const int row = wi.row0 + r;
      const uint32_t m = mb[d];
      Raw graw[MK];
#pragma unroll
      for (int k = 0; k < MK; ++k) graw[k] = buf[d][k];
      if (m != cur) {
        if constexpr (SCATTER) {
          if (cur != 0xffffffffu) scatter_run<MK>(rg, bx, lane, ac, acc);
        }
        cur = m;
        rg = decode(m);
        if constexpr (PREFETCH) {
          if (nm == m) {
#pragma unroll
            for (int k = 0; k < MK; ++k) xr[k] = xn[k];
          } else {
            load_patch_x<MK>(rg, wi.u0, wi.v0, Kx, Ky, X, lane, xr);
          }
          int q = r + 1;
          while (q < r1 && meta_of(q) == m) ++q;
          nm = q < r1 ? meta_of(q) : 0xffffffffu;
          if (q < r1) load_patch_x<MK>(decode(nm), wi.u0, wi.v0, Kx, Ky, X, lane, xn);
        } else if constexpr (GATHER) {
          load_patch_x<MK>(rg, wi.u0, wi.v0, Kx, Ky, X, lane, xr);
        }
#pragma unroll
        for (int k = 0; k < MK; ++k) ac[k] = make_float2(0.f, 0.f);
      }
      if (rp < r1) request(d);   // row r + D (in-bounds: past a row's taps reads zero)
      float2 g[MK];
#pragma unroll
      for (int k = 0; k < MK; ++k) g[k] = widen<STORE>(graw[k]);
      float yx, yy;
      if constexpr (GATHER) {
        float sx = 0.f, sy = 0.f;
#pragma unroll
        for (int k = 0; k < MK; ++k) {  // y += g X, one fused multiply-add per term
          sx = fmaf(g[k].x, xr[k].x, sx);
          sx = fmaf(-g[k].y, xr[k].y, sx);
          sy = fmaf(g[k].x, xr[k].y, sy);
          sy = fmaf(g[k].y, xr[k].x, sy);
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
          ac[k].x = fmaf(g[k].x, yx, ac[k].x);
          ac[k].x = fmaf(g[k].y, yy, ac[k].x);
          ac[k].y = fmaf(g[k].x, yy, ac[k].y);
          ac[k].y = fmaf(-g[k].y, yx, ac[k].y);
        }
      }
    }
  }
  if constexpr (SCATTER) {
    if (cur != 0xffffffffu) scatter_run<MK>(rg, bx, lane, ac, acc);
    __syncthreads();
    window_flush(acc, bx, wi.u0, wi.v0, Kx, Ky, Y);
  }
}

template <int STORE, int MK, int MODE>
__global__ __launch_bounds__(GNT) void k_rows(const WorkItem* __restrict__ wis,
                                              const uint32_t* __restrict__ meta,
                                              const uint32_t* __restrict__ voff,
                                              const int32_t* __restrict__ perm,
                                              const void* __restrict__ vals,
                                              const float2* __restrict__ X,
                                              float2* __restrict__ Y,
                                              float2* __restrict__ vis, int Kx, int Ky) {
  extern __shared__ double acc[];
  // Items are ordered largest first and dealt round-robin over the XCDs by the hardware,
  // which spreads the dense uv core (many items) evenly and schedules longest first.
  row_item<STORE, MK, MODE>(wis[blockIdx.x], meta, voff, perm, vals, X, Y, vis, Kx, Ky, acc);
}

// Persistent form over the items of every layer of a sweep (one patch class): resident
// workgroups take items from a queue (queue[0]) until it is drained; each item's layer
// (its bin field) selects its grids, its row data and its visibilities (vis_base plus
// the layer's offset).  The last workgroup to leave clears the queue and the exit count
// (queue[1]), so that the next launch, or the next replay of a captured graph, starts
// from zero without a separate clearing step.
template <int STORE, int MK, int MODE>
__global__ __launch_bounds__(GNT) void k_rows_sweep(const WorkItem* __restrict__ wis,
                                                    int nitems,
                                                    const SweepLayer* __restrict__ layers,
                                                    float2* __restrict__ vis_base,
                                                    int* __restrict__ queue, int Kx, int Ky) {
  extern __shared__ double acc[];
  __shared__ int slot;
  for (;;) {
    if (threadIdx.x == 0) slot = atomicAdd(queue, 1);
    __syncthreads();
    const int i = slot;
    __syncthreads();
    if (i >= nitems) break;
    const WorkItem wi = wis[i];
    const SweepLayer& L = layers[wi.bin];
    row_item<STORE, MK, MODE>(wi, L.meta, L.voff, L.perm, L.vals, L.X, L.Y,
                              vis_base ? vis_base + L.vis_off : nullptr, Kx, Ky, acc);
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(queue + 1, 1) == (int)gridDim.x - 1) {
      atomicExch(queue, 0);
      atomicExch(queue + 1, 0);
    }
  }
}

// ------------------------------------------------------------------ launchers

template <typename K>
static hipError_t set_lds(K kern, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Largest (odd) patch side of a class of MK taps per lane.
constexpr int class_tmax(int mk) {
  int t = 1;
  while ((t + 2) * (t + 2) <= 64 * mk) t += 2;
  return t;
}

template <int STORE, int MK, int MODE>
static hipError_t launch_one(const WorkItem* wi, int nwi, const uint32_t* meta,
                             const uint32_t* voff, const int32_t* perm, const void* vals,
                             const float2* X, float2* Y, float2* vis, int Kx, int Ky, int tile,
                             hipStream_t s) {
  // the box accumulator of an item: rows' cells lie in one tile and their patches of
  // side <= class_tmax reach tile + side - 1 cells per axis; two FP64 planes
  const size_t side = (size_t)tile + class_tmax(MK) - 1;
  const size_t lds = MODE == 1 ? 0 : side * side * 2 * sizeof(double);
  hipError_t e = set_lds(k_rows<STORE, MK, MODE>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_rows<STORE, MK, MODE>), dim3(nwi), dim3(GNT), lds, s, wi, meta, voff,
                     perm, vals, X, Y, vis, Kx, Ky);
  return hipGetLastError();
}

template <int STORE, int MODE>
static hipError_t launch_cls(int cls, const WorkItem* wi, int nwi, const uint32_t* meta,
                             const uint32_t* voff, const int32_t* perm, const void* vals,
                             const float2* X, float2* Y, float2* vis, int Kx, int Ky, int tile,
                             hipStream_t s) {
#define WF_ONE(MK) \
  launch_one<STORE, MK, MODE>(wi, nwi, meta, voff, perm, vals, X, Y, vis, Kx, Ky, tile, s)
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
                              int Ky, int tile, hipStream_t s) {
  if (nwi <= 0) return hipSuccess;
  switch (store) {
    case WF_STORE_F32:
      return launch_cls<WF_STORE_F32, MODE>(cls, wi, nwi, meta, voff, perm, vals, X, Y, vis,
                                            Kx, Ky, tile, s);
    case WF_STORE_F16:
      return launch_cls<WF_STORE_F16, MODE>(cls, wi, nwi, meta, voff, perm, vals, X, Y, vis,
                                            Kx, Ky, tile, s);
    default:
      return launch_cls<WF_STORE_BF16, MODE>(cls, wi, nwi, meta, voff, perm, vals, X, Y, vis,
                                             Kx, Ky, tile, s);
  }
}

template <int STORE, int MK, int MODE>
static hipError_t launch_sweep_one(const WorkItem* wi, int nwi, const SweepLayer* layers,
                                   float2* vis_base, int* queue, int Kx, int Ky, int tile,
                                   int grid_cap, hipStream_t s) {
  const size_t side = (size_t)tile + class_tmax(MK) - 1;
  const size_t lds = MODE == 1 ? 0 : side * side * 2 * sizeof(double);
  hipError_t e = set_lds(k_rows_sweep<STORE, MK, MODE>, lds);
  if (e != hipSuccess) return e;
  // resident workgroups only: as many as the device holds at once, capped by the items
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rows_sweep<STORE, MK, MODE>,
                                                   GNT, lds);
  if (e != hipSuccess) return e;
  const int grid = std::max(1, std::min(nwi, std::max(1, per_cu) * grid_cap));
  hipLaunchKernelGGL((k_rows_sweep<STORE, MK, MODE>), dim3(grid), dim3(GNT), lds, s, wi, nwi,
                     layers, vis_base, queue, Kx, Ky);
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_sweep_mode(int cls, const WorkItem* wi, int nwi,
                                    const SweepLayer* layers, wf_store store, float2* vis_base,
                                    int* queue, int Kx, int Ky, int tile, int ncu,
                                    hipStream_t s) {
  if (nwi <= 0) return hipSuccess;
#define WF_SW(ST, MK) \
  launch_sweep_one<ST, MK, MODE>(wi, nwi, layers, vis_base, queue, Kx, Ky, tile, ncu, s)
#define WF_SWC(ST)                 \
  switch (cls) {                   \
    case 0: return WF_SW(ST, 2);   \
    case 1: return WF_SW(ST, 4);   \
    case 2: return WF_SW(ST, 7);   \
    case 3: return WF_SW(ST, 12);  \
    case 4: return WF_SW(ST, 16);  \
    default: return WF_SW(ST, 22); \
  }
  switch (store) {
    case WF_STORE_F32: WF_SWC(WF_STORE_F32)
    case WF_STORE_F16: WF_SWC(WF_STORE_F16)
    default: WF_SWC(WF_STORE_BF16)
  }
#undef WF_SWC
#undef WF_SW
}

hipError_t launch_rows_sweep(int mode, int cls, const WorkItem* wi, int nwi,
                             const SweepLayer* layers, wf_store store, float2* vis_base,
                             int* queue, int Kx, int Ky, int tile, int ncu, hipStream_t s) {
  switch (mode) {
    case 0: return launch_sweep_mode<0>(cls, wi, nwi, layers, store, vis_base, queue, Kx, Ky,
                                        tile, ncu, s);
    case 1: return launch_sweep_mode<1>(cls, wi, nwi, layers, store, vis_base, queue, Kx, Ky,
                                        tile, ncu, s);
    default: return launch_sweep_mode<2>(cls, wi, nwi, layers, store, vis_base, queue, Kx, Ky,
                                         tile, ncu, s);
  }
}

hipError_t launch_gtg(int cls, const WorkItem* wi, int nwi, const uint32_t* meta,
                      const uint32_t* voff, const void* vals, wf_store store, const float2* X,
                      float2* Y, int Kx, int Ky, int tile, hipStream_t s) {
  return launch_mode<0>(cls, wi, nwi, meta, voff, nullptr, vals, store, X, Y, nullptr, Kx, Ky,
                        tile, s);
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
                       wf_store store, const float2* vis, float2* Y, int Kx, int Ky, int tile,
                       hipStream_t s) {
  return launch_mode<2>(cls, wi, nwi, meta, voff, perm, vals, store, nullptr, Y,
                        const_cast<float2*>(vis), Kx, Ky, tile, s);
}

}  // namespace wf
