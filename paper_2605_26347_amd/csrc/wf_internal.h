// Internal declarations of the widefield operator library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <exception>
#include <new>
#include <string>
#include <vector>

#include "wf.h"

namespace wf {

// Complex grids are stored in strips of SW adjacent columns: element (row r, column q)
// of an R x Q complex array lives at ((q / SW) * R + r) * SW + q % SW.  A 128-byte
// line then holds one row of one strip, so row passes touch whole lines and column
// passes read each strip as one contiguous block.
constexpr int SW = 16;

__host__ __device__ inline int64_t strip_index(int r, int q, int R) {
  return ((int64_t)(q >> 4) * R + r) * SW + (q & (SW - 1));
}

// One unit of work of the fused G^dag G, de-gridding and gridding kernels: a run of
// consecutive sorted rows of one bin whose patch centres fall in one grid tile.  The
// kernel accumulates into an LDS window of side W = tile + 2 halo whose origin on the
// periodic grid is (u0, v0) (possibly negative or past the edge; wrapped mod K).
struct WorkItem {
  int64_t voff;   // index (complex units) of the first value of the first row
  int32_t row0;   // first sorted row
  int32_t nrows;  // rows in this item
  int32_t u0, v0; // window origin
  int32_t bin;
  int32_t box;    // window-local bounding box of the rows' patches: u0 | v0 << 8 |
                  // width << 16 | height << 24
};
static_assert(sizeof(WorkItem) == 32, "WorkItem layout");

// Patch-size classes of the row kernels: class c covers T*T <= 64 * cls_taps(c) taps,
// i.e. patch sides up to 11, 15, 21, 27, 31, 37.
constexpr int NCLS = 6;
__host__ __device__ inline int tap_class(int T) {
  const int k = (T * T + 63) / 64;
  return k <= 2 ? 0 : k <= 4 ? 1 : k <= 7 ? 2 : k <= 12 ? 3 : k <= 16 ? 4 : 5;
}

// Interleaved bits of a base tile's (v, u) indices (10 bits each): the tiles of every
// aligned 2^s x 2^s block are consecutive in this order, so the rows of one patch class in
// such a block form one contiguous range of the sorted rows.
__host__ __device__ inline uint32_t tile_morton(uint32_t tv, uint32_t tu) {
  uint32_t m = 0;
  for (int b = 0; b < 10; ++b)
    m |= (((tu >> b) & 1u) << (2 * b)) | (((tv >> b) & 1u) << (2 * b + 1));
  return m;
}
inline void tile_unmorton(uint32_t m, int* tv, int* tu) {
  int v = 0, u = 0;
  for (int b = 0; b < 10; ++b) {
    u |= (int)((m >> (2 * b)) & 1u) << b;
    v |= (int)((m >> (2 * b + 1)) & 1u) << b;
  }
  *tv = v;
  *tu = u;
}
// Sort key of a built row: bin 8 | patch class 3 | base tile (interleaved) 20 | patch
// side 6 | cell v in the tile 7 | cell u 7 | 13 zero bits.
constexpr int KEY_LO_BIT = 13;
__host__ __device__ inline uint64_t row_key(int bin, int T, uint32_t tv, uint32_t tu,
                                            uint32_t lv, uint32_t lu) {
  return ((uint64_t)bin << 56) | ((uint64_t)tap_class(T) << 53) |
         ((uint64_t)tile_morton(tv, tu) << 33) | ((uint64_t)T << 27) | ((uint64_t)lv << 20) |
         ((uint64_t)lu << 13);
}

// Per-row metadata word: window-local patch origin and patch side.
__host__ __device__ inline uint32_t pack_meta(int lu0, int lv0, int T) {
  return (uint32_t)lu0 | ((uint32_t)lv0 << 8) | ((uint32_t)T << 16);
}
// Taps per lane of patch class c (the row kernels' MK).
__host__ __device__ constexpr int class_mk(int c) {
  return c == 0 ? 2 : c == 1 ? 4 : c == 2 ? 7 : c == 3 ? 12 : c == 4 ? 16 : 22;
}
// One (channel, bin) layer of a sweep: its work grids, pruning masks, row data of G,
// w-layer centroid, channel, and the offset of its channel's visibilities.  A sweep
// holds the grids of every layer at once so that each stage of the apply runs as one
// launch over all layers.
struct SweepLayer {
  float2* X;
  float2* Y;
  float2* A;
  const uint32_t* smask;   // needed column strips (null: all)
  const uint32_t* tile;    // needed tiles (null: all)
  const void* vals;
  const uint32_t* meta;
  const uint32_t* voff;
  const int32_t* perm;
  const float2* ctab;      // column table of the w-layer modulation (null: direct form)
  int64_t vis_off;         // first visibility of the layer's channel in caller order
  double wp;               // w-layer centroid
  int32_t chan;
  int32_t pad;
};

// Active uv support of one bin for the column passes: tiles that hold rows, dilated by
// one tile (the LDS windows reach into neighbours), the column strips under them, and the
// column groups (col_width columns each) that cover those strips.
struct ColPrune {
  const uint32_t* strip;   // [Kx/16] bits
  const uint32_t* tile;    // [Ky/tile][Kx/tile] bits
  const int32_t* groups;   // active column-group indices
  int ngroups;
  int tiles_x;
  int tsh;                 // log2(tile)
};

// Columns per workgroup of the column passes for a column length of Ky.
inline int col_width_for(int Ky) { return (16384 / Ky) > 16 ? 16 : (16384 / Ky); }

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Parameters of the residual-w kernel and interpolation kernel, shared by the build
// kernels.
struct KernelParams {
  double Lx, Ly;      // field sides nx*cell, ny*cell
  double oLx, oLy;    // padded field sides
  double alpha;       // sampling margin
  double eps;         // dropped energy
  double beta;        // Kaiser-Bessel shape
  double i0beta;      // I0(beta)
  int J;              // Kaiser-Bessel support
  int smax;           // kernel side cap
  int o;              // oversampling
};

// A run of consecutive sorted rows of one (bin, tile, patch class); work items are
// pieces of one group.
struct RowGroup {
  int64_t voff;   // index (complex units) of the group's first value
  int32_t row0, nrows;
  int32_t u0, v0; // LDS window origin of the tile
  int32_t bin, cls;
};

// One active grid tile of a bin's holographic matrix: dense stencil of side D, values
// [D * D][tile * tile] from voff (complex units) on.
struct HTile {
  int32_t tile;   // tv * tiles_x + tu
  int32_t D;
  int64_t voff;
};
static_assert(sizeof(HTile) == 16, "HTile layout");

// Host index of the stored rows for the diagnostic row reader (built on first use).
// Rows of one order (caller or sorted) grouped by kernel-side class, each class's rows
// ascending: class c occupies [off[c], off[c + 1]) of the device list d and its host copy.
struct RowClasses {
  const int32_t* d = nullptr;
  std::vector<int32_t> h;
  int64_t off[5] = {0, 0, 0, 0, 0};
};
// One launch range's rows per class: device pointers into a RowClasses list and counts.
struct ClassSlices {
  const int32_t* rows[4];
  int64_t n[4];
};

// Rows of a factorised on-the-fly chunk by kept-kernel side class: n' <= 3, 7, 11, 15,
// 21, 31 (the expansion's lane slots are sized for the class's largest n').
constexpr int NXC = 6;
__host__ __device__ constexpr int xclass_of(int np) {
  return np <= 3 ? 0 : np <= 7 ? 1 : np <= 11 ? 2 : np <= 15 ? 3 : np <= 21 ? 4 : 5;
}
struct ExpSlices {
  const int32_t* rows[NXC];
  int64_t n[NXC];
};

struct DebugIndex {
  uint64_t gen = 0;                        // operator generation + 1 when valid
  std::vector<int32_t> sorted_of;          // caller row -> sorted row
  std::vector<int32_t> item_of;            // sorted row -> work item
  std::vector<WorkItem> items;
};

struct ChanOp {
  double freq = 0, scale = 0;
  int64_t vis_off = 0;   // offset of this channel's rows in the caller's vis vector
  int64_t nrows = 0;     // rows built (flagged rows excluded)
  int64_t nvis = 0;      // rows of the channel in the caller's vis vector
  DevBuf flagged;        // int32 caller-order indices of the flagged rows
  int64_t nflag = 0;
  int P = 0;
  std::vector<double> centroids;
  std::vector<int64_t> bin_row0, bin_nrows;
  std::vector<int32_t> bin_wi0, bin_nwi;
  std::vector<int32_t> cls_wi0, cls_nwi;   // [bin * NCLS + class]
  std::vector<int64_t> bin_taps;           // stored values per bin
  std::vector<RowGroup> groups;            // in sorted-row order
  int32_t max_rows = 1024;                 // rows per work item of the current split
  // per bin: work items cover aligned blocks of 2^s x 2^s base tiles (item tile side
  // tile << s); the rows' patch words are relative to their item's window
  std::vector<int8_t> bin_tsh;
  // per bin: the column table of its w-layer modulation ([P][nx] complex FP32, FP64
  // phases), used by the row FFT passes where cfast[p] (field and w_p small enough for
  // the series forms; otherwise the direct form)
  DevBuf ctab;
  std::vector<uint8_t> cfast;
  double measured_ms = 0;                  // last timed apply of this channel (0 = none)
  int64_t ntaps = 0;
  int64_t nwork = 0;
  bool holo = false;                       // strategy (b): H only
  DevBuf htiles, hvals;                    // HTile [tiles of all bins], stencil values
  std::vector<int64_t> h_t0, h_nt;         // per bin: first tile, tile count
  std::vector<int32_t> h_dmax;             // per bin: largest stencil side
  int64_t h_values = 0;                    // stored stencil values (complex)
  // strategy (c), G on the fly: no values are kept; each bin is cut into chunks of whole
  // row groups whose values are rebuilt into a branch's transient buffer at every apply
  bool otf = false;
  DevBuf uvw, wts, uperm, row_wi, mids, cents, crow;  // value-pass inputs on the device
  std::vector<ClassSlices> ck_cls;         // per chunk: its rows by kernel-side class
  // factorised form: each row's kept residual kernel (times its weight) is stored, and an
  // apply only convolves it with the Kaiser-Bessel taps
  bool fact = false;
  DevBuf khat, kof, ktap;                  // kernels (value format); per sorted row its
                                           // kernel offset and 2J taps (FP32)
  std::vector<int64_t> ck_kbase;           // per chunk: its first kernel value
  DevBuf xrow;                             // sorted rows of every chunk by n' class
  std::vector<ExpSlices> ck_xcls;          // per chunk: its slices of xrow
  std::vector<int32_t> gchunk;             // chunk of each row group
  std::vector<int64_t> ck_s0, ck_s1, ck_vbase, ck_taps;  // sorted rows, first value, values
  std::vector<int32_t> ck_first, ck_count; // per bin: first chunk, chunk count
  std::vector<int32_t> ck_wi0, ck_nwi;     // [chunk * NCLS + class] work-item ranges
  int64_t ck_max = 0;                      // values of the largest chunk
  DevBuf meta, voff, perm, vals, work;
  DevBuf prune;                            // per bin: strip bits, tile bits, groups
  std::vector<size_t> pr_strip, pr_tile, pr_groups;  // byte offsets into prune per bin
  std::vector<int32_t> pr_ngroups;
  std::vector<double> active_tile_frac;
  wf_plan_info info{};
  mutable DebugIndex dbg;
};

struct Profiler {
  bool enabled = false;
  std::vector<hipEvent_t> ev;   // pairs
  size_t used = 0;
  int64_t launches = 0;
  double total_ms = 0;
};

constexpr int NPROF = 6;

// One concurrent branch of an apply: its own stream and work grids (branch 0 runs on the
// caller's stream and owns the operator's first set of grids).  acc receives the partial
// image sum of a channel whose bins are split over several branches.
struct Branch {
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  DevBuf X, Y, A, acc;
  DevBuf gbuf;   // transient G values of on-the-fly channels
  DevBuf net_x, net_pred;   // network inputs and outputs (on-the-fly with the network)
};

// Work of one branch for one channel: a list of its non-empty bins.  A direct segment
// writes the channel's output itself; the others accumulate into their branch's acc,
// added into the output after the join.
struct Segment {
  int chan = 0;
  int branch = 0;
  bool direct = true;
  std::vector<int> bins;
};

// Layer-batched applies (wf_set_sweep): the grids of every (channel, bin) layer at once,
// the layer table, the (layer, column group) pairs of the column passes, each channel's
// layer range, and the lanes.
//
// One lane of a sweep: a contiguous range of channels (and so of layers, column pairs
// and work items) whose stages run in order on the lane's stream.  Lane k > 0 starts once
// lane k - 1 has issued its forward passes, so that one lane's fused kernel runs beside
// the next lane's FFT passes.
struct SweepLane {
  int l0 = 0, nl = 0;              // layers [l0, l0 + nl)
  int p0 = 0, np = 0;              // column pairs [p0, p0 + np)
  int c0 = 0, nc = 0;              // channels [c0, c0 + nc)
  DevBuf items[2 * NCLS];          // work items per (patch class, item-tile shift) of all
                                   // its layers (bin = layer index), largest first, drained
                                   // by one persistent launch through a two-int queue
  int nitems[2 * NCLS] = {};
  hipStream_t s = nullptr;         // lanes > 0: a stream of their own (default priority)
  hipEvent_t fwd = nullptr;        // the lane's forward passes are issued
  hipEvent_t end = nullptr;        // all of the lane's stages are issued
};

struct Sweep {
  bool on = false;
  int nlayers = 0;
  std::vector<DevBuf> grids;         // per layer: X, Y, A
  DevBuf layers;                     // SweepLayer [nlayers]
  DevBuf pairs;                      // int2 [npairs]
  int npairs = 0;
  DevBuf chan_layers;                // int2 [nchan]: first layer, count
  // work items per (patch class, item-tile shift): list k * 2 + s
  static constexpr int NLIST = 2 * NCLS;
  static constexpr int MAXLANES = 4;
  std::vector<SweepLane> lanes;
  DevBuf queues;                     // int [lanes][2 * NLIST]
  DevBuf done;                       // int [nchan]: workgroups finished (completion stamps)
  hipEvent_t fork = nullptr;         // the caller's stream reached the sweep
  int ncu = 0;
};

}  // namespace wf

struct wf_op {
  wf_options opt;
  wf_image_shape shape;
  int Kx = 0, Ky = 0;
  int tile = 64, halo = 10, win = 84;
  int max_tsh = 0;   // largest item-tile shift whose LDS accumulator fits
  int device = 0;
  wf::KernelParams kp;
  std::vector<wf::ChanOp> chans;
  int64_t total_rows = 0;
  wf::DevBuf twx, twy, sx, sy;
  wf::Profiler prof[wf::NPROF];
  std::vector<wf::Branch> br;        // br[0]: the operator's own grids
  int nbranch = 1;                   // branches the segments use
  std::vector<wf::Segment> segs;     // issue order of the applies
  hipEvent_t fork = nullptr;
  wf::DevBuf stamps;                 // [nchan + 1] wall-clock stamps, when enabled
  bool stamping = false;
  bool capturing = false;
  uint64_t generation = 0;           // bumped when work items or branches change
  wf::DevBuf fb_h, fb_x, fb_c, fb_red;  // forward-backward work images and reductions
  size_t otf_bytes = 0;              // transient value buffer per branch (strategy (c))
  wf::DevBuf otf_mis;                // counters the on-the-fly value pass writes
  // strategy (c) with the kernel network: a copy of its parameters taken at build (FP32
  // and the BF16 inference form), so that every apply infers exactly what the build did
  bool net_otf = false;
  float net_logtol = 0.f;
  wf::DevBuf net_params, net_wt;
  wf::Sweep sweep;                   // layer-batched applies (wf_set_sweep)
};

// Residual-kernel network: FP32 parameters with Adam state, per-batch activations, and
// the transposed BF16 weights of the inference kernel (refreshed when the parameters
// change).
struct wf_mlp {
  int device = 0;
  wf::DevBuf params, grad, m, v;
  mutable wf::DevBuf wt;          // BF16 [2][3 x 256 x 256 + 512 x 256] (high, residual)
  mutable bool wt_dirty = true;
  int64_t t = 0;                  // Adam steps taken
  int bcap = 0;                   // batch capacity of the buffers below
  wf::DevBuf xb, tb, P, dP, dA, dB, idx, loss;
  wf::DevBuf H[4], Z[4];
};

namespace wf {

// ------------------------------------------------------------------ kernel launchers
// (defined in the .hip translation units; all asynchronous on `s`)

// Pruning arguments may be null (full grid).
// Column table of the w-layer modulation of bin wp (see the FFT passes): ct[nx].
hipError_t launch_chirp_table(float2* ct, int nx, double cell, double wp, const float* sx,
                              hipStream_t s);
hipError_t launch_fwd_rows(const float* img, float2* A, const float2* tw, const float* sx,
                           const float* sy, int nx, int ny, int Kx, double cell, double wp,
                           const uint32_t* smask, const float2* ctab, hipStream_t s);
hipError_t launch_fwd_cols(const float2* A, float2* X, const float2* tw, int ny, int Kx,
                           int Ky, const ColPrune* pr, hipStream_t s);
hipError_t launch_inv_cols(float2* Y, float2* A, const float2* tw, int ny, int Kx, int Ky,
                           const ColPrune* pr, hipStream_t s);
// mode 0: out complex, overwrite; 1: complex, accumulate; 2: real part, overwrite;
// 3: real part, accumulate
hipError_t launch_inv_rows(const float2* A, void* out, const float2* tw, const float* sx,
                           const float* sy, int nx, int ny, int Kx, double cell, double wp,
                           int mode, const uint32_t* smask, const float2* ctab,
                           hipStream_t s);

// Row kernels over the work items of one patch-size class `cls`; `tile` is the grid
// tile side of the sort (it sizes each item's LDS accumulator).
hipError_t launch_gtg(int cls, const WorkItem* wi, int nwi, const uint32_t* meta,
                      const uint32_t* voff, const void* vals, wf_store store, const float2* X,
                      float2* Y, int Kx, int Ky, int tile, hipStream_t s);
hipError_t launch_degrid(int cls, const WorkItem* wi, int nwi, const uint32_t* meta,
                         const uint32_t* voff, const int32_t* perm, const void* vals,
                         wf_store store, const float2* X, float2* vis, int Kx, int Ky,
                         hipStream_t s);
hipError_t launch_grid(int cls, const WorkItem* wi, int nwi, const uint32_t* meta,
                       const uint32_t* voff, const int32_t* perm, const void* vals,
                       wf_store store, const float2* vis, float2* Y, int Kx, int Ky, int tile,
                       hipStream_t s);
hipError_t launch_fill_zero(void* p, int64_t nfloats, hipStream_t s);
// out[idx[i]] = 0 for the n complex values listed (flagged visibilities).
hipError_t launch_scatter_zero(float2* out, const int32_t* idx, int64_t n, hipStream_t s);
// Briggs weighting: density of natural weights over the nx x ny Fourier cells (each
// sample and its conjugate, FP64 atomics); sums[0] += sum w W_c(k), sums[1] += sum w;
// out = sqrt(w / (1 + W_c(k) f2)).  w null: ones; flags non-zero: weight 0.
hipError_t launch_density(const double* uvw, int64_t n, double scale, double du, double dv,
                          int nx, int ny, const float* w, const uint8_t* flags, double* W,
                          hipStream_t s);
hipError_t launch_briggs_sums(const double* uvw, int64_t n, double scale, double du,
                              double dv, int nx, int ny, const float* w,
                              const uint8_t* flags, const double* W, double* sums,
                              hipStream_t s);
hipError_t launch_briggs_out(const double* uvw, int64_t n, double scale, double du, double dv,
                             int nx, int ny, const float* w, const uint8_t* flags,
                             const double* W, double f2, float* out, hipStream_t s);
// Allocation-free Briggs weighting: the device address of this device's static scratch
// (density then two sums), found once per device; f^2 = a2 sums[1] / sums[0] on the device.
hipError_t briggs_scratch(double** out);
hipError_t launch_briggs_out_dev(const double* uvw, int64_t n, double scale, double du,
                                 double dv, int nx, int ny, const float* w,
                                 const uint8_t* flags, const double* W, const double* sums,
                                 double a2, float* out, hipStream_t s);
hipError_t launch_stamp(unsigned long long* dst, hipStream_t s);
hipError_t launch_add_into(float* out, const float* in, int64_t nfloats, hipStream_t s);
// Forward-backward driver (eq. 4): x <- max(x + gamma (dirty - hx) - t, 0); *out = a.b;
// dst = src / sqrt(*nrm2); fill with a value; real part of complex values.
hipError_t launch_fb_step(float* x, const float* dirty, const float* hx, float gamma, float t,
                          int64_t n, hipStream_t s);
hipError_t launch_dot(const float* a, const float* b, int64_t n, float* out, hipStream_t s);
hipError_t launch_normalize(float* dst, const float* src, int64_t n, const float* nrm2,
                            hipStream_t s);
hipError_t launch_fill_value(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_real_part(const float2* src, float* dst, int64_t n, hipStream_t s);
// Holographic matrix: accumulate the stencils of one bin from its work items (values g
// of that bin from vbase on, FP32), pack FP32 stencils to FP16 / BF16, and apply.
hipError_t launch_hbuild(const WorkItem* wi, int nwi, const uint32_t* meta, const uint32_t* voff,
                         const float2* g, int64_t vbase, const int32_t* slot_of_tile,
                         const HTile* ht, int tiles_x, int tsh, int Kx, int Ky, float* h,
                         hipStream_t s);
hipError_t launch_hpack(const float2* src, uint32_t* dst, int64_t n, wf_store store,
                        int* overflow, hipStream_t s);
hipError_t launch_happly(const HTile* ht, int ntiles, int Dmax, const void* hv, wf_store store,
                         const float2* X, float2* Y, int tiles_x, int tsh, int Kx, int Ky,
                         hipStream_t s);
hipError_t launch_strip_to_rowmajor(const float2* src, float2* dst, int R, int Q,
                                    hipStream_t s);
// Sweep stages (one launch over every layer; grid sides 2048 .. 16384 with K = 2 n).
// Forward rows over all layers (images of all channels from img); forward or inverse
// columns over the (layer, column group) pairs; inverse rows per (row, channel) summing
// the channel's layers and writing its image once (stamps/done: completion clocks,
// may be null); the row kernels in persistent form over one class's items of all layers
// (queue: two ints, zero between launches; ncu: compute units).
hipError_t launch_sweep_fwd_rows(const float* img, const SweepLayer* sl, int nlayers,
                                 const float2* tw, const float* sx, const float* sy, int nx,
                                 int ny, int Kx, double cell, hipStream_t s);
hipError_t launch_sweep_cols(bool inverse, const SweepLayer* sl, const int2* pairs, int npairs,
                             const float2* tw, int ny, int Ky, int tsh, int tiles_x,
                             hipStream_t s);
hipError_t launch_sweep_inv_rows(const SweepLayer* sl, const int2* chan_layers, int c0,
                                 int nchan, void* out, bool real_out, const float2* tw,
                                 const float* sx,
                                 const float* sy, int nx, int ny, int Kx, double cell,
                                 unsigned long long* stamps, int* done, hipStream_t s);
hipError_t launch_rows_sweep(int mode, int cls, const WorkItem* wi, int nwi,
                             const SweepLayer* layers, wf_store store, float2* vis_base,
                             int* queue, int Kx, int Ky, int tile, int ncu, hipStream_t s);

// Kernels predicted by the residual-kernel network for a chunk of rows (null pred: every
// row exact).  pred [rows of the chunk][451]; rows whose predicted log10 error exceeds
// logtol, or whose side is out of the network's range, use the exact construction.
// Kernel-side class whose residual kernels the network predicts (sides 9..15): smaller
// kernels cost less to build exactly than one inference, wider ones exceed its window.
constexpr int NET_CLASS = 1;
// Rows per network inference of an on-the-fly apply (per-branch input/output buffers).
constexpr int64_t NET_CHUNK = 1 << 18;

struct Surrogate {
  const float* pred = nullptr;
  float logtol = -3.f;
  int* used = nullptr;          // counts rows built from the prediction (may be null)
  bool by_slot = false;         // predictions indexed by the row's slot in the launched
                                // list (else by its index minus the range start)
};

// Build kernels (FP64).  Symbolic pass over the caller-order rows listed in cs
// (predictions, when given, indexed by k - r0): bin, grid
// position, residual kernel side after thresholding, sort key.
hipError_t launch_rowsym(const double* uvw, int64_t r0, const ClassSlices& cs, double scale,
                         double gsx, double gsy, const double* mids, int P, const double* cents,
                         int Kx, int Ky, int tile, const KernelParams& kp, uint64_t* keys,
                         float* dropped, const Surrogate& sg, hipStream_t s);
// Kernel-side class (0: n_k <= 7, 1: <= 15, 2: <= 21, 3: <= 31) of rows [r0, r1) in
// caller order.  The build kernels take the rows of one class per launch.
hipError_t launch_row_class(const double* uvw, int64_t r0, int64_t r1, double scale, double gsx,
                            double gsy, const double* mids, int P, const double* cents,
                            const KernelParams& kp, uint8_t* cls, hipStream_t s);
// The rows of [lo, hi) (in the lists' order) of each class.
ClassSlices slice_classes(const RowClasses& rc, int64_t lo, int64_t hi);
// Value pass over the sorted rows listed in cs (rows of [s0, s1) by kernel-side class;
// predictions, when given, are indexed by s - s0): writes each row's T*T values at its
// value offset minus vbase, scaled by the row's data weight wts[perm[s]] (wts may be
// null: ones).
// mismatch[0] counts rows whose patch side (or class) differs from the symbolic pass, mismatch[1]
// rows with a value beyond the FP16 range (FP16 store only).
hipError_t launch_gbuild(const double* uvw, int64_t s0, const ClassSlices& cs,
                         const int32_t* perm, const uint32_t* meta, const uint32_t* voff,
                         const int32_t* row_wi, const WorkItem* wi, double scale, double gsx,
                         double gsy, const double* mids, int P, const double* cents,
                         const KernelParams& kp, void* vals, int64_t vbase, wf_store store,
                         int* mismatch, const Surrogate& sg, const float* wts, hipStream_t s);
// Factorised strategy (c).  Build: the kept residual kernel of each listed sorted row,
// times its data weight, in the value format at khat[kabs[s] ..] (n' x n', [s_v][s_u]),
// and its 2J Kaiser-Bessel taps in FP32 at taps[s 2J ..] (u then v); mismatch[0] counts
// rows whose class or patch side differs from the symbolic pass.
hipError_t launch_khat(const double* uvw, int64_t s0, const ClassSlices& cs, const int32_t* perm,
                       const uint32_t* meta, const int64_t* kabs, double scale, double gsx,
                       double gsy, const double* mids, int P, const double* cents,
                       const KernelParams& kp, void* khat, float* taps, wf_store store,
                       int* mismatch, const Surrogate& sg, const float* wts, hipStream_t s);
// Apply: the G rows of the listed sorted rows (by kept-kernel side class) from their
// kernels at khat[kof[s] ..] (khat points at the chunk's first kernel) and taps, written
// as launch_gbuild writes them; over counts values beyond the FP16 range (FP16 store only).
hipError_t launch_expand(const ExpSlices& cs, const uint32_t* meta, const uint32_t* voff,
                         const int32_t* row_wi, const WorkItem* wi, const KernelParams& kp,
                         const void* khat, const uint32_t* kof, const float* taps, void* vals,
                         int64_t vbase, wf_store store, int* over, hipStream_t s);
// Network inputs of the rows at positions [r0, r0 + nr) of list (identity when null),
// positions in caller order, or in sorted order through perm.
hipError_t launch_row_inputs(const double* uvw, const int32_t* list, const int32_t* perm,
                             int64_t r0, int64_t nr,
                             double scale, double gsx, double gsy, const double* mids, int P,
                             const double* cents, const KernelParams& kp, double L, float* x,
                             hipStream_t s);
// Training inputs and exact training targets of (w_proj, field side) examples.
hipError_t launch_train_inputs(const double* w, const double* L, const double* fu,
                               const double* fv, int64_t n, const KernelParams& kp, float* x,
                               int32_t* nk, hipStream_t s);
hipError_t launch_exact_targets(const double* w, const double* L, int64_t n,
                                const KernelParams& kp, float* t, hipStream_t s);

// Residual-kernel network kernels.
hipError_t launch_mlp_gemm(bool ta, bool tb, int epi, const float* A, int lda, const float* B,
                           int ldb, float* C, int ldc, float* Z, const float* bias, int M,
                           int N, int K, hipStream_t s);
hipError_t launch_mlp_gelu_bwd(float* dH, const float* Z, int64_t n, hipStream_t s);
hipError_t launch_mlp_colsum(const float* D, int ld, int rows, int N, float* db,
                             hipStream_t s);
hipError_t launch_mlp_loss(const float* P, const float* T, float* dP, int B, float* loss,
                           hipStream_t s);
hipError_t launch_mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                           float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_mlp_gather(const float* X, int cx, const float* T, int ct,
                             const int32_t* idx, int B, float* xb, float* tb, hipStream_t s);
hipError_t launch_mlp_prep_bf16(const float* params, uint16_t* wt, hipStream_t s);
// Copy of a network's FP32 parameters and their BF16 inference form (allocated here).
wf_status mlp_snapshot(const wf_mlp* m, DevBuf& params, DevBuf& wt, hipStream_t s);
hipError_t launch_mlp_infer_bf16(const float* x, int64_t n, const float* params,
                                 const uint16_t* wt, bool split, float* out, hipStream_t s);

// ------------------------------------------------------------------ host helpers
// Record the thread-local error message of the ABI and return the status.
wf_status fail(wf_status s, const std::string& m);
// Run an entry point's body with C++ exceptions turned into status codes, so that none
// crosses the C ABI: host allocation failures give WF_ENOMEM, anything else WF_EINVAL.
template <typename F>
wf_status guarded(F&& body) {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail(WF_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(WF_EINVAL, e.what());
  } catch (...) {
    return fail(WF_EINVAL, "unexpected exception");
  }
}
wf_status dalloc(DevBuf& b, size_t bytes);
void dfree(DevBuf& b);

#define WF_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::wf::fail(WF_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

double i0_series(double x);
double kb_phihat(double nu, int J, double beta);

struct PlanResult {
  int P = 1;
  int p_wsclean = 1;
  int p_star = 1;
  wf_strategy strategy = WF_PRECOMP_G;
  double k_est = 0, mem_model = 0, cost_model = 0;
  std::vector<double> centroids;
};

// Sect. 3.4 planner on the host (eq. 5, eq. 9 GPU form, eq. 10, Fig. 2).
int plan_channel(const double* w_all, int64_t M, const wf_image_shape& shape,
                 const wf_options& opt, uint64_t budget, PlanResult* out, std::string* err);
std::vector<double> kmeans_1d(std::vector<double> wsub, int P);
int nk_rule(double wproj, const KernelParams& kp, bool capped);

// BF16 inference of the residual-kernel network (out [n][451]); split: hi/lo operands.
wf_status mlp_infer_bf16(const wf_mlp* m, const float* x, int64_t n, bool split, float* out,
                         hipStream_t s);

// Stable LSD radix sort of (key, idx) by key bits [lo_bit, 64).
void radix_sort_pairs(std::vector<uint64_t>& key, std::vector<int32_t>& idx, int lo_bit);

}  // namespace wf
