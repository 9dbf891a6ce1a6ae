// C ABI of the widefield operator (include/wf.h): build orchestration and the apply
// sequences of Phi, Phi^dag and Phi^dag Phi (Sect. 3.2-3.6).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <stdexcept>
#include <string>
#include <vector>

#include "mlp_defs.h"
#include "wf_internal.h"

using namespace wf;

struct wf_graph {
  wf_op* op;
  int device;
  uint64_t gen;      // operator generation at capture
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace wf {

thread_local std::string g_err;

wf_status fail(wf_status s, const std::string& m) {
  g_err = m;
  return s;
}

wf_status dalloc(DevBuf& b, size_t bytes) {
  b.bytes = bytes;
  if (bytes == 0) {
    b.p = nullptr;
    return WF_OK;
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(WF_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                               hipGetErrorString(e));
  }
  return WF_OK;
}

void dfree(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

}  // namespace wf

namespace {

constexpr double C_LIGHT = 299792458.0;

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// IEEE binary16 bit pattern to float (host side, diagnostics only).
float half_bits_to_float(uint16_t h) {
  const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
  const int e = (h >> 10) & 0x1f;
  const uint32_t m = h & 0x3ffu;
  float f;
  if (e == 0) {
    f = std::ldexp((float)m, -24);
  } else if (e == 31) {
    f = m ? NAN : INFINITY;
  } else {
    f = std::ldexp((float)(m | 0x400u), e - 25);
  }
  uint32_t b;
  std::memcpy(&b, &f, 4);
  b |= sign;
  std::memcpy(&f, &b, 4);
  return f;
}

void release_branch(Branch& B, bool own_stream);
void release_sweep(wf_op* op);

void destroy_op(wf_op* op) {
  if (!op) return;
  (void)hipSetDevice(op->device);
  (void)hipDeviceSynchronize();
  for (auto& c : op->chans) {
    dfree(c.meta);
    dfree(c.voff);
    dfree(c.perm);
    dfree(c.vals);
    dfree(c.work);
    dfree(c.prune);
    dfree(c.htiles);
    dfree(c.hvals);
    dfree(c.flagged);
    dfree(c.ctab);
    for (DevBuf* b : {&c.uvw, &c.wts, &c.uperm, &c.row_wi, &c.mids, &c.cents, &c.crow,
                      &c.khat, &c.kof, &c.ktap, &c.xrow})
      dfree(*b);
  }
  dfree(op->otf_mis);
  dfree(op->net_params);
  dfree(op->net_wt);
  release_sweep(op);
  for (size_t b = 0; b < op->br.size(); ++b) release_branch(op->br[b], b > 0);
  if (op->fork) (void)hipEventDestroy(op->fork);
  dfree(op->stamps);
  dfree(op->fb_h);
  dfree(op->fb_x);
  dfree(op->fb_c);
  dfree(op->fb_red);
  dfree(op->twx);
  dfree(op->twy);
  dfree(op->sx);
  dfree(op->sy);
  for (auto& p : op->prof)
    for (auto e : p.ev) (void)hipEventDestroy(e);
  delete op;
}

struct OpGuard {
  wf_op* op;
  ~OpGuard() {
    if (op) destroy_op(op);
  }
};

std::vector<float2> twiddles(int N) {
  std::vector<float2> t(N);
  for (int m = 0; m < N; ++m) {
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)m /
                          (long double)N;
    t[m] = make_float2((float)cosl(a), (float)sinl(a));
  }
  return t;
}

// Launch-time profiling: events around each launch of one kernel class.
struct ProfScope {
  Profiler* p;
  hipStream_t s;
  hipEvent_t b = nullptr, e = nullptr;
  ProfScope(Profiler* prof, hipStream_t st) : p(prof), s(st) {
    if (!p || !p->enabled) return;
    if (p->used + 2 > p->ev.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t ev;
        if (hipEventCreate(&ev) == hipSuccess) p->ev.push_back(ev);
      }
    }
    if (p->used + 2 <= p->ev.size()) {
      b = p->ev[p->used];
      e = p->ev[p->used + 1];
      p->used += 2;
      (void)hipEventRecord(b, s);
    }
  }
  ~ProfScope() {
    if (b) (void)hipEventRecord(e, s);
  }
};

// Split the channel's row groups into work items of at most maxrows rows and 2^17
// values (so that the classes of wide patches, few rows each, still fill the device; the
// row kernels keep a wavefront's metadata for at most 128 rows in registers), then order
// them by (bin, patch class) -- one launch per class -- with the largest items of a
// launch first so that the hardware's in-order dispatch starts the longest work first.
// An item covers the rows of one patch class in one aligned block of 2^s x 2^s base
// tiles (s = ch.bin_tsh of its bin, 0 when empty); the rows of such a block are
// consecutive because the sort orders each class's tiles by interleaved index.
// trow: patch side of each sorted row; meta_base: patch words relative to each row's
// base-tile window.  Writes the words relative to the item's window (meta_out), each
// row's value offset inside its item (voff) and, if row_wi is given, its item index.  An
// on-the-fly channel (ch.gchunk set) orders by (chunk, class, size) instead and records
// each chunk's item range per class.
void split_items(ChanOp& ch, const uint8_t* trow, const uint32_t* meta_base, int64_t maxrows,
                 int tile, int halo, std::vector<WorkItem>& wis, uint32_t* voff,
                 uint32_t* meta_out, int32_t* row_wi) {
  const int64_t maxtaps = 1 << 17;
  const bool chunked = !ch.gchunk.empty();
  std::vector<WorkItem> w0;
  std::vector<int> wcls, wck;
  std::vector<int64_t> wtaps;
  int bb[4] = {255, 255, 0, 0};   // running box of the last item: u0, v0, u1, v1
  auto close_box = [&]() {
    if (w0.empty()) return;
    w0.back().box = (int32_t)((uint32_t)bb[0] | ((uint32_t)bb[1] << 8) |
                              ((uint32_t)(bb[2] - bb[0]) << 16) |
                              ((uint32_t)(bb[3] - bb[1]) << 24));
  };
  int64_t prev_block = -1;
  for (size_t gi = 0; gi < ch.groups.size(); ++gi) {
    const RowGroup& g = ch.groups[gi];
    const int sh = ch.bin_tsh.empty() ? 0 : ch.bin_tsh[g.bin];
    const int tu = (g.u0 + halo) / tile, tv = (g.v0 + halo) / tile;
    const int su = (tu >> sh) << sh, sv = (tv >> sh) << sh;
    // (bin, class, block, chunk) of this group; a new block opens a new item
    const int64_t block = ((((int64_t)g.bin * NCLS + g.cls) * 1024 + sv) * 1024 + su) * 4096 +
                          (chunked ? ch.gchunk[gi] : 0);
    const bool open = block != prev_block;
    prev_block = block;
    const uint32_t shift = (uint32_t)((tu - su) * tile) | ((uint32_t)((tv - sv) * tile) << 8);
    int64_t abs = g.voff;
    int64_t taps_in = open || w0.empty() ? 0 : wtaps.back();
    for (int64_t r = g.row0; r < (int64_t)g.row0 + g.nrows; ++r) {
      const int64_t t2 = (int64_t)trow[r] * trow[r];
      if ((open && r == g.row0) || w0.back().nrows >= maxrows || taps_in + t2 > maxtaps) {
        close_box();
        bb[0] = bb[1] = 255;
        bb[2] = bb[3] = 0;
        WorkItem wi{};
        wi.voff = abs;
        wi.row0 = (int32_t)r;
        wi.nrows = 0;
        wi.u0 = su * tile - halo;
        wi.v0 = sv * tile - halo;
        wi.bin = g.bin;
        w0.push_back(wi);
        wcls.push_back(g.cls);
        wck.push_back(chunked ? ch.gchunk[gi] : 0);
        wtaps.push_back(0);
        taps_in = 0;
      }
      {
        const uint32_t m = meta_base[r] + shift;
        meta_out[r] = m;
        const int lu0 = (int)(m & 0xff), lv0 = (int)((m >> 8) & 0xff);
        const int T = (int)((m >> 16) & 0xff);
        bb[0] = std::min(bb[0], lu0);
        bb[1] = std::min(bb[1], lv0);
        bb[2] = std::max(bb[2], lu0 + T);
        bb[3] = std::max(bb[3], lv0 + T);
      }
      voff[r] = (uint32_t)taps_in;
      if (row_wi) row_wi[r] = (int32_t)(w0.size() - 1);
      w0.back().nrows++;
      wtaps.back() += t2;
      taps_in += t2;
      abs += t2;
    }
  }
  close_box();
  std::vector<int32_t> order(w0.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    if (w0[x].bin != w0[y].bin) return w0[x].bin < w0[y].bin;
    if (wck[x] != wck[y]) return wck[x] < wck[y];   // chunks ascend with the bins
    if (wcls[x] != wcls[y]) return wcls[x] < wcls[y];
    return wtaps[x] > wtaps[y];
  });
  wis.assign(w0.size(), WorkItem{});
  std::vector<int32_t> newidx(w0.size());
  ch.bin_wi0.assign(ch.P, 0);
  ch.bin_nwi.assign(ch.P, 0);
  ch.cls_wi0.assign((size_t)ch.P * NCLS, 0);
  ch.cls_nwi.assign((size_t)ch.P * NCLS, 0);
  const size_t nck = chunked ? ch.ck_s0.size() : 0;
  ch.ck_wi0.assign(nck * NCLS, 0);
  ch.ck_nwi.assign(nck * NCLS, 0);
  for (size_t i = 0; i < order.size(); ++i) {
    const WorkItem& w = w0[order[i]];
    wis[i] = w;
    newidx[order[i]] = (int32_t)i;
    const int b = w.bin, c = wcls[order[i]];
    if (ch.bin_nwi[b] == 0) ch.bin_wi0[b] = (int32_t)i;
    ch.bin_nwi[b]++;
    if (ch.cls_nwi[b * NCLS + c] == 0) ch.cls_wi0[b * NCLS + c] = (int32_t)i;
    ch.cls_nwi[b * NCLS + c]++;   // (class ranges of a chunked bin are not contiguous)
    if (chunked) {
      const size_t k = (size_t)wck[order[i]] * NCLS + c;
      if (ch.ck_nwi[k] == 0) ch.ck_wi0[k] = (int32_t)i;
      ch.ck_nwi[k]++;
    }
  }
  if (row_wi)
    for (int64_t r = 0; r < ch.nrows; ++r) row_wi[r] = newidx[row_wi[r]];
  ch.max_rows = (int32_t)maxrows;
  ch.nwork = (int64_t)wis.size();
}

// Data weights and flags of one channel (Sect. 2): the rows that are built and the
// weight of each.
struct RowSel {
  const float* w = nullptr;          // weight per built row (null: ones)
  const int32_t* keep = nullptr;     // built row -> caller row (null: identity)
  std::vector<int32_t> flagged;      // caller rows that are discarded
  int64_t nvis = 0;                  // caller rows of the channel
};

// Stencil tiles of a holographic operator (one per active 32 x 32 grid tile and bin,
// side 2 Tmax - 1), the transient G chunk its build needs, and its device bytes.
struct HoloTiles {
  std::vector<HTile> ht;
  std::vector<int32_t> slot;      // [bin][tile] -> index among the bin's tiles, or -1
  std::vector<int64_t> t0, nt;    // per bin: first tile, tile count
  std::vector<int32_t> dmax;      // per bin: largest stencil side
  std::vector<int64_t> gtaps;     // values of each row group
  int64_t hv = 0;                 // stencil values
  int64_t cht = 0;                // values of the largest transient G chunk
  double need = 0;                // device bytes of the stencils and the chunk
};

HoloTiles holo_tiles(const ChanOp& ch, const uint8_t* trow, int64_t taps_total, int tile,
                     int halo, int Kx, int Ky, const wf_options& opt, uint64_t budget) {
  HoloTiles H;
  const int tx = Kx / tile, ty = Ky / tile;
  H.slot.assign((size_t)ch.P * tx * ty, -1);
  H.t0.assign(ch.P, 0);
  H.nt.assign(ch.P, 0);
  H.dmax.assign(ch.P, 0);
  std::vector<int> tmax((size_t)tx * ty);
  int64_t maxbin = 0;
  size_t gi = 0;
  for (int p = 0; p < ch.P; ++p) {
    std::fill(tmax.begin(), tmax.end(), 0);
    for (; gi < ch.groups.size() && ch.groups[gi].bin == p; ++gi) {
      const RowGroup& g = ch.groups[gi];
      int Tg = 0;
      for (int64_t r = g.row0; r < (int64_t)g.row0 + g.nrows; ++r) Tg = std::max<int>(Tg, trow[r]);
      const int tu = (g.u0 + halo) / tile, tv = (g.v0 + halo) / tile;
      const int dil = (halo + tile - 1) / tile;   // patches stay within the LDS window
      for (int dv = -dil; dv <= dil; ++dv)
        for (int du = -dil; du <= dil; ++du) {
          const size_t t = (size_t)(((tv + dv) % ty + ty) % ty) * tx + ((tu + du) % tx + tx) % tx;
          tmax[t] = std::max(tmax[t], Tg);
        }
    }
    H.t0[p] = (int64_t)H.ht.size();
    for (size_t t = 0; t < tmax.size(); ++t) {
      if (!tmax[t]) continue;
      HTile h;
      h.tile = (int32_t)t;
      h.D = 2 * tmax[t] - 1;
      h.voff = H.hv;
      H.slot[(size_t)p * tx * ty + t] = (int32_t)(H.ht.size() - H.t0[p]);
      H.ht.push_back(h);
      H.hv += (int64_t)h.D * h.D * tile * tile;
      H.dmax[p] = std::max(H.dmax[p], h.D);
    }
    H.nt[p] = (int64_t)H.ht.size() - H.t0[p];
    maxbin = std::max(maxbin, ch.bin_taps[p]);
  }
  // G is built for runs of whole row groups of one bin at a time, at most cht values
  H.gtaps.resize(ch.groups.size());
  int64_t maxgroup = 0;
  for (size_t i = 0; i < ch.groups.size(); ++i) {
    const int64_t end = i + 1 < ch.groups.size() ? ch.groups[i + 1].voff : taps_total;
    H.gtaps[i] = end - ch.groups[i].voff;
    maxgroup = std::max(maxgroup, H.gtaps[i]);
  }
  const int64_t cap = std::max<int64_t>(1 << 16, (int64_t)(0.1 * opt.budget_fraction *
                                                            (double)budget / 8.0));
  H.cht = std::max<int64_t>(maxgroup, std::min<int64_t>(maxbin, cap));
  const int b_v = opt.store == WF_STORE_F32 ? 8 : 4;
  H.need = (double)b_v * H.hv + (opt.store == WF_STORE_F32 ? 0.0 : 8.0 * H.hv) + 8.0 * H.cht;
  return H;
}

// Strategy (c): cut every bin into runs of whole row groups of at most ck values (the
// transient buffer of one branch: 2.5% of the budget share, so that four branches hold
// a tenth of it) and record each chunk's sorted rows and values.
void chunk_groups(ChanOp& ch, int64_t taps_total, int b_v, double share) {
  const size_t ng = ch.groups.size();
  std::vector<int64_t> gt(ng);
  int64_t maxgroup = 0;
  for (size_t i = 0; i < ng; ++i) {
    gt[i] = (i + 1 < ng ? ch.groups[i + 1].voff : taps_total) - ch.groups[i].voff;
    maxgroup = std::max(maxgroup, gt[i]);
  }
  const int64_t ck = std::max<int64_t>(maxgroup, std::max<int64_t>(1 << 16,
                                                                  (int64_t)(0.025 * share / b_v)));
  ch.gchunk.assign(ng, 0);
  ch.ck_s0.clear();
  ch.ck_s1.clear();
  ch.ck_vbase.clear();
  ch.ck_taps.clear();
  ch.ck_first.assign(ch.P, 0);
  ch.ck_count.assign(ch.P, 0);
  ch.ck_max = 0;
  for (size_t i = 0; i < ng; ++i) {
    const RowGroup& g = ch.groups[i];
    if (ch.ck_s0.empty() || ch.groups[i - 1].bin != g.bin || ch.ck_taps.back() + gt[i] > ck) {
      if (ch.ck_count[g.bin] == 0) ch.ck_first[g.bin] = (int32_t)ch.ck_s0.size();
      ch.ck_count[g.bin]++;
      ch.ck_s0.push_back(g.row0);
      ch.ck_s1.push_back(g.row0);
      ch.ck_vbase.push_back(g.voff);
      ch.ck_taps.push_back(0);
    }
    ch.gchunk[i] = (int32_t)(ch.ck_s0.size() - 1);
    ch.ck_s1.back() = (int64_t)g.row0 + g.nrows;
    ch.ck_taps.back() += gt[i];
    ch.ck_max = std::max(ch.ck_max, ch.ck_taps.back());
  }
}

wf_status build_channel(wf_op* op, int c, const double* uvw, int64_t M, double freq,
                        int64_t vis_off, uint64_t budget, const RowSel& sel, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  ChanOp& ch = op->chans[c];
  const wf_options& opt = op->opt;
  ch.freq = freq;
  ch.scale = freq / C_LIGHT;
  ch.vis_off = vis_off;
  ch.nrows = M;
  ch.nvis = sel.nvis;
  ch.nflag = (int64_t)sel.flagged.size();
  std::vector<double> w(M);
  for (int64_t k = 0; k < M; ++k) w[k] = uvw[3 * k + 2] * ch.scale;
  PlanResult pr;
  std::string perr;
  if (M > 0) {
    if (plan_channel(w.data(), M, op->shape, opt, budget, &pr, &perr) != 0)
      return fail(WF_ENOTSUP, "channel " + std::to_string(c) + ": " + perr);
  } else {
    pr.P = 1;
    pr.centroids = {0.0};
  }
  ch.P = pr.P;
  ch.centroids = pr.centroids;
  std::vector<double> mids(ch.P > 1 ? ch.P - 1 : 1, 0.0);
  for (int p = 0; p + 1 < ch.P; ++p) mids[p] = 0.5 * (ch.centroids[p] + ch.centroids[p + 1]);

  const int Kx = op->Kx, Ky = op->Ky, tile = op->tile, halo = op->halo;
  const double gsx = Kx * op->shape.cell_rad, gsy = Ky * op->shape.cell_rad;
  DevBuf duvw, dmids, dcents, dkeys, ddrop;
  struct Tmp {
    std::vector<DevBuf*> b;
    ~Tmp() {
      for (auto* x : b) dfree(*x);
    }
  } tmp{{&duvw, &dmids, &dcents, &dkeys, &ddrop}};
  wf_status st;
  if ((st = dalloc(duvw, sizeof(double) * 3 * std::max<int64_t>(M, 1))) != WF_OK) return st;
  if ((st = dalloc(dmids, sizeof(double) * mids.size())) != WF_OK) return st;
  if ((st = dalloc(dcents, sizeof(double) * ch.P)) != WF_OK) return st;
  if ((st = dalloc(dkeys, sizeof(uint64_t) * std::max<int64_t>(M, 1))) != WF_OK) return st;
  if ((st = dalloc(ddrop, sizeof(float) * std::max<int64_t>(M, 1))) != WF_OK) return st;
  WF_HIP(hipMemcpyAsync(duvw.p, uvw, sizeof(double) * 3 * M, hipMemcpyHostToDevice, s));
  DevBuf dwts;
  tmp.b.push_back(&dwts);
  if (sel.w && M > 0) {
    if ((st = dalloc(dwts, sizeof(float) * M)) != WF_OK) return st;
    WF_HIP(hipMemcpyAsync(dwts.p, sel.w, sizeof(float) * M, hipMemcpyHostToDevice, s));
  }
  if (ch.nflag > 0) {
    if ((st = dalloc(ch.flagged, sizeof(int32_t) * ch.nflag)) != WF_OK) return st;
    WF_HIP(hipMemcpyAsync(ch.flagged.p, sel.flagged.data(), sizeof(int32_t) * ch.nflag,
                          hipMemcpyHostToDevice, s));
  }
  WF_HIP(hipMemcpyAsync(dmids.p, mids.data(), sizeof(double) * mids.size(),
                        hipMemcpyHostToDevice, s));
  WF_HIP(hipMemcpyAsync(dcents.p, ch.centroids.data(), sizeof(double) * ch.P,
                        hipMemcpyHostToDevice, s));
  // residual kernels from the network where it is trusted: inputs and BF16 inference over
  // chunks of rows, once in caller order (symbolic pass) and once in sorted order (values)
  const wf_mlp* mlp = opt.surrogate;
  const float logtol = mlp ? (float)std::log10(opt.surrogate_tol) : 0.f;
  const double Lfield = op->shape.nx * op->shape.cell_rad;
  const int64_t CH = std::min<int64_t>(std::max<int64_t>(M, 1), 1 << 20);
  DevBuf dx, dpred, dused;
  tmp.b.push_back(&dx);
  tmp.b.push_back(&dpred);
  tmp.b.push_back(&dused);
  if (mlp) {
    if ((st = dalloc(dx, sizeof(float) * MLP_IN * CH)) != WF_OK) return st;
    if ((st = dalloc(dpred, sizeof(float) * MLP_OUT * CH)) != WF_OK) return st;
    if ((st = dalloc(dused, sizeof(int))) != WF_OK) return st;
    WF_HIP(hipMemsetAsync(dused.p, 0, sizeof(int), s));
  }
  // kernel-side class of every row: the build kernels take one class per launch, each
  // with an LDS scratch sized for it, from per-class row lists (caller order for the
  // symbolic pass, sorted order for the value pass)
  DevBuf dclsk, dlk, dls;
  tmp.b.push_back(&dclsk);
  tmp.b.push_back(&dlk);
  tmp.b.push_back(&dls);
  if ((st = dalloc(dclsk, std::max<int64_t>(M, 1))) != WF_OK) return st;
  if ((st = dalloc(dlk, sizeof(int32_t) * std::max<int64_t>(M, 1))) != WF_OK) return st;
  if ((st = dalloc(dls, sizeof(int32_t) * std::max<int64_t>(M, 1))) != WF_OK) return st;
  WF_HIP(launch_row_class((const double*)duvw.p, 0, M, ch.scale, gsx, gsy,
                          (const double*)dmids.p, ch.P, (const double*)dcents.p, op->kp,
                          (uint8_t*)dclsk.p, s));
  std::vector<uint8_t> clsk(M);
  WF_HIP(hipMemcpyAsync(clsk.data(), dclsk.p, M, hipMemcpyDeviceToHost, s));
  WF_HIP(hipStreamSynchronize(s));
  dfree(dclsk);
  // counting sort of rows by class; order_of(i) gives the i-th row of the order
  auto class_lists = [&](auto&& order_of, DevBuf& dl, RowClasses& rc) -> wf_status {
    int64_t cnt[4] = {0, 0, 0, 0};
    for (int64_t i = 0; i < M; ++i) ++cnt[clsk[order_of(i)]];
    rc.off[0] = 0;
    for (int c = 0; c < 4; ++c) rc.off[c + 1] = rc.off[c] + cnt[c];
    int64_t at[4] = {rc.off[0], rc.off[1], rc.off[2], rc.off[3]};
    rc.h.assign(M, 0);
    for (int64_t i = 0; i < M; ++i) rc.h[at[clsk[order_of(i)]]++] = (int32_t)i;
    rc.d = (const int32_t*)dl.p;
    WF_HIP(hipMemcpyAsync(dl.p, rc.h.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, s));
    return WF_OK;
  };
  RowClasses rck, rcs;
  if ((st = class_lists([](int64_t i) { return i; }, dlk, rck)) != WF_OK) return st;
  // Residual kernels from the network where it pays: the rows of kernel-side class 1
  // (sides 9..15).  Smaller kernels cost less to build exactly than one inference, and
  // wider ones exceed the network's window.  That class's rows are inferred in chunks of
  // its row list (predictions indexed by slot); the other classes launch once, exact.
  auto surrogate_pass = [&](const RowClasses& rc, const int32_t* order,
                            auto&& launch) -> wf_status {
    const ClassSlices all = slice_classes(rc, 0, M);
    if (!mlp) return launch(all, Surrogate{});
    ClassSlices rest = all;
    rest.n[NET_CLASS] = 0;
    wf_status e = launch(rest, Surrogate{});
    if (e != WF_OK) return e;
    for (int64_t c0 = 0; c0 < all.n[NET_CLASS]; c0 += CH) {
      const int64_t n = std::min<int64_t>(CH, all.n[NET_CLASS] - c0);
      WF_HIP(launch_row_inputs((const double*)duvw.p, rc.d, order, rc.off[NET_CLASS] + c0, n,
                               ch.scale, gsx, gsy, (const double*)dmids.p, ch.P,
                               (const double*)dcents.p, op->kp, Lfield, (float*)dx.p, s));
      if ((e = mlp_infer_bf16(mlp, (const float*)dx.p, n, true, (float*)dpred.p, s)) != WF_OK)
        return e;
      ClassSlices one{};
      one.rows[NET_CLASS] = all.rows[NET_CLASS] + c0;
      one.n[NET_CLASS] = n;
      Surrogate sg;
      sg.pred = (const float*)dpred.p;
      sg.logtol = logtol;
      sg.by_slot = true;
      sg.used = order ? nullptr : (int*)dused.p;
      if ((e = launch(one, sg)) != WF_OK) return e;
    }
    return WF_OK;
  };
  st = surrogate_pass(rck, nullptr, [&](const ClassSlices& cs, const Surrogate& sg) -> wf_status {
    WF_HIP(launch_rowsym((const double*)duvw.p, 0, cs, ch.scale, gsx, gsy,
                         (const double*)dmids.p, ch.P, (const double*)dcents.p, Kx, Ky, tile,
                         op->kp, (uint64_t*)dkeys.p, (float*)ddrop.p, sg, s));
    return WF_OK;
  });
  if (st != WF_OK) return st;
  int nused = 0;
  if (mlp) {
    WF_HIP(hipMemcpyAsync(&nused, dused.p, sizeof(int), hipMemcpyDeviceToHost, s));
  }
  std::vector<uint64_t> keys(M);
  std::vector<float> dropped(M);
  WF_HIP(hipMemcpyAsync(keys.data(), dkeys.p, sizeof(uint64_t) * M, hipMemcpyDeviceToHost, s));
  WF_HIP(hipMemcpyAsync(dropped.data(), ddrop.p, sizeof(float) * M, hipMemcpyDeviceToHost, s));
  WF_HIP(hipStreamSynchronize(s));
  dfree(dkeys);
  dfree(ddrop);
  for (int64_t k = 0; k < M; ++k)
    if (keys[k] == ~0ull) return fail(WF_EINVAL, "kernel-side class disagreement in the symbolic pass");
  int64_t ncapped = 0;
  double maxdrop = 0.0;
  for (int64_t k = 0; k < M; ++k) {
    float d = dropped[k];
    if (std::signbit(d)) {
      ++ncapped;
      d = -d;
    }
    maxdrop = std::max(maxdrop, (double)d);
  }
  std::vector<float>().swap(dropped);

  std::vector<int32_t> idx(M);
  std::iota(idx.begin(), idx.end(), 0);
  radix_sort_pairs(keys, idx, KEY_LO_BIT);

  // rows grouped in runs of one (bin, tile, patch class); the work items split the
  // groups (split_items)
  std::vector<uint32_t> meta(M), voff(M);
  std::vector<uint8_t> trow(M);
  std::vector<int32_t> row_wi(M);
  ch.bin_row0.assign(ch.P, 0);
  ch.bin_nrows.assign(ch.P, 0);
  ch.bin_taps.assign(ch.P, 0);
  ch.groups.clear();
  int64_t taps_total = 0;
  uint64_t cur = ~0ull;
  int curcls = -1;
  for (int64_t sidx = 0; sidx < M; ++sidx) {
    const uint64_t k = keys[sidx];
    const int bin = (int)(k >> 56);
    int tv, tu;
    tile_unmorton((uint32_t)((k >> 33) & 0xfffff), &tv, &tu);
    const int T = (int)((k >> 27) & 63);
    const int lv = (int)((k >> 20) & 127), lu = (int)((k >> 13) & 127);
    const uint64_t grp = k >> 33;   // bin, class, base tile
    const int cls = tap_class(T);
    if (grp != cur || cls != curcls) {
      RowGroup g{};
      g.voff = taps_total;
      g.row0 = (int32_t)sidx;
      g.nrows = 0;
      g.u0 = tu * tile - halo;
      g.v0 = tv * tile - halo;
      g.bin = bin;
      g.cls = cls;
      if (ch.groups.empty() || ch.groups.back().bin != bin) ch.bin_row0[bin] = sidx;
      ch.groups.push_back(g);
      cur = grp;
      curcls = cls;
    }
    const int off = (T - 1) / 2;
    meta[sidx] = pack_meta(lu + halo - off, lv + halo - off, T);
    trow[sidx] = (uint8_t)T;
    ch.groups.back().nrows++;
    taps_total += (int64_t)T * T;
    ch.bin_nrows[bin]++;
    ch.bin_taps[bin] += (int64_t)T * T;
  }
  // Fig. 2: (a) G when it fits; (b) H when the tree reaches it and the stencils fit;
  // else (c), G rebuilt at every apply
  const int b_v = opt.store == WF_STORE_F32 ? 8 : 4;
  const double share = opt.budget_fraction * (double)budget;
  bool holo = opt.strategy == WF_PRECOMP_H ||
              (opt.strategy == WF_AUTO && pr.strategy == WF_PRECOMP_H);
  bool otf = opt.strategy == WF_ONTHEFLY;
  if (holo && opt.strategy == WF_AUTO &&
      (tile != 32 ||
       holo_tiles(ch, trow.data(), taps_total, tile, halo, Kx, Ky, opt, budget).need > share)) {
    holo = false;
    otf = true;
  }
  if (holo && mlp)
    return fail(WF_ENOTSUP, "the holographic strategy builds exact kernels only (no kernel network)");
  ch.gchunk.clear();
  double vp_flops = 0.0;
  bool fact = false;
  int64_t khat_values = 0;
  if (otf) {
    chunk_groups(ch, taps_total, b_v, share);
    for (int64_t r = 0; r < M; ++r) {
      const int64_t np = (int64_t)trow[r] - opt.J + 1;
      khat_values += np * np;
    }
    const double meta_bytes = (24.0 + 20.0 + (sel.w ? 4.0 : 0.0) + (sel.keep ? 4.0 : 0.0)) * M;
    const double transient = 4.0 * b_v * (double)ch.ck_max;
    if (meta_bytes + transient > share)
      return fail(WF_EBUDGET, "no strategy fits the memory budget: the on-the-fly row data "
                              "alone needs " + std::to_string(meta_bytes / 1e9) + " GB");
    // factorised form: the kernels (value format), and per row a 32-bit offset, its 2J
    // taps (FP32) and its entry in the expansion's row lists
    const double khat_bytes = (double)b_v * khat_values + (8.0 + 8.0 * opt.J) * M;
    const bool fits = meta_bytes + khat_bytes + transient <= share;
    if (opt.otf_form == 2 && !fits)
      return fail(WF_EBUDGET, "the factorised on-the-fly kernels need " +
                                  std::to_string(khat_bytes / 1e9) + " GB");
    fact = opt.otf_form == 2 || (opt.otf_form == 0 && fits);
    // work of one apply's value pass.  Rebuilt: two length-nk DFT sweeps of the nk x nk
    // residual kernel (16 nk^3) and its Kaiser-Bessel convolution (4 J (n' T + T^2)), in
    // FP64; factorised: the convolution alone, in FP32
    for (const RowGroup& g : ch.groups)
      for (int64_t r = g.row0; r < (int64_t)g.row0 + g.nrows; ++r) {
        const double T = trow[r], np = T - opt.J + 1;
        const double conv = 4.0 * opt.J * (np * T + T * T);
        if (fact) {
          vp_flops += conv;
        } else {
          const int nk = nk_rule(w[idx[r]] - ch.centroids[g.bin], op->kp, true);
          vp_flops += (nk > 1 ? 16.0 * nk * nk * nk : 0.0) + conv;
        }
      }
  }
  if (otf && !fact && mlp && !op->net_otf) {
    // every apply re-infers the kernels of the network's rows: keep the parameters the
    // build used, so that the predictions (and the patch sides they decide) never change
    if ((st = mlp_snapshot(mlp, op->net_params, op->net_wt, s)) != WF_OK) return st;
    op->net_otf = true;
    op->net_logtol = logtol;
  }
  std::vector<WorkItem> wis;
  ch.max_rows = opt.max_rows_per_item > 0 ? opt.max_rows_per_item : 1024;
  ch.bin_tsh.assign(ch.P, 0);
  split_items(ch, trow.data(), meta.data(), ch.max_rows, tile, halo, wis, voff.data(),
              meta.data(), row_wi.data());

  // active uv support per bin: tiles holding rows, dilated to cover the LDS windows'
  // halo, the column strips under them and the column groups of the column passes
  {
    const int tx = Kx / tile, ty = Ky / tile;
    int tsh = 0;
    while ((1 << tsh) < tile) ++tsh;
    const int dil = (halo + tile - 1) / tile;
    const int nstrip = Kx / SW;
    const int cw = col_width_for(Ky);
    const int ngroup_all = Kx / cw;
    const size_t wt = ((size_t)tx * ty + 31) / 32, ws = ((size_t)nstrip + 31) / 32;
    std::vector<uint32_t> hbuf;
    ch.pr_strip.assign(ch.P, 0);
    ch.pr_tile.assign(ch.P, 0);
    ch.pr_groups.assign(ch.P, 0);
    ch.pr_ngroups.assign(ch.P, 0);
    ch.active_tile_frac.assign(ch.P, 0.0);
    std::vector<uint8_t> act((size_t)ch.P * tx * ty, 0), need((size_t)tx * ty);
    for (const RowGroup& g : ch.groups) {
      const int tu = (g.u0 + halo) / tile, tv = (g.v0 + halo) / tile;
      act[((size_t)g.bin * ty + tv) * tx + tu] = 1;
    }
    for (int p = 0; p < ch.P; ++p) {
      std::fill(need.begin(), need.end(), 0);
      const uint8_t* ap = act.data() + (size_t)p * tx * ty;
      for (int tv = 0; tv < ty; ++tv)
        for (int tu = 0; tu < tx; ++tu) {
          if (!ap[(size_t)tv * tx + tu]) continue;
          for (int dv = -dil; dv <= dil; ++dv)
            for (int du = -dil; du <= dil; ++du)
              need[(size_t)(((tv + dv) % ty + ty) % ty) * tx + ((tu + du) % tx + tx) % tx] = 1;
        }
      std::vector<uint32_t> tb(wt, 0), sb(ws, 0);
      int64_t nneed = 0;
      std::vector<uint8_t> colneed(tx, 0);
      for (size_t i = 0; i < need.size(); ++i)
        if (need[i]) {
          tb[i >> 5] |= 1u << (i & 31);
          colneed[i % tx] = 1;
          ++nneed;
        }
      ch.active_tile_frac[p] = (double)nneed / (double)need.size();
      for (int st2 = 0; st2 < nstrip; ++st2) {
        const int c0 = (st2 * SW) >> tsh, c1 = ((st2 + 1) * SW - 1) >> tsh;
        bool any = false;
        for (int c = c0; c <= c1; ++c) any = any || colneed[c];
        if (any) sb[st2 >> 5] |= 1u << (st2 & 31);
      }
      std::vector<uint32_t> gl;
      for (int g = 0; g < ngroup_all; ++g) {
        const int st2 = (g * cw) / SW;
        if ((sb[st2 >> 5] >> (st2 & 31)) & 1u) gl.push_back((uint32_t)g);
      }
      ch.pr_strip[p] = hbuf.size() * 4;
      hbuf.insert(hbuf.end(), sb.begin(), sb.end());
      ch.pr_tile[p] = hbuf.size() * 4;
      hbuf.insert(hbuf.end(), tb.begin(), tb.end());
      ch.pr_groups[p] = hbuf.size() * 4;
      hbuf.insert(hbuf.end(), gl.begin(), gl.end());
      ch.pr_ngroups[p] = (int32_t)gl.size();
    }
    if ((st = dalloc(ch.prune, sizeof(uint32_t) * std::max<size_t>(hbuf.size(), 1))) != WF_OK)
      return st;
    WF_HIP(hipMemcpyAsync(ch.prune.p, hbuf.data(), sizeof(uint32_t) * hbuf.size(),
                          hipMemcpyHostToDevice, s));
    WF_HIP(hipStreamSynchronize(s));
  }
  std::vector<uint64_t>().swap(keys);
  ch.ntaps = taps_total;
  ch.nwork = (int64_t)wis.size();
  DevBuf drowwi, dmis;
  tmp.b.push_back(&drowwi);
  tmp.b.push_back(&dmis);
  if ((st = dalloc(dmis, 2 * sizeof(int))) != WF_OK) return st;
  WF_HIP(hipMemsetAsync(dmis.p, 0, 2 * sizeof(int), s));
  if ((st = dalloc(ch.meta, sizeof(uint32_t) * std::max<int64_t>(M, 1))) != WF_OK) return st;
  if ((st = dalloc(ch.voff, sizeof(uint32_t) * std::max<int64_t>(M, 1))) != WF_OK) return st;
  if ((st = dalloc(ch.perm, sizeof(int32_t) * std::max<int64_t>(M, 1))) != WF_OK) return st;
  if ((st = dalloc(ch.work, sizeof(WorkItem) * std::max<size_t>(wis.size(), 1))) != WF_OK)
    return st;
  if ((st = dalloc(drowwi, sizeof(int32_t) * std::max<int64_t>(M, 1))) != WF_OK) return st;
  WF_HIP(hipMemcpyAsync(ch.meta.p, meta.data(), sizeof(uint32_t) * M, hipMemcpyHostToDevice, s));
  WF_HIP(hipMemcpyAsync(ch.voff.p, voff.data(), sizeof(uint32_t) * M, hipMemcpyHostToDevice, s));
  WF_HIP(hipMemcpyAsync(ch.perm.p, idx.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, s));
  if ((st = class_lists([&](int64_t i) { return (int64_t)idx[i]; }, dls, rcs)) != WF_OK)
    return st;
  WF_HIP(hipMemcpyAsync(drowwi.p, row_wi.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, s));
  WF_HIP(hipMemcpyAsync(ch.work.p, wis.data(), sizeof(WorkItem) * wis.size(),
                        hipMemcpyHostToDevice, s));
  if (holo) {
    // holographic matrix (Sect. 3.3): stencil tiles of every bin, accumulated from that
    // bin's rows of G built one bin at a time in FP32; G itself is not kept
    if (tile != 32) return fail(WF_EINVAL, "the holographic strategy needs tile 32");
    const int tx = Kx / tile, ty = Ky / tile;
    int tsh = 0;
    while ((1 << tsh) < tile) ++tsh;
    HoloTiles H = holo_tiles(ch, trow.data(), taps_total, tile, halo, Kx, Ky, opt, budget);
    if (H.need > share)
      return fail(WF_EBUDGET, "holographic matrix needs " + std::to_string(H.need / 1e9) +
                                  " GB");
    const std::vector<HTile>& ht = H.ht;
    const std::vector<int32_t>& slot = H.slot;
    const std::vector<int64_t>& gtaps = H.gtaps;
    ch.h_t0 = H.t0;
    ch.h_nt = H.nt;
    ch.h_dmax = H.dmax;
    const int64_t hv = H.hv, CHT = H.cht;
    ch.h_values = hv;
    DevBuf hacc, gtmp, dslot;
    tmp.b.push_back(&gtmp);
    tmp.b.push_back(&dslot);
    if ((st = dalloc(hacc, sizeof(float2) * std::max<int64_t>(hv, 1))) != WF_OK) return st;
    struct HGuard {
      DevBuf* b;
      bool keep = false;
      ~HGuard() {
        if (!keep) dfree(*b);
      }
    } hguard{&hacc};
    if ((st = dalloc(gtmp, sizeof(float2) * std::max<int64_t>(CHT, 1))) != WF_OK) return st;
    // work items in row order, so that a run of groups maps to a slice of them
    std::vector<WorkItem> wrow(wis);
    std::sort(wrow.begin(), wrow.end(),
              [](const WorkItem& a, const WorkItem& b) { return a.row0 < b.row0; });
    DevBuf dwrow;
    tmp.b.push_back(&dwrow);
    if ((st = dalloc(dwrow, sizeof(WorkItem) * std::max<size_t>(wrow.size(), 1))) != WF_OK)
      return st;
    WF_HIP(hipMemcpyAsync(dwrow.p, wrow.data(), sizeof(WorkItem) * wrow.size(),
                          hipMemcpyHostToDevice, s));
    if ((st = dalloc(dslot, sizeof(int32_t) * slot.size())) != WF_OK) return st;
    if ((st = dalloc(ch.htiles, sizeof(HTile) * std::max<size_t>(ht.size(), 1))) != WF_OK)
      return st;
    WF_HIP(hipMemsetAsync(hacc.p, 0, hacc.bytes, s));
    WF_HIP(hipMemcpyAsync(dslot.p, slot.data(), sizeof(int32_t) * slot.size(),
                          hipMemcpyHostToDevice, s));
    WF_HIP(hipMemcpyAsync(ch.htiles.p, ht.data(), sizeof(HTile) * ht.size(),
                          hipMemcpyHostToDevice, s));
    size_t wi_at = 0;
    for (size_t ga = 0; ga < ch.groups.size();) {
      const int p = ch.groups[ga].bin;
      size_t gb = ga;
      int64_t taps = 0;
      while (gb < ch.groups.size() && ch.groups[gb].bin == p && taps + gtaps[gb] <= CHT)
        taps += gtaps[gb++];
      const int64_t s0 = ch.groups[ga].row0;
      const int64_t s1 = (int64_t)ch.groups[gb - 1].row0 + ch.groups[gb - 1].nrows;
      const int64_t vbase = ch.groups[ga].voff;
      size_t wj = wi_at;
      while (wj < wrow.size() && wrow[wj].row0 < s1) ++wj;
      WF_HIP(launch_gbuild((const double*)duvw.p, s0, slice_classes(rcs, s0, s1),
                           (const int32_t*)ch.perm.p, (const uint32_t*)ch.meta.p,
                           (const uint32_t*)ch.voff.p, (const int32_t*)drowwi.p,
                           (const WorkItem*)ch.work.p, ch.scale, gsx, gsy,
                           (const double*)dmids.p, ch.P, (const double*)dcents.p, op->kp,
                           gtmp.p, vbase, WF_STORE_F32, (int*)dmis.p, Surrogate{},
                           (const float*)dwts.p, s));
      WF_HIP(launch_hbuild((const WorkItem*)dwrow.p + wi_at, (int)(wj - wi_at),
                           (const uint32_t*)ch.meta.p, (const uint32_t*)ch.voff.p,
                           (const float2*)gtmp.p, vbase,
                           (const int32_t*)dslot.p + (size_t)p * tx * ty,
                           (const HTile*)ch.htiles.p + ch.h_t0[p], tx, tsh, Kx, Ky,
                           (float*)hacc.p, s));
      wi_at = wj;
      ga = gb;
    }
    if (opt.store == WF_STORE_F32) {
      ch.hvals = hacc;
      hguard.keep = true;
    } else {
      if ((st = dalloc(ch.hvals, sizeof(uint32_t) * std::max<int64_t>(hv, 1))) != WF_OK)
        return st;
      WF_HIP(launch_hpack((const float2*)hacc.p, (uint32_t*)ch.hvals.p, hv, opt.store,
                          (int*)dmis.p + 1, s));
    }
    WF_HIP(hipStreamSynchronize(s));
    ch.holo = true;
  }
  if (otf) {
    // the value pass's inputs stay on the device; every chunk is built once into a
    // transient buffer so that patch sides and the FP16 range are checked as for (a)
    DevBuf gtmp;
    tmp.b.push_back(&gtmp);
    if ((st = dalloc(gtmp, (size_t)b_v * std::max<int64_t>(ch.ck_max, 1))) != WF_OK) return st;
    const size_t nck = ch.ck_s0.size();
    ch.ck_cls.resize(nck);
    for (size_t k = 0; k < nck; ++k) ch.ck_cls[k] = slice_classes(rcs, ch.ck_s0[k], ch.ck_s1[k]);
    if (fact) {
      // kernel offsets: absolute for the build pass, relative to the chunk's first kernel
      // (32 bits: a chunk holds fewer kernel values than G values) for the applies
      std::vector<int64_t> kabs(M);
      std::vector<uint32_t> kof(M);
      int64_t at = 0;
      for (int64_t r = 0; r < M; ++r) {
        kabs[r] = at;
        const int64_t np = (int64_t)trow[r] - opt.J + 1;
        at += np * np;
      }
      ch.ck_kbase.assign(nck, 0);
      // the expansion takes each chunk's rows by kept-kernel side class
      std::vector<int32_t> xrow;
      xrow.reserve(M);
      std::vector<int64_t> xoff((size_t)nck * NXC), xcnt((size_t)nck * NXC, 0);
      for (size_t k = 0; k < nck; ++k) {
        ch.ck_kbase[k] = ch.ck_s0[k] < M ? kabs[ch.ck_s0[k]] : at;
        for (int64_t r = ch.ck_s0[k]; r < ch.ck_s1[k]; ++r) {
          const int64_t d = kabs[r] - ch.ck_kbase[k];
          if (d > (int64_t)UINT32_MAX) return fail(WF_EINVAL, "on-the-fly chunk too large");
          kof[r] = (uint32_t)d;
        }
        for (int c = 0; c < NXC; ++c) {
          xoff[(size_t)k * NXC + c] = (int64_t)xrow.size();
          for (int64_t r = ch.ck_s0[k]; r < ch.ck_s1[k]; ++r)
            if (xclass_of((int)trow[r] - opt.J + 1) == c) xrow.push_back((int32_t)r);
          xcnt[(size_t)k * NXC + c] = (int64_t)xrow.size() - xoff[(size_t)k * NXC + c];
        }
      }
      if ((st = dalloc(ch.xrow, sizeof(int32_t) * std::max<size_t>(xrow.size(), 1))) != WF_OK)
        return st;
      WF_HIP(hipMemcpyAsync(ch.xrow.p, xrow.data(), sizeof(int32_t) * xrow.size(),
                            hipMemcpyHostToDevice, s));
      ch.ck_xcls.assign(nck, ExpSlices{});
      for (size_t k = 0; k < nck; ++k)
        for (int c = 0; c < NXC; ++c) {
          ch.ck_xcls[k].rows[c] = (const int32_t*)ch.xrow.p + xoff[(size_t)k * NXC + c];
          ch.ck_xcls[k].n[c] = xcnt[(size_t)k * NXC + c];
        }
      DevBuf dkabs;
      tmp.b.push_back(&dkabs);
      if ((st = dalloc(dkabs, sizeof(int64_t) * std::max<int64_t>(M, 1))) != WF_OK) return st;
      if ((st = dalloc(ch.kof, sizeof(uint32_t) * std::max<int64_t>(M, 1))) != WF_OK) return st;
      if ((st = dalloc(ch.khat, (size_t)b_v * std::max<int64_t>(at, 1))) != WF_OK) return st;
      if ((st = dalloc(ch.ktap, sizeof(float) * 2 * opt.J * std::max<int64_t>(M, 1))) != WF_OK)
        return st;
      WF_HIP(hipMemcpyAsync(dkabs.p, kabs.data(), sizeof(int64_t) * M, hipMemcpyHostToDevice, s));
      WF_HIP(hipMemcpyAsync(ch.kof.p, kof.data(), sizeof(uint32_t) * M, hipMemcpyHostToDevice, s));
      st = surrogate_pass(rcs, (const int32_t*)ch.perm.p,
                          [&](const ClassSlices& cs, const Surrogate& sg) -> wf_status {
                            WF_HIP(launch_khat((const double*)duvw.p, 0, cs,
                                               (const int32_t*)ch.perm.p,
                                               (const uint32_t*)ch.meta.p,
                                               (const int64_t*)dkabs.p, ch.scale, gsx, gsy,
                                               (const double*)dmids.p, ch.P,
                                               (const double*)dcents.p, op->kp, ch.khat.p,
                                               (float*)ch.ktap.p, opt.store, (int*)dmis.p, sg,
                                               (const float*)dwts.p, s));
                            return WF_OK;
                          });
      if (st != WF_OK) return st;
      // every chunk expanded once, as an apply expands it, for the FP16 range check
      for (size_t k = 0; k < nck; ++k)
        WF_HIP(launch_expand(ch.ck_xcls[k], (const uint32_t*)ch.meta.p,
                             (const uint32_t*)ch.voff.p, (const int32_t*)drowwi.p,
                             (const WorkItem*)ch.work.p, op->kp,
                             (const char*)ch.khat.p + (size_t)ch.ck_kbase[k] * b_v,
                             (const uint32_t*)ch.kof.p, (const float*)ch.ktap.p, gtmp.p,
                             ch.ck_vbase[k], opt.store, (int*)dmis.p + 1, s));
    } else {
      for (size_t k = 0; k < nck; ++k)
        WF_HIP(launch_gbuild((const double*)duvw.p, ch.ck_s0[k], ch.ck_cls[k],
                             (const int32_t*)ch.perm.p, (const uint32_t*)ch.meta.p,
                             (const uint32_t*)ch.voff.p, (const int32_t*)drowwi.p,
                             (const WorkItem*)ch.work.p, ch.scale, gsx, gsy,
                             (const double*)dmids.p, ch.P, (const double*)dcents.p, op->kp,
                             gtmp.p, ch.ck_vbase[k], opt.store, (int*)dmis.p, Surrogate{},
                             (const float*)dwts.p, s));
    }
    std::swap(ch.row_wi, drowwi);
    if (fact) {
      // the applies read kernels, taps and row words only: the coordinates, weights,
      // centroids and class lists of the build are released with it
      ch.ck_cls.clear();
    } else {
      std::swap(ch.uvw, duvw);
      std::swap(ch.mids, dmids);
      std::swap(ch.cents, dcents);
      std::swap(ch.wts, dwts);
      std::swap(ch.crow, dls);   // the chunks' class slices point into this list
    }
    ch.otf = true;
    ch.fact = fact;
  }
  if (!holo && !otf) {
  if ((st = dalloc(ch.vals, (size_t)b_v * std::max<int64_t>(taps_total, 1))) != WF_OK)
    return st;
  st = surrogate_pass(rcs, (const int32_t*)ch.perm.p,
                      [&](const ClassSlices& cs, const Surrogate& sg) -> wf_status {
                        WF_HIP(launch_gbuild((const double*)duvw.p, 0, cs,
                                             (const int32_t*)ch.perm.p,
                                             (const uint32_t*)ch.meta.p,
                                             (const uint32_t*)ch.voff.p,
                                             (const int32_t*)drowwi.p,
                                             (const WorkItem*)ch.work.p, ch.scale, gsx, gsy,
                                             (const double*)dmids.p, ch.P,
                                             (const double*)dcents.p, op->kp, ch.vals.p,
                                             0, opt.store, (int*)dmis.p, sg,
                                             (const float*)dwts.p, s));
                        return WF_OK;
                      });
  if (st != WF_OK) return st;
  }
  int mismatch[2] = {0, 0};
  WF_HIP(hipMemcpyAsync(mismatch, dmis.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  WF_HIP(hipStreamSynchronize(s));
  if (mismatch[0] != 0)
    return fail(WF_EINVAL, std::to_string(mismatch[0]) +
                               " rows changed patch side between the symbolic and value passes");
  if (mismatch[1] != 0)
    return fail(WF_EINVAL, "weighted values exceed the FP16 range: scale the weights down "
                           "or store FP32 / BF16");
  if (sel.keep && !holo) {
    if (otf && !fact) {
      // the value pass reads coordinates through the built-row permutation
      if ((st = dalloc(ch.uperm, sizeof(int32_t) * M)) != WF_OK) return st;
      WF_HIP(hipMemcpyAsync(ch.uperm.p, ch.perm.p, sizeof(int32_t) * M,
                            hipMemcpyDeviceToDevice, s));
    }
    // visibilities are read and written in caller order: sorted row -> caller row
    for (int64_t i = 0; i < M; ++i) idx[i] = sel.keep[idx[i]];
    WF_HIP(hipMemcpyAsync(ch.perm.p, idx.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, s));
    WF_HIP(hipStreamSynchronize(s));
  }

  wf_plan_info& in = ch.info;
  in.nchan = (int32_t)op->chans.size();
  in.nbins = ch.P;
  in.strategy = holo ? WF_PRECOMP_H : otf ? WF_ONTHEFLY : WF_PRECOMP_G;
  in.store = opt.store;
  in.Kx = Kx;
  in.Ky = Ky;
  in.tile = tile;
  in.p_wsclean = pr.p_wsclean;
  in.p_star = pr.p_star;
  in.nrows = M;
  in.ntaps = taps_total;
  in.nwork = ch.nwork;
  in.k_estimate = pr.k_est;
  in.mem_g_bytes = otf ? (double)(ch.uvw.bytes + ch.wts.bytes + ch.uperm.bytes +
                                   ch.row_wi.bytes + ch.crow.bytes + ch.khat.bytes +
                                   ch.kof.bytes + ch.ktap.bytes + ch.xrow.bytes) + 12.0 * M +
                             sizeof(WorkItem) * wis.size()
                      : (double)b_v * taps_total + 12.0 * M + sizeof(WorkItem) * wis.size();
  in.mem_transient_bytes = otf ? (double)b_v * ch.ck_max : 0.0;
  in.value_pass_flops = vp_flops;
  in.mem_khat_bytes = (double)(ch.khat.bytes + ch.kof.bytes + ch.ktap.bytes);
  in.otf_form = otf ? (fact ? 2 : 1) : 0;
  in.mem_model_bytes = pr.mem_model;
  in.cost_model = pr.cost_model;
  in.capped_fraction = M ? (double)ncapped / (double)M : 0.0;
  in.max_dropped_energy = maxdrop;
  in.build_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  in.max_rows_per_item = ch.max_rows;
  in.surrogate_fraction = M ? (double)nused / (double)M : 0.0;
  in.mem_h_bytes = holo ? (double)b_v * ch.h_values + (double)ch.htiles.bytes : 0.0;
  in.nflagged = ch.nflag;
  {
    // column tables of the w-layer modulations (eq. 6): the series forms of the row FFT
    // passes hold where r2 = l^2 + m^2 <= 1/100 over the image and the phase beyond the
    // quadratic term, 2 pi |w_p| |n - 1 + r2/2|, stays within 1/4 radian
    const int nx = op->shape.nx;
    const double hl = 0.5 * nx * op->shape.cell_rad, hm = 0.5 * op->shape.ny * op->shape.cell_rad;
    const double r2 = hl * hl + hm * hm;
    const double dl = std::fabs(-r2 / (1.0 + std::sqrt(1.0 - r2)) + 0.5 * r2);
    ch.cfast.assign(ch.P, 0);
    bool any = false;
    for (int p = 0; p < ch.P; ++p) {
      ch.cfast[p] = r2 <= 0.01 && 2.0 * M_PI * std::fabs(ch.centroids[p]) * dl <= 0.25;
      any = any || ch.cfast[p];
    }
    if (any) {
      if ((st = dalloc(ch.ctab, sizeof(float2) * (size_t)ch.P * nx)) != WF_OK) return st;
      for (int p = 0; p < ch.P; ++p)
        if (ch.cfast[p])
          WF_HIP(launch_chirp_table((float2*)ch.ctab.p + (size_t)p * nx, nx,
                                    op->shape.cell_rad, ch.centroids[p],
                                    (const float*)op->sx.p, s));
    }
  }
  if (holo) {
    // only the stencils serve the applies of a holographic operator
    dfree(ch.meta);
    dfree(ch.voff);
    dfree(ch.perm);
    dfree(ch.work);
  }
  return WF_OK;
}

wf_status check_op(const wf_op* op) {
  if (!op) return fail(WF_EINVAL, "null operator handle");
  return WF_OK;
}

// Pruning masks of (channel, bin); pr = null selects the full grid.
ColPrune prune_of(const wf_op* op, const ChanOp& ch, int p) {
  ColPrune pr;
  const char* b = (const char*)ch.prune.p;
  pr.strip = (const uint32_t*)(b + ch.pr_strip[p]);
  pr.tile = (const uint32_t*)(b + ch.pr_tile[p]);
  pr.groups = (const int32_t*)(b + ch.pr_groups[p]);
  pr.ngroups = ch.pr_ngroups[p];
  pr.tiles_x = op->Kx / op->tile;
  int tsh = 0;
  while ((1 << tsh) < op->tile) ++tsh;
  pr.tsh = tsh;
  return pr;
}

// Work grids and stream of one branch for the current call.
struct Lane {
  float2* X;
  float2* Y;
  float2* A;
  float* acc;
  void* gbuf;   // transient G values (on-the-fly channels)
  hipStream_t s;
  float* net_x;      // network inputs / outputs (on-the-fly channels with the network)
  float* net_pred;
};

Lane lane_of(wf_op* op, int b, hipStream_t caller) {
  Branch& B = op->br[b];
  return Lane{(float2*)B.X.p, (float2*)B.Y.p, (float2*)B.A.p, (float*)B.acc.p, B.gbuf.p,
              b == 0 ? caller : B.s, (float*)B.net_x.p, (float*)B.net_pred.p};
}

Profiler* prof_of(wf_op* op, int k) { return op->capturing ? nullptr : &op->prof[k]; }

// Column table of bin p's w-layer modulation, or null where the direct form is used.
const float2* ctab_of(const wf_op* op, const ChanOp& ch, int p) {
  if (ch.cfast.empty() || !ch.cfast[p]) return nullptr;
  return (const float2*)ch.ctab.p + (size_t)p * op->shape.nx;
}

// Side of the grid block that one work item of bin p covers.
int bin_tile(const wf_op* op, const ChanOp& ch, int p) {
  return op->tile << (ch.bin_tsh.empty() ? 0 : ch.bin_tsh[p]);
}

// One w-layer's forward half: X_p = F Z_p x (only inside the bin's support if pr).
wf_status layer_forward(wf_op* op, const Lane& L, const float* x, double wp,
                        const ColPrune* pr, const float2* ctab = nullptr) {
  const int nx = op->shape.nx, ny = op->shape.ny;
  {
    ProfScope ps(prof_of(op, 1), L.s);
    WF_HIP(launch_fwd_rows(x, L.A, (const float2*)op->twx.p, (const float*)op->sx.p,
                           (const float*)op->sy.p, nx, ny, op->Kx, op->shape.cell_rad, wp,
                           pr ? pr->strip : nullptr, ctab, L.s));
  }
  {
    ProfScope ps(prof_of(op, 2), L.s);
    WF_HIP(launch_fwd_cols(L.A, L.X, (const float2*)op->twy.p, ny, op->Kx, op->Ky, pr, L.s));
  }
  return WF_OK;
}

// One w-layer's adjoint half from the gridded Y: out (+)= Z_p^dag F^dag Y (Y is cleared
// where it was read; outside the bin's support it is zero already).
wf_status layer_adjoint(wf_op* op, const Lane& L, void* out, double wp, int mode,
                        const ColPrune* pr, const float2* ctab = nullptr) {
  const int nx = op->shape.nx, ny = op->shape.ny;
  {
    ProfScope ps(prof_of(op, 3), L.s);
    WF_HIP(launch_inv_cols(L.Y, L.A, (const float2*)op->twy.p, ny, op->Kx, op->Ky, pr, L.s));
  }
  {
    ProfScope ps(prof_of(op, 4), L.s);
    WF_HIP(launch_inv_rows(L.A, out, (const float2*)op->twx.p, (const float*)op->sx.p,
                           (const float*)op->sy.p, nx, ny, op->Kx, op->shape.cell_rad, wp,
                           mode, pr ? pr->strip : nullptr, ctab, L.s));
  }
  return WF_OK;
}

bool valid_kind(int kind) { return kind >= WF_APPLY_FORWARD && kind <= WF_APPLY_PSF_RE; }

int64_t npix_of(const wf_op* op) { return (int64_t)op->shape.nx * op->shape.ny; }

// Floats of one channel's image output of an apply (not used by the forward apply).
int64_t out_floats(const wf_op* op, int kind) {
  return npix_of(op) * (kind == WF_APPLY_PSF_RE ? 1 : 2);
}

// Channel c's part of the caller's input and output buffers.
const float* chan_in(const wf_op* op, int kind, const float* in, int c) {
  return kind == WF_APPLY_ADJOINT ? in + 2 * op->chans[c].vis_off : in + c * npix_of(op);
}
float* chan_out(const wf_op* op, int kind, float* out, int c) {
  if (kind == WF_APPLY_FORWARD) return out + 2 * op->chans[c].vis_off;
  return out + c * out_floats(op, kind);
}

// Bin p of an on-the-fly channel (strategy (c)): each chunk of the bin's rows is written
// into the lane's transient buffer (factorised: the stored kernels convolved with the
// rows' taps; rebuilt: the FP64 value pass), then applied by the same row kernels as a
// stored G (the buffer stands for the values [vbase, vbase + taps) of G).
wf_status otf_bin_apply(wf_op* op, int kind, const Lane& L, const ChanOp& ch, int p,
                        const float* in, float* out, bool first) {
  wf_status st;
  const ColPrune pr = prune_of(op, ch, p);
  const double wp = ch.centroids[p];
  const WorkItem* wk = (const WorkItem*)ch.work.p;
  const wf_store store = op->opt.store;
  const size_t b_v = store == WF_STORE_F32 ? 8 : 4;
  const double gsx = op->Kx * op->shape.cell_rad, gsy = op->Ky * op->shape.cell_rad;
  const int32_t* uperm = (const int32_t*)(ch.uperm.p ? ch.uperm.p : ch.perm.p);
  const float2* ct = ctab_of(op, ch, p);
  if (kind != WF_APPLY_ADJOINT && (st = layer_forward(op, L, in, wp, &pr, ct)) != WF_OK)
    return st;
  for (int k = ch.ck_first[p]; k < ch.ck_first[p] + ch.ck_count[p]; ++k) {
    {
      ProfScope ps(prof_of(op, 5), L.s);
      auto gbuild = [&](const ClassSlices& cs, const Surrogate& sg) -> wf_status {
        WF_HIP(launch_gbuild((const double*)ch.uvw.p, ch.ck_s0[k], cs, uperm,
                             (const uint32_t*)ch.meta.p, (const uint32_t*)ch.voff.p,
                             (const int32_t*)ch.row_wi.p, wk, ch.scale, gsx, gsy,
                             (const double*)ch.mids.p, ch.P, (const double*)ch.cents.p,
                             op->kp, L.gbuf, ch.ck_vbase[k], store, (int*)op->otf_mis.p, sg,
                             (const float*)ch.wts.p, L.s));
        return WF_OK;
      };
      if (ch.fact) {
        // factorised: the stored kernels convolved with the rows' taps
        WF_HIP(launch_expand(ch.ck_xcls[k], (const uint32_t*)ch.meta.p,
                             (const uint32_t*)ch.voff.p, (const int32_t*)ch.row_wi.p, wk, op->kp,
                             (const char*)ch.khat.p + (size_t)ch.ck_kbase[k] * b_v,
                             (const uint32_t*)ch.kof.p, (const float*)ch.ktap.p, L.gbuf,
                             ch.ck_vbase[k], store, (int*)op->otf_mis.p + 1, L.s));
      } else if (!op->net_otf) {
        if ((st = gbuild(ch.ck_cls[k], Surrogate{})) != WF_OK) return st;
      } else {
        // as at build: the network's class from its predictions, the others exact
        const ClassSlices& all = ch.ck_cls[k];
        ClassSlices rest = all;
        rest.n[NET_CLASS] = 0;
        if ((st = gbuild(rest, Surrogate{})) != WF_OK) return st;
        const double Lfield = op->shape.nx * op->shape.cell_rad;
        for (int64_t c0 = 0; c0 < all.n[NET_CLASS]; c0 += NET_CHUNK) {
          const int64_t n = std::min<int64_t>(NET_CHUNK, all.n[NET_CLASS] - c0);
          WF_HIP(launch_row_inputs((const double*)ch.uvw.p, all.rows[NET_CLASS], uperm, c0, n,
                                   ch.scale, gsx, gsy, (const double*)ch.mids.p, ch.P,
                                   (const double*)ch.cents.p, op->kp, Lfield, L.net_x, L.s));
          WF_HIP(launch_mlp_infer_bf16(L.net_x, n, (const float*)op->net_params.p,
                                       (const uint16_t*)op->net_wt.p, true, L.net_pred, L.s));
          ClassSlices one{};
          one.rows[NET_CLASS] = all.rows[NET_CLASS] + c0;
          one.n[NET_CLASS] = n;
          Surrogate sg;
          sg.pred = L.net_pred;
          sg.logtol = op->net_logtol;
          sg.by_slot = true;
          if ((st = gbuild(one, sg)) != WF_OK) return st;
        }
      }
    }
    // item value offsets are absolute: shift the base so that they land in the buffer
    const void* vals = (const char*)L.gbuf - (size_t)ch.ck_vbase[k] * b_v;
    for (int c = 0; c < NCLS; ++c) {
      const int n = ch.ck_nwi[(size_t)k * NCLS + c];
      if (n == 0) continue;
      const WorkItem* items = wk + ch.ck_wi0[(size_t)k * NCLS + c];
      if (kind == WF_APPLY_FORWARD) {
        WF_HIP(launch_degrid(c, items, n, (const uint32_t*)ch.meta.p,
                             (const uint32_t*)ch.voff.p, (const int32_t*)ch.perm.p, vals, store,
                             L.X, (float2*)out, op->Kx, op->Ky, L.s));
      } else if (kind == WF_APPLY_ADJOINT) {
        WF_HIP(launch_grid(c, items, n, (const uint32_t*)ch.meta.p, (const uint32_t*)ch.voff.p,
                           (const int32_t*)ch.perm.p, vals, store, (const float2*)in, L.Y,
                           op->Kx, op->Ky, op->tile, L.s));
      } else {
        ProfScope ps(prof_of(op, 0), L.s);
        WF_HIP(launch_gtg(c, items, n, (const uint32_t*)ch.meta.p, (const uint32_t*)ch.voff.p,
                          vals, store, L.X, L.Y, op->Kx, op->Ky, op->tile, L.s));
      }
    }
  }
  if (kind == WF_APPLY_FORWARD) return WF_OK;
  const int mode = (kind == WF_APPLY_PSF_RE ? 2 : 0) + (first ? 0 : 1);
  return layer_adjoint(op, L, out, wp, mode, &pr, ct);
}

// Bin p of one channel: that w-layer's share of the apply.  first: the layer opens the
// channel's image sum in out (overwrite) instead of adding to it.
wf_status bin_apply(wf_op* op, int kind, const Lane& L, const ChanOp& ch, int p,
                    const float* in, float* out, bool first) {
  if (ch.otf) return otf_bin_apply(op, kind, L, ch, p, in, out, first);
  wf_status st;
  const ColPrune pr = prune_of(op, ch, p);
  const double wp = ch.centroids[p];
  const WorkItem* wk = (const WorkItem*)ch.work.p;
  const float2* ct = ctab_of(op, ch, p);
  if (kind == WF_APPLY_FORWARD) {
    if ((st = layer_forward(op, L, in, wp, &pr, ct)) != WF_OK) return st;
    for (int c = 0; c < NCLS; ++c) {
      const int n = ch.cls_nwi[p * NCLS + c];
      if (n == 0) continue;
      WF_HIP(launch_degrid(c, wk + ch.cls_wi0[p * NCLS + c], n, (const uint32_t*)ch.meta.p,
                           (const uint32_t*)ch.voff.p, (const int32_t*)ch.perm.p, ch.vals.p,
                           op->opt.store, L.X, (float2*)out, op->Kx, op->Ky, L.s));
    }
    return WF_OK;
  }
  if (kind == WF_APPLY_ADJOINT) {
    for (int c = 0; c < NCLS; ++c) {
      const int n = ch.cls_nwi[p * NCLS + c];
      if (n == 0) continue;
      WF_HIP(launch_grid(c, wk + ch.cls_wi0[p * NCLS + c], n, (const uint32_t*)ch.meta.p,
                         (const uint32_t*)ch.voff.p, (const int32_t*)ch.perm.p, ch.vals.p,
                         op->opt.store, (const float2*)in, L.Y, op->Kx, op->Ky,
                         bin_tile(op, ch, p), L.s));
    }
    return layer_adjoint(op, L, out, wp, first ? 0 : 1, &pr, ct);
  }
  if ((st = layer_forward(op, L, in, wp, &pr, ct)) != WF_OK) return st;
  if (ch.holo) {
    ProfScope ps(prof_of(op, 0), L.s);
    int tsh = 0;
    while ((1 << tsh) < op->tile) ++tsh;
    WF_HIP(launch_happly((const HTile*)ch.htiles.p + ch.h_t0[p], (int)ch.h_nt[p], ch.h_dmax[p],
                         ch.hvals.p, op->opt.store, L.X, L.Y, op->Kx / op->tile, tsh, op->Kx,
                         op->Ky, L.s));
  } else {
    ProfScope ps(prof_of(op, 0), L.s);
    for (int c = 0; c < NCLS; ++c) {
      const int n = ch.cls_nwi[p * NCLS + c];
      if (n == 0) continue;
      WF_HIP(launch_gtg(c, wk + ch.cls_wi0[p * NCLS + c], n, (const uint32_t*)ch.meta.p,
                        (const uint32_t*)ch.voff.p, ch.vals.p, op->opt.store, L.X, L.Y,
                        op->Kx, op->Ky, bin_tile(op, ch, p), L.s));
    }
  }
  const int mode = (kind == WF_APPLY_PSF_RE ? 2 : 0) + (first ? 0 : 1);
  return layer_adjoint(op, L, out, wp, mode, &pr, ct);
}

// All non-empty bins of channel c on one lane, written directly to the channel's output.
wf_status run_channel(wf_op* op, int kind, int c, const Lane& L, const float* in, float* out) {
  const ChanOp& ch = op->chans[c];
  const float* ci = chan_in(op, kind, in, c);
  float* co = chan_out(op, kind, out, c);
  bool first = true;
  wf_status st;
  for (int p = 0; p < ch.P; ++p) {
    if (ch.bin_nrows[p] == 0) continue;
    if ((st = bin_apply(op, kind, L, ch, p, ci, co, first)) != WF_OK) return st;
    first = false;
  }
  if (first && kind != WF_APPLY_FORWARD)
    WF_HIP(launch_fill_zero(co, out_floats(op, kind), L.s));
  return WF_OK;
}

// ------------------------------------------------------------------ sweep (layer-batched)

void release_sweep_lanes(Sweep& W) {
  for (SweepLane& L : W.lanes) {
    for (int c = 0; c < Sweep::NLIST; ++c) dfree(L.items[c]);
    if (L.s) (void)hipStreamDestroy(L.s);
    if (L.fwd) (void)hipEventDestroy(L.fwd);
    if (L.end) (void)hipEventDestroy(L.end);
  }
  W.lanes.clear();
  dfree(W.queues);
}

void release_sweep(wf_op* op) {
  Sweep& W = op->sweep;
  release_sweep_lanes(W);
  for (DevBuf& b : W.grids) dfree(b);
  W.grids.clear();
  dfree(W.layers);
  dfree(W.pairs);
  dfree(W.chan_layers);
  dfree(W.done);
  if (W.fork) (void)hipEventDestroy(W.fork);
  W.fork = nullptr;
  W.nlayers = 0;
  W.npairs = 0;
  W.on = false;
}

bool sweep_size_ok(int K) { return K == 2048 || K == 4096 || K == 8192 || K == 16384; }

// The lanes of a sweep: nlanes contiguous channel ranges of about equal cost (stored
// values plus the FFT passes of their layers), each with its work items per (patch
// class, item tile) -- bin field = layer, largest first -- its queues, and, beyond the
// first, a stream and two events.  The caller has synchronised the device.
wf_status sweep_lanes(wf_op* op, int nlanes) {
  Sweep& W = op->sweep;
  release_sweep_lanes(W);
  wf_status st;
  const int nchan = (int)op->chans.size();
  // layer and pair ranges of every channel, and its cost
  std::vector<int> lay0(nchan + 1, 0), pair0(nchan + 1, 0);
  std::vector<double> cost(nchan, 0.0);
  {
    std::vector<int2> cl(nchan);
    WF_HIP(hipMemcpy(cl.data(), W.chan_layers.p, sizeof(int2) * nchan, hipMemcpyDeviceToHost));
    std::vector<int2> pr(W.npairs);
    if (W.npairs)
      WF_HIP(hipMemcpy(pr.data(), W.pairs.p, sizeof(int2) * W.npairs, hipMemcpyDeviceToHost));
    const double b_v = op->opt.store == WF_STORE_F32 ? 8.0 : 4.0;
    const double layer_bytes = 48.0 * (double)op->Kx * op->shape.ny;   // FFT passes, roughly
    size_t pi = 0;
    for (int c = 0; c < nchan; ++c) {
      lay0[c] = cl[c].x;
      pair0[c] = (int)pi;
      while (pi < pr.size() && pr[pi].x < cl[c].x + cl[c].y) ++pi;
      cost[c] = b_v * (double)op->chans[c].ntaps + layer_bytes * cl[c].y;
    }
    lay0[nchan] = W.nlayers;
    pair0[nchan] = W.npairs;
  }
  nlanes = std::max(1, std::min({nlanes, nchan, Sweep::MAXLANES}));
  double total = 0;
  for (double c : cost) total += c;
  std::vector<int> cut(nlanes + 1, nchan);
  cut[0] = 0;
  {
    double acc = 0;
    int k = 1;
    for (int c = 0; c < nchan && k < nlanes; ++c) {
      acc += cost[c];
      if (acc >= total * k / nlanes && c + 1 < nchan) cut[k++] = c + 1;
    }
    for (; k < nlanes; ++k) cut[k] = nchan;
  }
  W.lanes.resize(nlanes);
  for (int k = 0; k < nlanes; ++k) {
    SweepLane& L = W.lanes[k];
    L.c0 = cut[k];
    L.nc = cut[k + 1] - cut[k];
    L.l0 = lay0[L.c0];
    L.nl = lay0[L.c0 + L.nc] - L.l0;
    L.p0 = pair0[L.c0];
    L.np = pair0[L.c0 + L.nc] - L.p0;
    std::vector<WorkItem> lists[Sweep::NLIST];
    int l = L.l0;
    for (int c = L.c0; c < L.c0 + L.nc; ++c) {
      const ChanOp& ch = op->chans[c];
      if (ch.nrows == 0) continue;
      std::vector<WorkItem> wk(ch.nwork);
      WF_HIP(hipMemcpy(wk.data(), ch.work.p, sizeof(WorkItem) * wk.size(),
                       hipMemcpyDeviceToHost));
      for (int p = 0; p < ch.P; ++p) {
        if (ch.bin_nrows[p] == 0) continue;
        const int sh = ch.bin_tsh.empty() ? 0 : ch.bin_tsh[p];
        for (int kc = 0; kc < NCLS; ++kc) {
          const int n = ch.cls_nwi[p * NCLS + kc];
          for (int i = 0; i < n; ++i) {
            WorkItem w = wk[ch.cls_wi0[p * NCLS + kc] + i];
            w.bin = l;
            lists[2 * kc + sh].push_back(w);
          }
        }
        ++l;
      }
    }
    for (int j = 0; j < Sweep::NLIST; ++j) {
      std::stable_sort(lists[j].begin(), lists[j].end(),
                       [](const WorkItem& a, const WorkItem& b) { return a.nrows > b.nrows; });
      L.nitems[j] = (int)lists[j].size();
      if ((st = dalloc(L.items[j], std::max<size_t>(sizeof(WorkItem) * lists[j].size(), 16))) !=
          WF_OK)
        return st;
      if (!lists[j].empty())
        WF_HIP(hipMemcpy(L.items[j].p, lists[j].data(), sizeof(WorkItem) * lists[j].size(),
                         hipMemcpyHostToDevice));
    }
    if (k > 0) {
      WF_HIP(hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking));
      WF_HIP(hipEventCreateWithFlags(&L.end, hipEventDisableTiming));
    }
    if (k + 1 < nlanes) WF_HIP(hipEventCreateWithFlags(&L.fwd, hipEventDisableTiming));
  }
  const size_t qb = sizeof(int) * 2 * Sweep::NLIST * nlanes;
  if ((st = dalloc(W.queues, qb)) != WF_OK) return st;
  WF_HIP(hipMemset(W.queues.p, 0, qb));
  WF_HIP(hipDeviceSynchronize());
  return WF_OK;
}

// Lay out a sweep: the grids of every non-empty (channel, bin) layer, the layer table,
// the column pairs of each layer's active column groups, each channel's layer range,
// then the lanes (sweep_lanes).  The caller has synchronised the device.
wf_status sweep_build(wf_op* op, int nlanes) {
  release_sweep(op);
  Sweep& W = op->sweep;
  wf_status st;
  const int nchan = (int)op->chans.size();
  const size_t grid = sizeof(float2) * (size_t)op->Kx * op->Ky;
  const size_t arow = sizeof(float2) * (size_t)op->shape.ny * op->Kx;
  std::vector<SweepLayer> tab;
  std::vector<int2> pairs, cl(nchan, int2{0, 0});
  for (int c = 0; c < nchan; ++c) {
    const ChanOp& ch = op->chans[c];
    cl[c].x = (int)tab.size();
    if (ch.nrows == 0) continue;
    std::vector<char> pr(ch.prune.bytes);
    WF_HIP(hipMemcpy(pr.data(), ch.prune.p, pr.size(), hipMemcpyDeviceToHost));
    for (int p = 0; p < ch.P; ++p) {
      if (ch.bin_nrows[p] == 0) continue;
      const int l = (int)tab.size();
      const ColPrune cp = prune_of(op, ch, p);
      SweepLayer L{};
      DevBuf X, Y, A;
      if ((st = dalloc(X, grid)) != WF_OK) return st;
      W.grids.push_back(X);
      if ((st = dalloc(Y, grid)) != WF_OK) return st;
      W.grids.push_back(Y);
      if ((st = dalloc(A, arow)) != WF_OK) return st;
      W.grids.push_back(A);
      WF_HIP(hipMemset(Y.p, 0, grid));
      L.X = (float2*)X.p;
      L.Y = (float2*)Y.p;
      L.A = (float2*)A.p;
      L.smask = cp.strip;
      L.tile = cp.tile;
      L.vals = ch.vals.p;
      L.meta = (const uint32_t*)ch.meta.p;
      L.voff = (const uint32_t*)ch.voff.p;
      L.perm = (const int32_t*)ch.perm.p;
      L.vis_off = ch.vis_off;
      L.wp = ch.centroids[p];
      L.ctab = ctab_of(op, ch, p);
      L.chan = c;
      tab.push_back(L);
      const int32_t* grp = (const int32_t*)(pr.data() + ch.pr_groups[p]);
      for (int g = 0; g < ch.pr_ngroups[p]; ++g) pairs.push_back(int2{l, grp[g]});
    }
    cl[c].y = (int)tab.size() - cl[c].x;
  }
  W.nlayers = (int)tab.size();
  W.npairs = (int)pairs.size();
  auto upload = [&](DevBuf& b, const void* src, size_t bytes) -> wf_status {
    wf_status r = dalloc(b, std::max<size_t>(bytes, 16));
    if (r != WF_OK) return r;
    if (bytes) WF_HIP(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
    return WF_OK;
  };
  if ((st = upload(W.layers, tab.data(), sizeof(SweepLayer) * tab.size())) != WF_OK) return st;
  if ((st = upload(W.pairs, pairs.data(), sizeof(int2) * pairs.size())) != WF_OK) return st;
  if ((st = upload(W.chan_layers, cl.data(), sizeof(int2) * cl.size())) != WF_OK) return st;
  if ((st = dalloc(W.done, sizeof(int) * std::max(nchan, 1))) != WF_OK) return st;
  WF_HIP(hipMemset(W.done.p, 0, sizeof(int) * std::max(nchan, 1)));
  WF_HIP(hipEventCreateWithFlags(&W.fork, hipEventDisableTiming));
  WF_HIP(hipDeviceGetAttribute(&W.ncu, hipDeviceAttributeMultiprocessorCount, op->device));
  if ((st = sweep_lanes(op, nlanes)) != WF_OK) return st;
  W.on = true;
  return WF_OK;
}

// A whole apply as one launch per stage and lane: forward rows, forward columns, the row
// kernels per (patch class, item tile) (persistent), inverse columns, inverse rows
// summing each channel's layers.  Lane k > 0 runs on its own stream and starts when lane
// k - 1 has issued its forward passes; the caller's stream joins every lane.  No stage
// waits on the host and nothing is allocated.
wf_status run_sweep(wf_op* op, int kind, const float* in, float* out, hipStream_t s) {
  const Sweep& W = op->sweep;
  const int nchan = (int)op->chans.size();
  const int nx = op->shape.nx, ny = op->shape.ny;
  const SweepLayer* sl = (const SweepLayer*)W.layers.p;
  const int2* pairs = (const int2*)W.pairs.p;
  unsigned long long* stamps = op->stamping ? (unsigned long long*)op->stamps.p : nullptr;
  const int tsh = [&] { int t = 0; while ((1 << t) < op->tile) ++t; return t; }();
  const int tiles_x = op->Kx / op->tile;
  if (stamps) WF_HIP(launch_stamp(stamps + nchan, s));
  const bool fwd = kind != WF_APPLY_ADJOINT;
  const bool back = kind != WF_APPLY_FORWARD;
  if (kind == WF_APPLY_FORWARD)
    for (const ChanOp& ch : op->chans)
      if (ch.nflag > 0)
        WF_HIP(launch_scatter_zero((float2*)out + ch.vis_off, (const int32_t*)ch.flagged.p,
                                   ch.nflag, s));
  const int nl = (int)W.lanes.size();
  if (nl > 1) WF_HIP(hipEventRecord(W.fork, s));
  for (int k = 0; k < nl; ++k) {
    const SweepLane& L = W.lanes[k];
    const hipStream_t ls = k == 0 ? s : L.s;
    if (k > 0) {
      WF_HIP(hipStreamWaitEvent(ls, W.fork, 0));
      WF_HIP(hipStreamWaitEvent(ls, W.lanes[k - 1].fwd, 0));
    }
    if (fwd) {
      {
        ProfScope ps(prof_of(op, 1), ls);
        WF_HIP(launch_sweep_fwd_rows(in, sl + L.l0, L.nl, (const float2*)op->twx.p,
                                     (const float*)op->sx.p, (const float*)op->sy.p, nx, ny,
                                     op->Kx, op->shape.cell_rad, ls));
      }
      ProfScope ps(prof_of(op, 2), ls);
      WF_HIP(launch_sweep_cols(false, sl, pairs + L.p0, L.np, (const float2*)op->twy.p, ny,
                               op->Ky, tsh, tiles_x, ls));
    }
    if (k + 1 < nl) WF_HIP(hipEventRecord(L.fwd, ls));
    {
      const int mode = kind == WF_APPLY_FORWARD ? 1 : (kind == WF_APPLY_ADJOINT ? 2 : 0);
      float2* vis = kind == WF_APPLY_FORWARD ? (float2*)out
                    : (kind == WF_APPLY_ADJOINT ? (float2*)in : nullptr);
      int* queues = (int*)W.queues.p + 2 * Sweep::NLIST * k;
      ProfScope ps(prof_of(op, 0), ls);
      for (int j = 0; j < Sweep::NLIST; ++j)
        WF_HIP(launch_rows_sweep(mode, j / 2, (const WorkItem*)L.items[j].p, L.nitems[j], sl,
                                 op->opt.store, vis, queues + 2 * j, op->Kx, op->Ky,
                                 op->tile << (j & 1), W.ncu, ls));
    }
    if (back) {
      {
        ProfScope ps(prof_of(op, 3), ls);
        WF_HIP(launch_sweep_cols(true, sl, pairs + L.p0, L.np, (const float2*)op->twy.p, ny,
                                 op->Ky, tsh, tiles_x, ls));
      }
      ProfScope ps(prof_of(op, 4), ls);
      WF_HIP(launch_sweep_inv_rows(sl, (const int2*)W.chan_layers.p, L.c0, L.nc, out,
                                   kind == WF_APPLY_PSF_RE, (const float2*)op->twx.p,
                                   (const float*)op->sx.p, (const float*)op->sy.p, nx, ny,
                                   op->Kx, op->shape.cell_rad, stamps, (int*)W.done.p, ls));
    } else if (stamps) {
      for (int c = L.c0; c < L.c0 + L.nc; ++c) WF_HIP(launch_stamp(stamps + c, ls));
    }
    if (k > 0) WF_HIP(hipEventRecord(L.end, ls));
  }
  for (int k = 1; k < nl; ++k) WF_HIP(hipStreamWaitEvent(s, W.lanes[k].end, 0));
  return WF_OK;
}

// A whole apply: fork the branches off the caller's stream, issue every segment, join,
// add the partial sums of split channels, and stamp each channel's completion.
wf_status run_apply(wf_op* op, int kind, const float* in, float* out, hipStream_t s) {
  if (op->sweep.on) return run_sweep(op, kind, in, out, s);
  wf_status st;
  const int nchan = (int)op->chans.size();
  unsigned long long* stamps = op->stamping ? (unsigned long long*)op->stamps.p : nullptr;
  if (stamps) WF_HIP(launch_stamp(stamps + nchan, s));
  if (kind == WF_APPLY_FORWARD)
    for (const ChanOp& ch : op->chans)
      if (ch.nflag > 0)
        WF_HIP(launch_scatter_zero((float2*)out + ch.vis_off, (const int32_t*)ch.flagged.p,
                                   ch.nflag, s));
  const int nb = op->nbranch;
  if (nb > 1) {
    WF_HIP(hipEventRecord(op->fork, s));
    for (int b = 1; b < nb; ++b) WF_HIP(hipStreamWaitEvent(op->br[b].s, op->fork, 0));
  }
  std::vector<int> nseg(nchan, 0);
  for (const Segment& g : op->segs) nseg[g.chan]++;
  for (const Segment& g : op->segs) {
    const Lane L = lane_of(op, g.branch, s);
    const ChanOp& ch = op->chans[g.chan];
    const float* ci = chan_in(op, kind, in, g.chan);
    // forward: every bin writes its own rows, so all segments write in place
    float* co = (g.direct || kind == WF_APPLY_FORWARD) ? chan_out(op, kind, out, g.chan) : L.acc;
    bool first = true;
    for (int p : g.bins) {
      if ((st = bin_apply(op, kind, L, ch, p, ci, co, first)) != WF_OK) return st;
      first = false;
    }
    if (stamps && nseg[g.chan] == 1) WF_HIP(launch_stamp(stamps + g.chan, L.s));
  }
  for (int c = 0; c < nchan; ++c) {
    if (nseg[c] != 0) continue;
    if (kind != WF_APPLY_FORWARD)
      WF_HIP(launch_fill_zero(chan_out(op, kind, out, c), out_floats(op, kind), s));
    if (stamps) WF_HIP(launch_stamp(stamps + c, s));
  }
  if (nb > 1)
    for (int b = 1; b < nb; ++b) {
      WF_HIP(hipEventRecord(op->br[b].done, op->br[b].s));
      WF_HIP(hipStreamWaitEvent(s, op->br[b].done, 0));
    }
  if (kind != WF_APPLY_FORWARD)
    for (const Segment& g : op->segs)
      if (!g.direct)
        WF_HIP(launch_add_into(chan_out(op, kind, out, g.chan),
                               (const float*)op->br[g.branch].acc.p, out_floats(op, kind), s));
  if (stamps)
    for (int c = 0; c < nchan; ++c)
      if (nseg[c] > 1) WF_HIP(launch_stamp(stamps + c, s));
  return WF_OK;
}

wf_status apply_entry(wf_op* op, int kind, const float* in, float* out, void* stream) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (!in || !out) return fail(WF_EINVAL, "null pointer");
  if (kind == WF_APPLY_FORWARD || kind == WF_APPLY_ADJOINT)
    for (const auto& ch : op->chans)
      if (ch.holo)
        return fail(WF_ENOTSUP, "a holographic operator applies Phi^dag Phi only");
  WF_HIP(hipSetDevice(op->device));
  return run_apply(op, kind, in, out, (hipStream_t)stream);
}

// Rough device cost of one bin (bytes moved): stored values plus the FFT passes over
// the bin's active support.
double bin_cost(const wf_op* op, const ChanOp& ch, int p) {
  const double bv = op->opt.store == WF_STORE_F32 ? 8.0 : 4.0;
  const double grid = 8.0 * op->Kx * op->Ky;
  return bv * (double)ch.bin_taps[p] + grid * (0.5 + 3.0 * ch.active_tile_frac[p]);
}

// Place the (channel, bin) layers on branches: channels largest first onto the least
// loaded branch; a single channel splits its bins the same way.  Segments are issued
// round-robin over the branches so that every branch starts at once.
void assign_segments(wf_op* op) {
  const int nchan = (int)op->chans.size();
  const int req = std::max(1, (int)op->opt.branches);
  op->segs.clear();
  for (auto& ch : op->chans) ch.info.branch = 0;
  if (nchan == 1 && req > 1) {
    const ChanOp& ch = op->chans[0];
    std::vector<int> bins;
    for (int p = 0; p < ch.P; ++p)
      if (ch.bin_nrows[p] > 0) bins.push_back(p);
    std::stable_sort(bins.begin(), bins.end(),
                     [&](int a, int b) { return bin_cost(op, ch, a) > bin_cost(op, ch, b); });
    const int nb = std::max(1, std::min<int>(req, (int)bins.size()));
    std::vector<double> load(nb, 0.0);
    std::vector<std::vector<int>> own(nb);
    for (int p : bins) {
      const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      own[b].push_back(p);
      load[b] += bin_cost(op, ch, p);
    }
    for (int b = 0; b < nb; ++b) {
      if (own[b].empty()) continue;
      std::sort(own[b].begin(), own[b].end());
      Segment g;
      g.chan = 0;
      g.branch = b;
      g.direct = (b == 0);
      g.bins = own[b];
      op->segs.push_back(g);
    }
    op->nbranch = nb;
    return;
  }
  bool measured = true;
  std::vector<int> chans;
  for (int c = 0; c < nchan; ++c)
    if (op->chans[c].nrows > 0) {
      chans.push_back(c);
      measured = measured && op->chans[c].measured_ms > 0;
    }
  std::vector<double> cost(nchan, 0.0);
  for (int c : chans) {
    const ChanOp& ch = op->chans[c];
    if (measured) {
      cost[c] = ch.measured_ms;
    } else {
      for (int p = 0; p < ch.P; ++p)
        if (ch.bin_nrows[p] > 0) cost[c] += bin_cost(op, ch, p);
    }
  }
  std::stable_sort(chans.begin(), chans.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  const int nb = std::max(1, std::min<int>(req, (int)chans.size()));
  std::vector<double> load(nb, 0.0);
  std::vector<std::vector<int>> own(nb);
  for (int c : chans) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    own[b].push_back(c);
    load[b] += cost[c];
  }
  size_t depth = 0;
  for (auto& o : own) depth = std::max(depth, o.size());
  for (size_t k = 0; k < depth; ++k)
    for (int b = 0; b < nb; ++b) {
      if (k >= own[b].size()) continue;
      const int c = own[b][k];
      const ChanOp& ch = op->chans[c];
      Segment g;
      g.chan = c;
      g.branch = b;
      g.direct = true;
      for (int p = 0; p < ch.P; ++p)
        if (ch.bin_nrows[p] > 0) g.bins.push_back(p);
      op->segs.push_back(g);
      op->chans[c].info.branch = b;
    }
  op->nbranch = nb;
}

void release_branch(Branch& B, bool own_stream) {
  dfree(B.X);
  dfree(B.Y);
  dfree(B.A);
  dfree(B.acc);
  dfree(B.gbuf);
  dfree(B.net_x);
  dfree(B.net_pred);
  if (own_stream && B.s) (void)hipStreamDestroy(B.s);
  if (B.done) (void)hipEventDestroy(B.done);
  B.s = nullptr;
  B.done = nullptr;
}

// Allocate the grids (and streams) of branches [0, op->nbranch) and the accumulators the
// segments need; release branches beyond.  The caller has synchronised the device.
wf_status ensure_branches(wf_op* op) {
  const int nb = op->nbranch;
  const size_t grid = sizeof(float2) * (size_t)op->Kx * op->Ky;
  const size_t arow = sizeof(float2) * (size_t)op->shape.ny * op->Kx;
  for (size_t b = nb; b < op->br.size(); ++b) release_branch(op->br[b], b > 0);
  if ((int)op->br.size() > nb) op->br.resize(nb);
  if ((int)op->br.size() < nb) op->br.resize(nb);
  std::vector<bool> need_acc(nb, false);
  for (const Segment& g : op->segs)
    if (!g.direct) need_acc[g.branch] = true;
  wf_status st;
  for (int b = 0; b < nb; ++b) {
    Branch& B = op->br[b];
    if (b > 0 && !B.s) WF_HIP(hipStreamCreateWithFlags(&B.s, hipStreamNonBlocking));
    if (b > 0 && !B.done) WF_HIP(hipEventCreateWithFlags(&B.done, hipEventDisableTiming));
    if (!B.X.p) {
      if ((st = dalloc(B.X, grid)) != WF_OK) return st;
      if ((st = dalloc(B.Y, grid)) != WF_OK) return st;
      if ((st = dalloc(B.A, arow)) != WF_OK) return st;
      WF_HIP(hipMemset(B.Y.p, 0, grid));
      WF_HIP(hipMemset(B.X.p, 0, grid));
    }
    if (op->otf_bytes > B.gbuf.bytes) {
      dfree(B.gbuf);
      if ((st = dalloc(B.gbuf, op->otf_bytes)) != WF_OK) return st;
    }
    if (op->net_otf && !B.net_x.p) {
      if ((st = dalloc(B.net_x, sizeof(float) * MLP_IN * NET_CHUNK)) != WF_OK) return st;
      if ((st = dalloc(B.net_pred, sizeof(float) * MLP_OUT * NET_CHUNK)) != WF_OK) return st;
    }
    if (need_acc[b] && !B.acc.p) {
      if ((st = dalloc(B.acc, sizeof(float2) * (size_t)npix_of(op))) != WF_OK) return st;
    } else if (!need_acc[b] && B.acc.p) {
      dfree(B.acc);
    }
  }
  if (nb > 1 && !op->fork) WF_HIP(hipEventCreateWithFlags(&op->fork, hipEventDisableTiming));
  WF_HIP(hipDeviceSynchronize());
  return WF_OK;
}

wf_status set_branches(wf_op* op, int n) {
  WF_HIP(hipDeviceSynchronize());
  op->opt.branches = n;
  assign_segments(op);
  op->generation++;
  return ensure_branches(op);
}

// Patch words relative to each row's base-tile window, from words relative to the
// windows of the current items (in place).
void base_meta(const ChanOp& ch, int tile, int halo, uint32_t* meta) {
  if (ch.bin_tsh.empty()) return;
  for (const RowGroup& g : ch.groups) {
    const int sh = ch.bin_tsh[g.bin];
    if (!sh) continue;
    const int mask = (1 << sh) - 1;
    const int tu = (g.u0 + halo) / tile, tv = (g.v0 + halo) / tile;
    const uint32_t d = (uint32_t)((tu & mask) * tile) | ((uint32_t)((tv & mask) * tile) << 8);
    for (int64_t r = g.row0; r < (int64_t)g.row0 + g.nrows; ++r) meta[r] -= d;
  }
}

// Re-split channel c's stored rows into work items of at most maxrows rows, each bin's
// items covering blocks of 2^tsh[p] x 2^tsh[p] base tiles (tsh null: unchanged).  Only the
// item table, the rows' patch words and their offsets inside their items change; the
// values stay put.
wf_status retune_channel(wf_op* op, int c, int32_t maxrows, const int8_t* tsh = nullptr) {
  ChanOp& ch = op->chans[c];
  if (ch.nrows == 0 || ch.holo) return WF_OK;
  std::vector<int8_t> ntsh = ch.bin_tsh;
  if (ntsh.empty()) ntsh.assign(ch.P, 0);
  if (tsh && !ch.otf)
    for (int p = 0; p < ch.P; ++p) ntsh[p] = (int8_t)std::min<int>(tsh[p], op->max_tsh);
  const bool same_tiles = ntsh == (ch.bin_tsh.empty() ? std::vector<int8_t>(ch.P, 0)
                                                       : ch.bin_tsh);
  if (ch.max_rows == maxrows && same_tiles) return WF_OK;
  const int64_t M = ch.nrows;
  WF_HIP(hipDeviceSynchronize());
  std::vector<uint32_t> meta(M), voff(M);
  WF_HIP(hipMemcpy(meta.data(), ch.meta.p, sizeof(uint32_t) * M, hipMemcpyDeviceToHost));
  base_meta(ch, op->tile, op->halo, meta.data());
  ch.bin_tsh = ntsh;
  std::vector<uint8_t> trow(M);
  for (int64_t r = 0; r < M; ++r) trow[r] = (uint8_t)((meta[r] >> 16) & 0xff);
  std::vector<WorkItem> wis;
  std::vector<int32_t> row_wi(ch.otf ? M : 0);
  split_items(ch, trow.data(), meta.data(), maxrows, op->tile, op->halo, wis, voff.data(),
              meta.data(), ch.otf ? row_wi.data() : nullptr);
  if (ch.otf)   // the on-the-fly value pass finds each row's item through row_wi
    WF_HIP(hipMemcpy(ch.row_wi.p, row_wi.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice));
  if (ch.work.bytes < sizeof(WorkItem) * wis.size()) {
    dfree(ch.work);
    wf_status st = dalloc(ch.work, sizeof(WorkItem) * wis.size());
    if (st != WF_OK) return st;
  }
  WF_HIP(hipMemcpy(ch.meta.p, meta.data(), sizeof(uint32_t) * M, hipMemcpyHostToDevice));
  WF_HIP(hipMemcpy(ch.voff.p, voff.data(), sizeof(uint32_t) * M, hipMemcpyHostToDevice));
  WF_HIP(hipMemcpy(ch.work.p, wis.data(), sizeof(WorkItem) * wis.size(),
                   hipMemcpyHostToDevice));
  ch.info.nwork = ch.nwork;
  ch.info.max_rows_per_item = ch.max_rows;
  op->generation++;
  return WF_OK;
}

// The fused G^dag G launches of bin p alone on lane L (autotuning: X is read as it is,
// Y is added into).
wf_status bin_gtg(wf_op* op, const ChanOp& ch, int p, const Lane& L) {
  const WorkItem* wk = (const WorkItem*)ch.work.p;
  for (int c = 0; c < NCLS; ++c) {
    const int n = ch.cls_nwi[p * NCLS + c];
    if (n == 0) continue;
    WF_HIP(launch_gtg(c, wk + ch.cls_wi0[p * NCLS + c], n, (const uint32_t*)ch.meta.p,
                      (const uint32_t*)ch.voff.p, ch.vals.p, op->opt.store, L.X, L.Y,
                      op->Kx, op->Ky, bin_tile(op, ch, p), L.s));
  }
  return WF_OK;
}

// Mean duration in ms of `reps` runs of fn on stream s, after one untimed run.
template <class F>
wf_status time_runs(hipStream_t s, int reps, F&& fn, double* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  WF_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(WF_EHIP, "hipEventCreate failed");
  }
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{e0, e1};
  wf_status st = fn();
  if (st != WF_OK) return st;
  WF_HIP(hipEventRecord(e0, s));
  for (int i = 0; i < reps; ++i)
    if ((st = fn()) != WF_OK) return st;
  WF_HIP(hipEventRecord(e1, s));
  WF_HIP(hipEventSynchronize(e1));
  float t = 0;
  WF_HIP(hipEventElapsedTime(&t, e0, e1));
  *ms = (double)t / reps;
  return WF_OK;
}

}  // namespace

extern "C" {

void wf_default_options(wf_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->J = 7;
  o->beta = 2.34 * 7;
  o->oversample = 2;
  o->alpha = 2.0;
  o->smax = 31;
  o->eps_w = 1e-6;
  o->nbins = 0;
  o->strategy = WF_AUTO;
  o->store = WF_STORE_F32;
  o->plan_fraction = 0.01;
  o->budget_fraction = 0.65;
  o->seed = 0;
  o->tile = 0;
  o->max_rows_per_item = 0;
  o->branches = 0;
  o->surrogate = nullptr;
  o->surrogate_tol = 1e-3;
}

const char* wf_last_error(void) { return g_err.c_str(); }

wf_status wf_build_operator(const double* uvw_m, int64_t nrows, const int64_t* chan_rows,
                            const double* freqs_hz, int32_t nchan, wf_image_shape shape,
                            uint64_t memory_budget_bytes, const wf_options* opt_in,
                            void* hip_stream, wf_op** out) {
  try {
    g_err.clear();
    if (!out) return fail(WF_EINVAL, "out is null");
    *out = nullptr;
    if (nrows < 0 || nchan <= 0 || !freqs_hz) return fail(WF_EINVAL, "bad row/channel counts");
    if (nrows > 0 && !uvw_m) return fail(WF_EINVAL, "uvw is null");
    if (!is_pow2(shape.nx) || !is_pow2(shape.ny) || shape.nx < 8 || shape.ny < 8 ||
        shape.nx > 8192 || shape.ny > 8192)
      return fail(WF_EINVAL, "nx, ny must be powers of two in [8, 8192]");
    if (!(shape.cell_rad > 0.0) || !std::isfinite(shape.cell_rad))
      return fail(WF_EINVAL, "cell must be positive");
    wf_options opt;
    if (opt_in) opt = *opt_in;
    else wf_default_options(&opt);
    if (opt.oversample != 2) return fail(WF_EINVAL, "oversample must be 2");
    if (opt.J < 3 || opt.J > 15 || (opt.J % 2) == 0) return fail(WF_EINVAL, "J must be odd in [3,15]");
    if (opt.smax < 1 || opt.smax > 31 || (opt.smax % 2) == 0)
      return fail(WF_EINVAL, "smax must be odd in [1,31]");
    if (opt.J - 1 + opt.smax > 37)
      return fail(WF_EINVAL, "patch side J - 1 + smax must not exceed 37");
    if (opt.nbins < 0 || opt.nbins > 255) return fail(WF_EINVAL, "nbins must be in [0,255]");
    if (opt.max_rows_per_item < 0 || opt.max_rows_per_item > 1024)
      return fail(WF_EINVAL, "max_rows_per_item must be in [0,1024]");
    if (opt.branches < 0 || opt.branches > 16)
      return fail(WF_EINVAL, "branches must be in [0,16]");
    if (opt.otf_form < 0 || opt.otf_form > 2) return fail(WF_EINVAL, "otf_form must be in [0,2]");
    if (opt.surrogate && !(opt.surrogate_tol > 0))
      return fail(WF_EINVAL, "surrogate_tol must be positive");
    if (opt.surrogate && shape.nx != shape.ny)
      return fail(WF_ENOTSUP, "the kernel network is defined for square fields only");
    if (!(opt.beta > 0) || !(opt.alpha > 0) || !(opt.eps_w >= 0) || opt.eps_w >= 1)
      return fail(WF_EINVAL, "bad beta / alpha / eps_w");
    if (!(opt.plan_fraction > 0) || opt.plan_fraction > 1 || !(opt.budget_fraction > 0) ||
        opt.budget_fraction > 1)
      return fail(WF_EINVAL, "bad plan / budget fraction");
    const double Lx = shape.nx * shape.cell_rad, Ly = shape.ny * shape.cell_rad;
    if (Lx * Lx + Ly * Ly >= 1.0) return fail(WF_EINVAL, "field too wide: 2L^2 >= 1");
    int64_t total = 0;
    if (chan_rows) {
      for (int c = 0; c < nchan; ++c) {
        if (chan_rows[c] < 0) return fail(WF_EINVAL, "negative channel row count");
        total += chan_rows[c];
      }
      if (total != nrows) return fail(WF_EINVAL, "channel row counts do not sum to nrows");
    }
    for (int c = 0; c < nchan; ++c)
      if (!(freqs_hz[c] > 0) || !std::isfinite(freqs_hz[c]))
        return fail(WF_EINVAL, "frequencies must be positive");
    for (int64_t k = 0; k < 3 * nrows; ++k)
      if (!std::isfinite(uvw_m[k])) return fail(WF_EINVAL, "non-finite uvw coordinate");
    const int64_t nvis_total = chan_rows ? nrows : nrows * (int64_t)nchan;
    if (opt.weights)
      for (int64_t k = 0; k < nvis_total; ++k)
        if (!std::isfinite(opt.weights[k])) return fail(WF_EINVAL, "non-finite weight");
    const int64_t per_chan_max = chan_rows ? 0 : nrows;
    if (per_chan_max > INT32_MAX) return fail(WF_EINVAL, "too many rows per channel");
    if (chan_rows)
      for (int c = 0; c < nchan; ++c)
        if (chan_rows[c] > INT32_MAX) return fail(WF_EINVAL, "too many rows per channel");

    OpGuard guard{new wf_op()};
    wf_op* op = guard.op;
    op->opt = opt;
    op->opt.weights = nullptr;   // caller arrays, read during the build only
    op->opt.flags = nullptr;
    op->shape = shape;
    op->Kx = 2 * shape.nx;
    op->Ky = 2 * shape.ny;
    int tile = opt.tile > 0 ? opt.tile : 32;
    if (!is_pow2(tile) || tile < 8 || tile > 128)
      return fail(WF_EINVAL, "tile must be a power of two in [8,128]");
    tile = std::min({tile, op->Kx, op->Ky});
    op->tile = tile;
    op->halo = (opt.J - 1) / 2 + (opt.smax - 1) / 2;
    op->win = tile + 2 * op->halo;
    {   // items over 2 x 2 base tiles: their window and LDS accumulator must still fit
      const int w2 = 2 * tile + 2 * op->halo;
      op->max_tsh = (w2 <= 255 && 2 * tile <= 128 && (size_t)w2 * w2 * 16 <= 160 * 1024) ? 1 : 0;
    }
    if (op->win > 255 || (op->Kx / tile) > 1024 || (op->Ky / tile) > 1024)
      return fail(WF_EINVAL, "tile/halo too large");
    // an item's FP64 accumulator in LDS: (tile + largest patch side - 1)^2 cells x 16 B
    if ((size_t)op->win * op->win * 16 > 160 * 1024)
      return fail(WF_EINVAL, "tile too large for the LDS accumulator (tile + J + smax - 2 must "
                             "not exceed 101)");
    KernelParams& kp = op->kp;
    kp.Lx = Lx;
    kp.Ly = Ly;
    kp.oLx = opt.oversample * Lx;
    kp.oLy = opt.oversample * Ly;
    kp.alpha = opt.alpha;
    kp.eps = opt.eps_w;
    kp.beta = opt.beta;
    kp.i0beta = i0_series(opt.beta);
    kp.J = opt.J;
    kp.smax = opt.smax;
    kp.o = opt.oversample;
    WF_HIP(hipGetDevice(&op->device));
    hipStream_t s = (hipStream_t)hip_stream;

    const int nx = shape.nx, ny = shape.ny, Kx = op->Kx, Ky = op->Ky;
    std::vector<float> sx(nx), sy(ny);
    for (int i = 0; i < nx; ++i)
      sx[i] = (float)(1.0 / kb_phihat((double)(i - nx / 2) / Kx, opt.J, opt.beta));
    for (int j = 0; j < ny; ++j)
      sy[j] = (float)(1.0 / kb_phihat((double)(j - ny / 2) / Ky, opt.J, opt.beta));
    auto twx = twiddles(Kx), twy = twiddles(Ky);
    wf_status st;
    op->br.resize(1);
    Branch& B0 = op->br[0];
    if ((st = dalloc(B0.X, sizeof(float2) * (size_t)Kx * Ky)) != WF_OK) return st;
    if ((st = dalloc(B0.Y, sizeof(float2) * (size_t)Kx * Ky)) != WF_OK) return st;
    if ((st = dalloc(B0.A, sizeof(float2) * (size_t)ny * Kx)) != WF_OK) return st;
    if ((st = dalloc(op->twx, sizeof(float2) * Kx)) != WF_OK) return st;
    if ((st = dalloc(op->twy, sizeof(float2) * Ky)) != WF_OK) return st;
    if ((st = dalloc(op->sx, sizeof(float) * nx)) != WF_OK) return st;
    if ((st = dalloc(op->sy, sizeof(float) * ny)) != WF_OK) return st;
    WF_HIP(hipMemsetAsync(B0.Y.p, 0, B0.Y.bytes, s));
    WF_HIP(hipMemsetAsync(B0.X.p, 0, B0.X.bytes, s));
    WF_HIP(hipMemcpyAsync(op->twx.p, twx.data(), sizeof(float2) * Kx, hipMemcpyHostToDevice, s));
    WF_HIP(hipMemcpyAsync(op->twy.p, twy.data(), sizeof(float2) * Ky, hipMemcpyHostToDevice, s));
    WF_HIP(hipMemcpyAsync(op->sx.p, sx.data(), sizeof(float) * nx, hipMemcpyHostToDevice, s));
    WF_HIP(hipMemcpyAsync(op->sy.p, sy.data(), sizeof(float) * ny, hipMemcpyHostToDevice, s));

    op->chans.resize(nchan);
    int64_t off = 0;
    for (int c = 0; c < nchan; ++c) {
      const int64_t Mc = chan_rows ? chan_rows[c] : nrows;
      const double* u = chan_rows ? uvw_m + 3 * off : uvw_m;
      // flagged rows are dropped before planning; the others keep their weights
      RowSel sel;
      sel.nvis = Mc;
      sel.w = opt.weights ? opt.weights + op->total_rows : nullptr;
      std::vector<int32_t> keep;
      std::vector<double> ukeep;
      std::vector<float> wkeep;
      int64_t Mb = Mc;
      if (opt.flags) {
        const uint8_t* f = opt.flags + op->total_rows;
        for (int64_t k = 0; k < Mc; ++k) (f[k] ? sel.flagged : keep).push_back((int32_t)k);
        if (!sel.flagged.empty()) {
          Mb = (int64_t)keep.size();
          ukeep.resize(3 * Mb);
          for (int64_t i = 0; i < Mb; ++i)
            for (int d = 0; d < 3; ++d) ukeep[3 * i + d] = u[3 * (int64_t)keep[i] + d];
          if (sel.w) {
            wkeep.resize(Mb);
            for (int64_t i = 0; i < Mb; ++i) wkeep[i] = sel.w[keep[i]];
            sel.w = wkeep.data();
          }
          sel.keep = keep.data();
          u = ukeep.data();
        }
      }
      if ((st = build_channel(op, c, u, Mb, freqs_hz[c], op->total_rows, memory_budget_bytes,
                              sel, s)) != WF_OK)
        return st;
      op->total_rows += Mc;
      if (chan_rows) off += Mc;
    }
    for (auto& ch : op->chans) {
      ch.info.nchan = nchan;
      if (ch.otf)
        op->otf_bytes = std::max(op->otf_bytes, (size_t)ch.info.mem_transient_bytes);
    }
    if (op->otf_bytes > 0) {
      if ((st = dalloc(op->otf_mis, 2 * sizeof(int))) != WF_OK) return st;
      WF_HIP(hipMemsetAsync(op->otf_mis.p, 0, 2 * sizeof(int), s));
    }
    WF_HIP(hipStreamSynchronize(s));
    if ((st = set_branches(op, opt.branches > 0 ? opt.branches
                                                : (nchan > 1 ? std::min(nchan, 4) : 1))) !=
        WF_OK)
      return st;
    *out = op;
    guard.op = nullptr;
    return WF_OK;
  } catch (const std::bad_alloc&) {
    return fail(WF_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(WF_EINVAL, e.what());
  }
}

static wf_status wf_forward_body(wf_op* op, const float* d_img, float* d_vis, void* stream) {
  return apply_entry(op, WF_APPLY_FORWARD, d_img, d_vis, stream);
}

wf_status wf_forward(wf_op* op, const float* d_img, float* d_vis, void* stream) {
  return guarded([&] { return wf_forward_body(op, d_img, d_vis, stream); });
}

static wf_status wf_adjoint_body(wf_op* op, const float* d_vis, float* d_img, void* stream) {
  return apply_entry(op, WF_APPLY_ADJOINT, d_vis, d_img, stream);
}

wf_status wf_adjoint(wf_op* op, const float* d_vis, float* d_img, void* stream) {
  return guarded([&] { return wf_adjoint_body(op, d_vis, d_img, stream); });
}

static wf_status wf_psf_apply_body(wf_op* op, const float* d_img, float* d_out, void* stream) {
  return apply_entry(op, WF_APPLY_PSF, d_img, d_out, stream);
}

wf_status wf_psf_apply(wf_op* op, const float* d_img, float* d_out, void* stream) {
  return guarded([&] { return wf_psf_apply_body(op, d_img, d_out, stream); });
}

static wf_status wf_psf_apply_re_body(wf_op* op, const float* d_img, float* d_out, void* stream) {
  return apply_entry(op, WF_APPLY_PSF_RE, d_img, d_out, stream);
}

wf_status wf_psf_apply_re(wf_op* op, const float* d_img, float* d_out, void* stream) {
  return guarded([&] { return wf_psf_apply_re_body(op, d_img, d_out, stream); });
}

wf_status wf_plan(const double* uvw_m, int64_t nrows, double freq_hz, wf_image_shape shape,
                  uint64_t memory_budget_bytes, const wf_options* opt_in, wf_plan_info* out,
                  double* centroids, int32_t cap) {
  return guarded([&]() -> wf_status {
    g_err.clear();
    if (!out) return fail(WF_EINVAL, "out is null");
    if (nrows <= 0 || !uvw_m) return fail(WF_EINVAL, "need at least one row");
    if (!(freq_hz > 0) || !std::isfinite(freq_hz)) return fail(WF_EINVAL, "frequency must be positive");
    if (!is_pow2(shape.nx) || !is_pow2(shape.ny) || shape.nx < 8 || shape.ny < 8 ||
        shape.nx > 8192 || shape.ny > 8192)
      return fail(WF_EINVAL, "nx, ny must be powers of two in [8, 8192]");
    if (!(shape.cell_rad > 0.0) || !std::isfinite(shape.cell_rad))
      return fail(WF_EINVAL, "cell must be positive");
    wf_options opt;
    if (opt_in) opt = *opt_in;
    else wf_default_options(&opt);
    if (opt.oversample != 2) return fail(WF_EINVAL, "oversample must be 2");
    if (opt.J < 3 || opt.J > 15 || (opt.J % 2) == 0) return fail(WF_EINVAL, "J must be odd in [3,15]");
    if (opt.smax < 1 || opt.smax > 31 || (opt.smax % 2) == 0)
      return fail(WF_EINVAL, "smax must be odd in [1,31]");
    if (opt.nbins < 0 || opt.nbins > 255) return fail(WF_EINVAL, "nbins must be in [0,255]");
    if (!(opt.alpha > 0) || !(opt.plan_fraction > 0) || opt.plan_fraction > 1 ||
        !(opt.budget_fraction > 0) || opt.budget_fraction > 1)
      return fail(WF_EINVAL, "bad alpha / plan / budget fraction");
    const double Lx = shape.nx * shape.cell_rad, Ly = shape.ny * shape.cell_rad;
    if (Lx * Lx + Ly * Ly >= 1.0) return fail(WF_EINVAL, "field too wide: 2L^2 >= 1");
    for (int64_t k = 0; k < 3 * nrows; ++k)
      if (!std::isfinite(uvw_m[k])) return fail(WF_EINVAL, "non-finite uvw coordinate");
    const double scale = freq_hz / C_LIGHT;
    std::vector<double> w(nrows);
    for (int64_t k = 0; k < nrows; ++k) w[k] = uvw_m[3 * k + 2] * scale;
    PlanResult pr;
    std::string perr;
    if (plan_channel(w.data(), nrows, shape, opt, memory_budget_bytes, &pr, &perr) != 0)
      return fail(WF_ENOTSUP, perr);
    if (centroids && cap < (int32_t)pr.centroids.size())
      return fail(WF_EINVAL, "centroid capacity too small");
    wf_plan_info in{};
    in.nchan = 1;
    in.nbins = pr.P;
    in.strategy = pr.strategy;
    in.store = opt.store;
    in.Kx = 2 * shape.nx;
    in.Ky = 2 * shape.ny;
    in.p_wsclean = pr.p_wsclean;
    in.p_star = pr.p_star;
    in.nrows = nrows;
    in.k_estimate = pr.k_est;
    in.mem_model_bytes = pr.mem_model;
    in.cost_model = pr.cost_model;
    *out = in;
    if (centroids) std::copy(pr.centroids.begin(), pr.centroids.end(), centroids);
    return WF_OK;
  });
}

wf_status wf_get_plan(const wf_op* op, int32_t chan, wf_plan_info* out) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (!out || chan < 0 || chan >= (int)op->chans.size()) return fail(WF_EINVAL, "bad channel");
  *out = op->chans[chan].info;
  return WF_OK;
}

wf_status wf_get_centroids(const wf_op* op, int32_t chan, double* out, int32_t cap) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (!out || chan < 0 || chan >= (int)op->chans.size()) return fail(WF_EINVAL, "bad channel");
  const auto& c = op->chans[chan].centroids;
  if (cap < (int)c.size()) return fail(WF_EINVAL, "capacity too small");
  std::copy(c.begin(), c.end(), out);
  return WF_OK;
}

wf_status wf_get_bin_rows(const wf_op* op, int32_t chan, int64_t* out, int32_t cap) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (!out || chan < 0 || chan >= (int)op->chans.size()) return fail(WF_EINVAL, "bad channel");
  const auto& c = op->chans[chan].bin_nrows;
  if (cap < (int)c.size()) return fail(WF_EINVAL, "capacity too small");
  std::copy(c.begin(), c.end(), out);
  return WF_OK;
}

wf_status wf_get_row(const wf_op* op, int32_t chan, int64_t row, int32_t* T, int32_t* qu0,
                     int32_t* qv0, int32_t* bin, float* vals, int32_t cap) {
  try {
    wf_status st = check_op(op);
    if (st != WF_OK) return st;
    if (chan < 0 || chan >= (int)op->chans.size()) return fail(WF_EINVAL, "bad channel");
    const ChanOp& ch = op->chans[chan];
    if (row < 0 || row >= ch.nvis) return fail(WF_EINVAL, "row out of range");
    if (ch.holo) return fail(WF_ENOTSUP, "a holographic operator keeps no rows of G");
    if (ch.otf) return fail(WF_ENOTSUP, "an on-the-fly operator keeps no rows of G");
    WF_HIP(hipSetDevice(op->device));
    WF_HIP(hipDeviceSynchronize());
    // host index of the stored rows, built on first use (and after a re-split)
    DebugIndex& dx = ch.dbg;
    if (dx.gen != op->generation + 1) {
      std::vector<int32_t> perm(ch.nrows);
      WF_HIP(hipMemcpy(perm.data(), ch.perm.p, sizeof(int32_t) * ch.nrows,
                       hipMemcpyDeviceToHost));
      dx.sorted_of.assign(ch.nvis, -1);
      for (int64_t i = 0; i < ch.nrows; ++i) dx.sorted_of[perm[i]] = (int32_t)i;
      dx.items.resize(ch.nwork);
      WF_HIP(hipMemcpy(dx.items.data(), ch.work.p, sizeof(WorkItem) * ch.nwork,
                       hipMemcpyDeviceToHost));
      dx.item_of.assign(ch.nrows, 0);
      for (int64_t i = 0; i < ch.nwork; ++i)
        for (int32_t r = 0; r < dx.items[i].nrows; ++r)
          dx.item_of[dx.items[i].row0 + r] = (int32_t)i;
      dx.gen = op->generation + 1;
    }
    const int64_t s = dx.sorted_of[row];
    if (s < 0) return fail(WF_EINVAL, "row is flagged (not built)");
    uint32_t m, vo;
    WF_HIP(hipMemcpy(&m, (const uint32_t*)ch.meta.p + s, 4, hipMemcpyDeviceToHost));
    WF_HIP(hipMemcpy(&vo, (const uint32_t*)ch.voff.p + s, 4, hipMemcpyDeviceToHost));
    const std::vector<WorkItem>& wis = dx.items;
    const int64_t w = dx.item_of[s];
    const int t = (m >> 16) & 0xff, lu0 = m & 0xff, lv0 = (m >> 8) & 0xff;
    if (T) *T = t;
    if (qu0) *qu0 = (wis[w].u0 + lu0) & (op->Kx - 1);
    if (qv0) *qv0 = (wis[w].v0 + lv0) & (op->Ky - 1);
    if (bin) *bin = wis[w].bin;
    if (vals) {
      if (cap < t * t) return fail(WF_EINVAL, "capacity too small");
      const int64_t vb = wis[w].voff + vo;
      if (op->opt.store == WF_STORE_F32) {
        WF_HIP(hipMemcpy(vals, (const float2*)ch.vals.p + vb, 8 * t * t, hipMemcpyDeviceToHost));
      } else {
        std::vector<uint16_t> h(2 * t * t);
        WF_HIP(hipMemcpy(h.data(), (const uint32_t*)ch.vals.p + vb, 4 * t * t,
                         hipMemcpyDeviceToHost));
        for (int i = 0; i < 2 * t * t; ++i) {
          if (op->opt.store == WF_STORE_BF16) {
            uint32_t b = (uint32_t)h[i] << 16;
            std::memcpy(&vals[i], &b, 4);
          } else {
            vals[i] = half_bits_to_float(h[i]);
          }
        }
      }
    }
    return WF_OK;
  } catch (const std::exception& e) {
    return fail(WF_ENOMEM, e.what());
  }
}

static wf_status wf_layer_grid_body(wf_op* op, int32_t chan, int32_t bin, const float* d_img,
                                    float* d_grid, void* stream) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (chan < 0 || chan >= (int)op->chans.size()) return fail(WF_EINVAL, "bad channel");
  const ChanOp& ch = op->chans[chan];
  if (bin < 0 || bin >= ch.P || !d_img || !d_grid) return fail(WF_EINVAL, "bad bin/pointer");
  WF_HIP(hipSetDevice(op->device));
  hipStream_t s = (hipStream_t)stream;
  const int64_t npix = (int64_t)op->shape.nx * op->shape.ny;
  const Lane L = lane_of(op, 0, s);
  if ((st = layer_forward(op, L, d_img + chan * npix, ch.centroids[bin], nullptr)) != WF_OK)
    return st;
  WF_HIP(launch_strip_to_rowmajor(L.X, (float2*)d_grid, op->Ky, op->Kx, s));
  return WF_OK;
}

wf_status wf_layer_grid(wf_op* op, int32_t chan, int32_t bin, const float* d_img, float* d_grid,
                        void* stream) {
  return guarded([&] { return wf_layer_grid_body(op, chan, bin, d_img, d_grid, stream); });
}

static wf_status wf_profile_enable_body(wf_op* op, int32_t kernel_id, int32_t enable) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (kernel_id < 0 || kernel_id >= NPROF) return fail(WF_EINVAL, "bad kernel id");
  Profiler& p = op->prof[kernel_id];
  p.enabled = enable != 0;
  p.used = 0;
  p.launches = 0;
  p.total_ms = 0;
  return WF_OK;
}

wf_status wf_profile_enable(wf_op* op, int32_t kernel_id, int32_t enable) {
  return guarded([&] { return wf_profile_enable_body(op, kernel_id, enable); });
}

static wf_status wf_profile_read_body(wf_op* op, int32_t kernel_id, int64_t* launches,
                                      double* total_ms) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (kernel_id < 0 || kernel_id >= NPROF) return fail(WF_EINVAL, "bad kernel id");
  Profiler& p = op->prof[kernel_id];
  WF_HIP(hipSetDevice(op->device));
  for (size_t i = 0; i + 1 < p.used; i += 2) {
    WF_HIP(hipEventSynchronize(p.ev[i + 1]));
    float ms = 0;
    WF_HIP(hipEventElapsedTime(&ms, p.ev[i], p.ev[i + 1]));
    p.total_ms += ms;
    p.launches++;
  }
  p.used = 0;
  if (launches) *launches = p.launches;
  if (total_ms) *total_ms = p.total_ms;
  return WF_OK;
}

wf_status wf_profile_read(wf_op* op, int32_t kernel_id, int64_t* launches, double* total_ms) {
  return guarded([&] { return wf_profile_read_body(op, kernel_id, launches, total_ms); });
}

static wf_status wf_set_sweep_body(wf_op* op, int32_t enable) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  WF_HIP(hipSetDevice(op->device));
  WF_HIP(hipDeviceSynchronize());
  if (!enable) {
    release_sweep(op);
    op->generation++;
    return WF_OK;
  }
  if (op->Kx != 2 * op->shape.nx || op->Ky != 2 * op->shape.ny || !sweep_size_ok(op->Kx) ||
      !sweep_size_ok(op->Ky))
    return fail(WF_ENOTSUP, "the sweep needs grid sides of 2048 .. 16384");
  for (const ChanOp& ch : op->chans)
    if (ch.otf || ch.holo)
      return fail(WF_ENOTSUP, "the sweep needs every channel to store G (strategy (a))");
  if (enable < 0) return fail(WF_EINVAL, "enable must be 0 (off) or a lane count >= 1");
  st = sweep_build(op, std::min<int>(enable, Sweep::MAXLANES));
  op->generation++;
  if (st != WF_OK) {
    release_sweep(op);
    return st;
  }
  return WF_OK;
}

wf_status wf_set_sweep(wf_op* op, int32_t enable) {
  return guarded([&] { return wf_set_sweep_body(op, enable); });
}

static wf_status wf_set_branches_body(wf_op* op, int32_t branches) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (branches < 1 || branches > 16) return fail(WF_EINVAL, "branches must be in [1,16]");
  WF_HIP(hipSetDevice(op->device));
  return set_branches(op, branches);
}

wf_status wf_set_branches(wf_op* op, int32_t branches) {
  return guarded([&] { return wf_set_branches_body(op, branches); });
}

static wf_status wf_graph_capture_body(wf_op* op, wf_apply_kind kind, const float* d_in,
                                       float* d_out, void* hip_stream, wf_graph** out) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (!out) return fail(WF_EINVAL, "out is null");
  *out = nullptr;
  if (!valid_kind(kind)) return fail(WF_EINVAL, "bad apply kind");
  if (!d_in || !d_out) return fail(WF_EINVAL, "null pointer");
  if (!hip_stream) return fail(WF_EINVAL, "graph capture needs a created (non-NULL) stream");
  WF_HIP(hipSetDevice(op->device));
  hipStream_t s = (hipStream_t)hip_stream;
  WF_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  op->capturing = true;
  st = run_apply(op, kind, d_in, d_out, s);
  op->capturing = false;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (st != WF_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return fail(WF_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  hipGraphExec_t x = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(WF_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
  }
  wf_graph* r = new (std::nothrow) wf_graph{op, op->device, op->generation, g, x};
  if (!r) {
    (void)hipGraphExecDestroy(x);
    (void)hipGraphDestroy(g);
    return fail(WF_ENOMEM, "host allocation failed");
  }
  *out = r;
  return WF_OK;
}

wf_status wf_graph_capture(wf_op* op, wf_apply_kind kind, const float* d_in, float* d_out,
                           void* hip_stream, wf_graph** out) {
  return guarded([&] { return wf_graph_capture_body(op, kind, d_in, d_out, hip_stream, out); });
}

static wf_status wf_graph_launch_body(wf_graph* g, void* hip_stream) {
  if (!g || !g->op) return fail(WF_EINVAL, "null graph");
  if (g->gen != g->op->generation)
    return fail(WF_EINVAL, "the operator's work items or branches changed since the capture");
  WF_HIP(hipSetDevice(g->op->device));
  WF_HIP(hipGraphLaunch(g->exec, (hipStream_t)hip_stream));
  return WF_OK;
}

wf_status wf_graph_launch(wf_graph* g, void* hip_stream) {
  return guarded([&] { return wf_graph_launch_body(g, hip_stream); });
}

static wf_status wf_graph_destroy_body(wf_graph* g) {
  if (!g) return fail(WF_EINVAL, "null graph");
  (void)hipSetDevice(g->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return WF_OK;
}

static wf_status wf_graph_nodes_body(const wf_graph* g, int64_t* kernels, int64_t* total) {
  if (!g || !g->graph) return fail(WF_EINVAL, "null graph");
  if (!kernels || !total) return fail(WF_EINVAL, "null output");
  size_t n = 0;
  WF_HIP(hipGraphGetNodes(g->graph, nullptr, &n));
  std::vector<hipGraphNode_t> nodes(n);
  if (n > 0) WF_HIP(hipGraphGetNodes(g->graph, nodes.data(), &n));
  int64_t k = 0;
  for (size_t i = 0; i < n; ++i) {
    hipGraphNodeType t;
    WF_HIP(hipGraphNodeGetType(nodes[i], &t));
    if (t == hipGraphNodeTypeKernel) ++k;
  }
  *kernels = k;
  *total = (int64_t)n;
  return WF_OK;
}

wf_status wf_graph_nodes(const wf_graph* g, int64_t* kernels, int64_t* total) {
  return guarded([&] { return wf_graph_nodes_body(g, kernels, total); });
}

wf_status wf_graph_destroy(wf_graph* g) {
  return guarded([&] { return wf_graph_destroy_body(g); });
}

static wf_status wf_latency_enable_body(wf_op* op, int32_t enable) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  WF_HIP(hipSetDevice(op->device));
  if (enable && !op->stamps.p) {
    const size_t bytes = sizeof(unsigned long long) * (op->chans.size() + 1);
    if ((st = dalloc(op->stamps, bytes)) != WF_OK) return st;
    WF_HIP(hipMemset(op->stamps.p, 0, bytes));
    WF_HIP(hipDeviceSynchronize());
  }
  // the stamp buffer stays allocated: graphs captured while enabled keep writing it
  op->stamping = enable != 0;
  return WF_OK;
}

wf_status wf_latency_enable(wf_op* op, int32_t enable) {
  return guarded([&] { return wf_latency_enable_body(op, enable); });
}

wf_status wf_read_latency(wf_op* op, double* ms, int32_t cap) {
  try {
    wf_status st = check_op(op);
    if (st != WF_OK) return st;
    const int nchan = (int)op->chans.size();
    if (!ms || cap < nchan) return fail(WF_EINVAL, "capacity too small");
    if (!op->stamps.p) return fail(WF_EINVAL, "latency stamps are not enabled");
    WF_HIP(hipSetDevice(op->device));
    WF_HIP(hipDeviceSynchronize());
    std::vector<unsigned long long> t(nchan + 1);
    WF_HIP(hipMemcpy(t.data(), op->stamps.p, sizeof(unsigned long long) * (nchan + 1),
                     hipMemcpyDeviceToHost));
    int khz = 0;
    WF_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, op->device));
    if (khz <= 0) return fail(WF_EHIP, "device wall-clock rate unavailable");
    for (int c = 0; c < nchan; ++c)
      ms[c] = (double)((long long)(t[c] - t[nchan])) / (double)khz;
    return WF_OK;
  } catch (const std::exception& e) {
    return fail(WF_ENOMEM, e.what());
  }
}

wf_status wf_get_bin_tiles(const wf_op* op, int32_t chan, int32_t* tiles, int32_t cap) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (chan < 0 || chan >= (int)op->chans.size()) return fail(WF_EINVAL, "bad channel");
  const ChanOp& ch = op->chans[chan];
  if (!tiles || cap < ch.P) return fail(WF_EINVAL, "capacity too small");
  for (int p = 0; p < ch.P; ++p) tiles[p] = bin_tile(op, ch, p);
  return WF_OK;
}

static wf_status wf_set_bin_tiles_body(wf_op* op, int32_t chan, const int32_t* tiles,
                                       int32_t n) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (chan < 0 || chan >= (int)op->chans.size()) return fail(WF_EINVAL, "bad channel");
  ChanOp& ch = op->chans[chan];
  if (!tiles || n != ch.P) return fail(WF_EINVAL, "tiles must hold one entry per bin");
  std::vector<int8_t> tsh(ch.P, 0);
  for (int p = 0; p < ch.P; ++p) {
    if (tiles[p] == op->tile) continue;
    if (tiles[p] != 2 * op->tile)
      return fail(WF_EINVAL, "a bin's tile must be the operator's tile or twice it");
    if (op->max_tsh < 1) return fail(WF_EINVAL, "items of twice the tile do not fit in LDS");
    if (ch.otf || ch.holo)
      return fail(WF_ENOTSUP, "wider work items need stored G (strategy (a))");
    tsh[p] = 1;
  }
  WF_HIP(hipSetDevice(op->device));
  if ((st = retune_channel(op, chan, ch.max_rows, tsh.data())) != WF_OK) return st;
  op->generation++;
  if (op->sweep.on) {
    WF_HIP(hipDeviceSynchronize());
    if ((st = sweep_lanes(op, (int)op->sweep.lanes.size())) != WF_OK) return st;
  }
  return WF_OK;
}

wf_status wf_set_bin_tiles(wf_op* op, int32_t chan, const int32_t* tiles, int32_t n) {
  return guarded([&] { return wf_set_bin_tiles_body(op, chan, tiles, n); });
}

wf_status wf_autotune(wf_op* op, const float* d_img, float* d_out, void* hip_stream, int32_t reps,
                      wf_tune_info* info) {
  try {
    wf_status st = check_op(op);
    if (st != WF_OK) return st;
    if (!d_img || !d_out || reps < 1) return fail(WF_EINVAL, "bad autotune arguments");
    WF_HIP(hipSetDevice(op->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const int kind = WF_APPLY_PSF_RE;
    auto sweep = [&]() { return run_apply(op, kind, d_img, d_out, s); };
    double before = 0;
    if ((st = time_runs(s, reps, sweep, &before)) != WF_OK) return st;
    int retuned = 0;
    int64_t big_bins = 0;
    const int32_t cand_rows[3] = {256, 512, 1024};
    const Lane L = lane_of(op, 0, s);
    const int64_t grid_floats = 2 * (int64_t)op->Kx * op->Ky;
    // the fused kernel alone reads X (any finite values) and adds into Y, which is
    // cleared again afterwards
    WF_HIP(launch_fill_zero(L.X, grid_floats, s));
    for (int c = 0; c < (int)op->chans.size(); ++c) {
      ChanOp& ch = op->chans[c];
      if (ch.nrows == 0) continue;
      const int32_t orig = ch.max_rows;
      if (ch.otf || ch.holo) {
        // no stored G to time alone: whole-channel applies choose the rows per item
        int32_t best = orig;
        double best_ms = 1e300;
        for (int32_t mr : cand_rows) {
          if ((st = retune_channel(op, c, mr)) != WF_OK) return st;
          double tc = 0;
          st = time_runs(s, reps, [&]() { return run_channel(op, kind, c, L, d_img, d_out); },
                         &tc);
          if (st != WF_OK) return st;
          if (tc < best_ms) {
            best_ms = tc;
            best = mr;
          }
        }
        if ((st = retune_channel(op, c, best)) != WF_OK) return st;
        ch.measured_ms = best_ms;
        if (best != orig) ++retuned;
        continue;
      }
      const std::vector<int8_t> orig_tsh = ch.bin_tsh;
      const int nsh = op->max_tsh + 1;
      // fused-kernel time of every bin under each (rows per item, item tile)
      std::vector<double> t((size_t)3 * nsh * ch.P, 0.0);
      for (int i = 0; i < 3; ++i)
        for (int sh = 0; sh < nsh; ++sh) {
          const std::vector<int8_t> all(ch.P, (int8_t)sh);
          if ((st = retune_channel(op, c, cand_rows[i], all.data())) != WF_OK) return st;
          for (int p = 0; p < ch.P; ++p) {
            if (ch.bin_nrows[p] == 0) continue;
            double ms = 0;
            st = time_runs(s, reps, [&]() { return bin_gtg(op, ch, p, L); }, &ms);
            if (st != WF_OK) return st;
            t[((size_t)i * nsh + sh) * ch.P + p] = ms;
          }
        }
      int best = 0;
      double best_ms = 1e300;
      std::vector<int8_t> best_tsh(ch.P, 0);
      for (int i = 0; i < 3; ++i) {
        double sum = 0;
        std::vector<int8_t> pick(ch.P, 0);
        for (int p = 0; p < ch.P; ++p) {
          double m = 1e300;
          for (int sh = 0; sh < nsh; ++sh) {
            const double v = t[((size_t)i * nsh + sh) * ch.P + p];
            if (v < m) {
              m = v;
              pick[p] = (int8_t)sh;
            }
          }
          sum += m;
        }
        if (sum < best_ms) {
          best_ms = sum;
          best = i;
          best_tsh = pick;
        }
      }
      if ((st = retune_channel(op, c, cand_rows[best], best_tsh.data())) != WF_OK) return st;
      for (int p = 0; p < ch.P; ++p) big_bins += best_tsh[p] > 0;
      double tc = 0;
      st = time_runs(s, reps, [&]() { return run_channel(op, kind, c, L, d_img, d_out); }, &tc);
      if (st != WF_OK) return st;
      ch.measured_ms = tc;
      if (cand_rows[best] != orig || ch.bin_tsh != orig_tsh) ++retuned;
    }
    WF_HIP(launch_fill_zero(L.Y, grid_floats, s));
    const int nchan = (int)op->chans.size();
    if (op->sweep.on) {
      // a layer-batched sweep has no branches: its item lists follow the new splits, and
      // its lane count (channel ranges on streams of their own) is timed instead
      int best_nl = 1;
      double best_ms = 1e300;
      for (int nl = 1; nl <= std::min(nchan, 3); ++nl) {
        WF_HIP(hipDeviceSynchronize());
        if ((st = sweep_lanes(op, nl)) != WF_OK) return st;
        double t = 0;
        if ((st = time_runs(s, reps, sweep, &t)) != WF_OK) return st;
        if (t < best_ms) {
          best_ms = t;
          best_nl = nl;
        }
      }
      WF_HIP(hipDeviceSynchronize());
      if ((st = sweep_lanes(op, best_nl)) != WF_OK) return st;
      op->generation++;
    } else {
      std::vector<int> cands = {1, 2, 4};
      if (nchan == 1) cands = {1, 2, 3, 4};
      if (nchan >= 8) cands.push_back(8);
      int best_nb = 1;
      double best_ms = 1e300;
      for (int nb : cands) {
        if (nchan > 1 && nb > nchan) continue;
        if ((st = set_branches(op, nb)) != WF_OK) return st;
        double t = 0;
        if ((st = time_runs(s, reps, sweep, &t)) != WF_OK) return st;
        if (t < best_ms) {
          best_ms = t;
          best_nb = nb;
        }
      }
      if ((st = set_branches(op, best_nb)) != WF_OK) return st;
    }
    double after = 0;
    if ((st = time_runs(s, reps, sweep, &after)) != WF_OK) return st;
    if (info) {
      info->branches = op->sweep.on ? (int32_t)op->sweep.lanes.size() : op->nbranch;
      info->retuned_chans = retuned;
      info->wide_tile_bins = (int32_t)big_bins;
      info->sweep_ms_before = before;
      info->sweep_ms_after = after;
    }
    return WF_OK;
  } catch (const std::bad_alloc&) {
    return fail(WF_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(WF_EINVAL, e.what());
  }
}

// ------------------------------------------------------------------ forward-backward

namespace {

wf_status fb_buffers(wf_op* op, bool complex_too) {
  const int64_t n = npix_of(op) * (int64_t)op->chans.size();
  wf_status st;
  if (!op->fb_h.p && (st = dalloc(op->fb_h, sizeof(float) * n)) != WF_OK) return st;
  if (!op->fb_x.p && (st = dalloc(op->fb_x, sizeof(float) * n)) != WF_OK) return st;
  if (!op->fb_red.p && (st = dalloc(op->fb_red, sizeof(float) * 4)) != WF_OK) return st;
  if (complex_too && !op->fb_c.p && (st = dalloc(op->fb_c, sizeof(float2) * n)) != WF_OK)
    return st;
  return WF_OK;
}

}  // namespace

static wf_status wf_dirty_image_body(wf_op* op, const float* d_vis, float* d_dirty, void* stream) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (!d_vis || !d_dirty) return fail(WF_EINVAL, "null pointer");
  for (const auto& ch : op->chans)
    if (ch.holo) return fail(WF_ENOTSUP, "a holographic operator has no Phi^dag");
  WF_HIP(hipSetDevice(op->device));
  if ((st = fb_buffers(op, true)) != WF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = run_apply(op, WF_APPLY_ADJOINT, d_vis, (float*)op->fb_c.p, s)) != WF_OK) return st;
  WF_HIP(launch_real_part((const float2*)op->fb_c.p, d_dirty,
                          npix_of(op) * (int64_t)op->chans.size(), s));
  return WF_OK;
}

wf_status wf_dirty_image(wf_op* op, const float* d_vis, float* d_dirty, void* stream) {
  return guarded([&] { return wf_dirty_image_body(op, d_vis, d_dirty, stream); });
}

static wf_status wf_op_norm_body(wf_op* op, int32_t iters, double* norm, void* stream) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (iters < 1 || !norm) return fail(WF_EINVAL, "bad power-iteration arguments");
  WF_HIP(hipSetDevice(op->device));
  if ((st = fb_buffers(op, false)) != WF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = npix_of(op) * (int64_t)op->chans.size();
  float* x = (float*)op->fb_x.p;
  float* z = (float*)op->fb_h.p;
  float* red = (float*)op->fb_red.p;
  WF_HIP(launch_fill_value(x, n, (float)(1.0 / std::sqrt((double)n)), s));
  for (int it = 0; it < iters; ++it) {
    if ((st = run_apply(op, WF_APPLY_PSF_RE, x, z, s)) != WF_OK) return st;
    if (it + 1 == iters) WF_HIP(launch_dot(x, z, n, red, s));
    WF_HIP(launch_dot(z, z, n, red + 1, s));
    WF_HIP(launch_normalize(x, z, n, red + 1, s));
  }
  float L = 0.f;
  WF_HIP(hipMemcpyAsync(&L, red, sizeof(float), hipMemcpyDeviceToHost, s));
  WF_HIP(hipStreamSynchronize(s));
  *norm = L;
  return WF_OK;
}

wf_status wf_op_norm(wf_op* op, int32_t iters, double* norm, void* stream) {
  return guarded([&] { return wf_op_norm_body(op, iters, norm, stream); });
}

static wf_status wf_fb_iterate_body(wf_op* op, const float* d_dirty, float* d_x, int32_t iters,
                                    double gamma, double lambda, void* stream) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (!d_dirty || !d_x || iters < 0 || !(gamma > 0) || !(lambda >= 0))
    return fail(WF_EINVAL, "bad forward-backward arguments");
  WF_HIP(hipSetDevice(op->device));
  if ((st = fb_buffers(op, false)) != WF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = npix_of(op) * (int64_t)op->chans.size();
  for (int it = 0; it < iters; ++it) {
    if ((st = run_apply(op, WF_APPLY_PSF_RE, d_x, (float*)op->fb_h.p, s)) != WF_OK) return st;
    WF_HIP(launch_fb_step(d_x, d_dirty, (const float*)op->fb_h.p, (float)gamma,
                          (float)(gamma * lambda), n, s));
  }
  return WF_OK;
}

wf_status wf_fb_iterate(wf_op* op, const float* d_dirty, float* d_x, int32_t iters, double gamma,
                        double lambda, void* stream) {
  return guarded([&] {
    return wf_fb_iterate_body(op, d_dirty, d_x, iters, gamma, lambda, stream);
  });
}

static wf_status wf_destroy_body(wf_op* op) {
  if (!op) return fail(WF_EINVAL, "null operator handle");
  destroy_op(op);
  return WF_OK;
}

wf_status wf_destroy(wf_op* op) {
  return guarded([&] { return wf_destroy_body(op); });
}

}  // extern "C"
