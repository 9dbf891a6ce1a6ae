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

#include "wf_internal.h"

using namespace wf;

namespace {

thread_local std::string g_err;

wf_status fail(wf_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define WF_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(WF_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

constexpr double C_LIGHT = 299792458.0;

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
  }
  dfree(op->X);
  dfree(op->Y);
  dfree(op->A);
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
    if (!p->enabled) return;
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

wf_status build_channel(wf_op* op, int c, const double* uvw, int64_t M, double freq,
                        int64_t vis_off, uint64_t budget, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  ChanOp& ch = op->chans[c];
  const wf_options& opt = op->opt;
  ch.freq = freq;
  ch.scale = freq / C_LIGHT;
  ch.vis_off = vis_off;
  ch.nrows = M;
  std::vector<double> w(M);
  for (int64_t k = 0; k < M; ++k) w[k] = uvw[3 * k + 2] * ch.scale;
  PlanResult pr;
  std::string perr;
  if (M > 0) {
    if (plan_channel(w.data(), M, op->shape, opt, budget, &pr, &perr) != 0) {
      return fail(WF_ENOTSUP, "channel " + std::to_string(c) + ": " + perr +
                                  "; holographic and on-the-fly strategies are not built");
    }
  } else {
    pr.P = 1;
    pr.centroids = {0.0};
  }
  if (opt.strategy == WF_PRECOMP_H || opt.strategy == WF_ONTHEFLY)
    return fail(WF_ENOTSUP, "only the precomputed-G strategy is built");
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
  WF_HIP(hipMemcpyAsync(dmids.p, mids.data(), sizeof(double) * mids.size(),
                        hipMemcpyHostToDevice, s));
  WF_HIP(hipMemcpyAsync(dcents.p, ch.centroids.data(), sizeof(double) * ch.P,
                        hipMemcpyHostToDevice, s));
  WF_HIP(launch_rowsym((const double*)duvw.p, M, ch.scale, gsx, gsy, (const double*)dmids.p,
                       ch.P, (const double*)dcents.p, Kx, Ky, tile, op->kp,
                       (uint64_t*)dkeys.p, (float*)ddrop.p, s));
  std::vector<uint64_t> keys(M);
  std::vector<float> dropped(M);
  WF_HIP(hipMemcpyAsync(keys.data(), dkeys.p, sizeof(uint64_t) * M, hipMemcpyDeviceToHost, s));
  WF_HIP(hipMemcpyAsync(dropped.data(), ddrop.p, sizeof(float) * M, hipMemcpyDeviceToHost, s));
  WF_HIP(hipStreamSynchronize(s));
  dfree(dkeys);
  dfree(ddrop);
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
  radix_sort_pairs(keys, idx, 16);

  // work items: runs of one (bin, tile, patch class), split for load balance; within a
  // bin the items are then grouped by patch class (one launch per class)
  // (the row kernels hold a wavefront's metadata for at most 128 rows in registers)
  const int64_t maxrows = opt.max_rows_per_item > 0 ? opt.max_rows_per_item : 1024;
  const int64_t maxtaps = 1 << 20;
  std::vector<WorkItem> wis0;
  std::vector<int> wcls;
  std::vector<uint32_t> meta(M), voff(M);
  std::vector<int32_t> row_wi(M);
  ch.bin_row0.assign(ch.P, 0);
  ch.bin_nrows.assign(ch.P, 0);
  int64_t taps_total = 0, taps_in = 0;
  uint64_t cur = ~0ull;
  int curcls = -1;
  for (int64_t sidx = 0; sidx < M; ++sidx) {
    const uint64_t k = keys[sidx];
    const int bin = (int)(k >> 56);
    const int tv = (int)((k >> 46) & 1023), tu = (int)((k >> 36) & 1023);
    const int T = (int)((k >> 30) & 63);
    const int lv = (int)((k >> 23) & 127), lu = (int)((k >> 16) & 127);
    const uint64_t grp = k >> 36;
    const int cls = tap_class(T);
    if (grp != cur || cls != curcls || wis0.back().nrows >= maxrows ||
        taps_in + T * T > maxtaps) {
      WorkItem wi{};
      wi.voff = taps_total;
      wi.row0 = (int32_t)sidx;
      wi.nrows = 0;
      wi.u0 = tu * tile - halo;
      wi.v0 = tv * tile - halo;
      wi.bin = bin;
      if (wis0.empty() || wis0.back().bin != bin) ch.bin_row0[bin] = sidx;
      wis0.push_back(wi);
      wcls.push_back(cls);
      cur = grp;
      curcls = cls;
      taps_in = 0;
    }
    WorkItem& wi = wis0.back();
    voff[sidx] = (uint32_t)taps_in;
    const int off = (T - 1) / 2;
    meta[sidx] = pack_meta(lu + halo - off, lv + halo - off, T);
    row_wi[sidx] = (int32_t)(wis0.size() - 1);
    wi.nrows++;
    taps_in += (int64_t)T * T;
    taps_total += (int64_t)T * T;
    ch.bin_nrows[bin]++;
  }
  // group by (bin, class); inside a group the largest items (most taps) come first so
  // that the hardware's in-order dispatch schedules longest work first
  std::vector<int64_t> wtaps(wis0.size());
  for (size_t i = 0; i < wis0.size(); ++i) {
    const int64_t end = (i + 1 < wis0.size()) ? wis0[i + 1].voff : taps_total;
    wtaps[i] = end - wis0[i].voff;
  }
  std::vector<int32_t> order(wis0.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    if (wis0[x].bin != wis0[y].bin) return wis0[x].bin < wis0[y].bin;
    if (wcls[x] != wcls[y]) return wcls[x] < wcls[y];
    return wtaps[x] > wtaps[y];
  });
  std::vector<WorkItem> wis(wis0.size());
  std::vector<int32_t> newidx(wis0.size());
  ch.bin_wi0.assign(ch.P, 0);
  ch.bin_nwi.assign(ch.P, 0);
  ch.cls_wi0.assign((size_t)ch.P * NCLS, 0);
  ch.cls_nwi.assign((size_t)ch.P * NCLS, 0);
  for (size_t i = 0; i < order.size(); ++i) {
    const WorkItem& w = wis0[order[i]];
    wis[i] = w;
    newidx[order[i]] = (int32_t)i;
    const int b = w.bin, c = wcls[order[i]];
    if (ch.bin_nwi[b] == 0) ch.bin_wi0[b] = (int32_t)i;
    ch.bin_nwi[b]++;
    if (ch.cls_nwi[b * NCLS + c] == 0) ch.cls_wi0[b * NCLS + c] = (int32_t)i;
    ch.cls_nwi[b * NCLS + c]++;
  }
  for (int64_t sidx = 0; sidx < M; ++sidx) row_wi[sidx] = newidx[row_wi[sidx]];

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
    std::vector<uint8_t> act((size_t)tx * ty), need((size_t)tx * ty);
    for (int p = 0; p < ch.P; ++p) {
      std::fill(act.begin(), act.end(), 0);
      std::fill(need.begin(), need.end(), 0);
      for (int i = 0; i < ch.bin_nwi[p]; ++i) {
        const WorkItem& w = wis[ch.bin_wi0[p] + i];
        const int tu = (w.u0 + halo) / tile, tv = (w.v0 + halo) / tile;
        act[(size_t)tv * tx + tu] = 1;
      }
      for (int tv = 0; tv < ty; ++tv)
        for (int tu = 0; tu < tx; ++tu) {
          if (!act[(size_t)tv * tx + tu]) continue;
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
  const int b_v = opt.store == WF_STORE_F32 ? 8 : 4;
  DevBuf drowwi, dmis;
  tmp.b.push_back(&drowwi);
  tmp.b.push_back(&dmis);
  if ((st = dalloc(dmis, sizeof(int))) != WF_OK) return st;
  WF_HIP(hipMemsetAsync(dmis.p, 0, sizeof(int), s));
  if ((st = dalloc(ch.meta, sizeof(uint32_t) * std::max<int64_t>(M, 1))) != WF_OK) return st;
  if ((st = dalloc(ch.voff, sizeof(uint32_t) * std::max<int64_t>(M, 1))) != WF_OK) return st;
  if ((st = dalloc(ch.perm, sizeof(int32_t) * std::max<int64_t>(M, 1))) != WF_OK) return st;
  if ((st = dalloc(ch.work, sizeof(WorkItem) * std::max<size_t>(wis.size(), 1))) != WF_OK)
    return st;
  if ((st = dalloc(drowwi, sizeof(int32_t) * std::max<int64_t>(M, 1))) != WF_OK) return st;
  if ((st = dalloc(ch.vals, (size_t)b_v * std::max<int64_t>(taps_total, 1))) != WF_OK)
    return st;
  WF_HIP(hipMemcpyAsync(ch.meta.p, meta.data(), sizeof(uint32_t) * M, hipMemcpyHostToDevice, s));
  WF_HIP(hipMemcpyAsync(ch.voff.p, voff.data(), sizeof(uint32_t) * M, hipMemcpyHostToDevice, s));
  WF_HIP(hipMemcpyAsync(ch.perm.p, idx.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, s));
  WF_HIP(hipMemcpyAsync(drowwi.p, row_wi.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, s));
  WF_HIP(hipMemcpyAsync(ch.work.p, wis.data(), sizeof(WorkItem) * wis.size(),
                        hipMemcpyHostToDevice, s));
  WF_HIP(launch_gbuild((const double*)duvw.p, M, (const int32_t*)ch.perm.p,
                       (const uint32_t*)ch.meta.p, (const uint32_t*)ch.voff.p,
                       (const int32_t*)drowwi.p, (const WorkItem*)ch.work.p, ch.scale, gsx,
                       gsy, (const double*)dmids.p, ch.P, (const double*)dcents.p, op->kp,
                       ch.vals.p, opt.store, (int*)dmis.p, s));
  int mismatch = 0;
  WF_HIP(hipMemcpyAsync(&mismatch, dmis.p, sizeof(int), hipMemcpyDeviceToHost, s));
  WF_HIP(hipStreamSynchronize(s));
  if (mismatch != 0)
    return fail(WF_EINVAL, std::to_string(mismatch) +
                               " rows changed patch side between the symbolic and value passes");

  wf_plan_info& in = ch.info;
  in.nchan = (int32_t)op->chans.size();
  in.nbins = ch.P;
  in.strategy = WF_PRECOMP_G;
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
  in.mem_g_bytes = (double)b_v * taps_total + 12.0 * M + sizeof(WorkItem) * wis.size();
  in.mem_model_bytes = pr.mem_model;
  in.cost_model = pr.cost_model;
  in.capped_fraction = M ? (double)ncapped / (double)M : 0.0;
  in.max_dropped_energy = maxdrop;
  in.build_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
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

// One w-layer's forward half: X_p = F Z_p x (only inside the bin's support if pr).
wf_status layer_forward(wf_op* op, const float* x, double wp, const ColPrune* pr,
                        hipStream_t s) {
  const int nx = op->shape.nx, ny = op->shape.ny;
  {
    ProfScope ps(&op->prof[1], s);
    WF_HIP(launch_fwd_rows(x, (float2*)op->A.p, (const float2*)op->twx.p,
                           (const float*)op->sx.p, (const float*)op->sy.p, nx, ny, op->Kx,
                           op->shape.cell_rad, wp, pr ? pr->strip : nullptr, s));
  }
  {
    ProfScope ps(&op->prof[2], s);
    WF_HIP(launch_fwd_cols((const float2*)op->A.p, (float2*)op->X.p, (const float2*)op->twy.p,
                           ny, op->Kx, op->Ky, pr, s));
  }
  return WF_OK;
}

// One w-layer's adjoint half from the gridded Y: out (+)= Z_p^dag F^dag Y (Y is cleared
// where it was read; outside the bin's support it is zero already).
wf_status layer_adjoint(wf_op* op, void* out, double wp, int mode, const ColPrune* pr,
                        hipStream_t s) {
  const int nx = op->shape.nx, ny = op->shape.ny;
  {
    ProfScope ps(&op->prof[3], s);
    WF_HIP(launch_inv_cols((float2*)op->Y.p, (float2*)op->A.p, (const float2*)op->twy.p, ny,
                           op->Kx, op->Ky, pr, s));
  }
  {
    ProfScope ps(&op->prof[4], s);
    WF_HIP(launch_inv_rows((const float2*)op->A.p, out, (const float2*)op->twx.p,
                           (const float*)op->sx.p, (const float*)op->sy.p, nx, ny, op->Kx,
                           op->shape.cell_rad, wp, mode, pr ? pr->strip : nullptr, s));
  }
  return WF_OK;
}

wf_status psf_common(wf_op* op, const float* d_img, float* d_out, void* stream, bool re) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (!d_img || !d_out) return fail(WF_EINVAL, "null image pointer");
  WF_HIP(hipSetDevice(op->device));
  hipStream_t s = (hipStream_t)stream;
  const int64_t npix = (int64_t)op->shape.nx * op->shape.ny;
  for (size_t c = 0; c < op->chans.size(); ++c) {
    ChanOp& ch = op->chans[c];
    const float* x = d_img + c * npix;
    void* out = re ? (void*)(d_out + c * npix) : (void*)(d_out + 2 * c * npix);
    bool first = true;
    for (int p = 0; p < ch.P; ++p) {
      if (ch.bin_nrows[p] == 0) continue;
      const double wp = ch.centroids[p];
      const ColPrune pr = prune_of(op, ch, p);
      if ((st = layer_forward(op, x, wp, &pr, s)) != WF_OK) return st;
      {
        ProfScope ps(&op->prof[0], s);
        for (int c = 0; c < NCLS; ++c) {
          const int n = ch.cls_nwi[p * NCLS + c];
          if (n == 0) continue;
          WF_HIP(launch_gtg(c, (const WorkItem*)ch.work.p + ch.cls_wi0[p * NCLS + c], n,
                            (const uint32_t*)ch.meta.p, (const uint32_t*)ch.voff.p, ch.vals.p,
                            op->opt.store, (const float2*)op->X.p, (float2*)op->Y.p, op->Kx,
                            op->Ky, op->win, s));
        }
      }
      const int mode = (re ? 2 : 0) + (first ? 0 : 1);
      if ((st = layer_adjoint(op, out, wp, mode, &pr, s)) != WF_OK) return st;
      first = false;
    }
    if (first) WF_HIP(hipMemsetAsync(out, 0, npix * (re ? 4 : 8), s));
  }
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
    const int64_t per_chan_max = chan_rows ? 0 : nrows;
    if (per_chan_max > INT32_MAX) return fail(WF_EINVAL, "too many rows per channel");
    if (chan_rows)
      for (int c = 0; c < nchan; ++c)
        if (chan_rows[c] > INT32_MAX) return fail(WF_EINVAL, "too many rows per channel");

    OpGuard guard{new wf_op()};
    wf_op* op = guard.op;
    op->opt = opt;
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
    if (op->win > 255 || (op->Kx / tile) > 1024 || (op->Ky / tile) > 1024)
      return fail(WF_EINVAL, "tile/halo too large");
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
    if ((st = dalloc(op->X, sizeof(float2) * (size_t)Kx * Ky)) != WF_OK) return st;
    if ((st = dalloc(op->Y, sizeof(float2) * (size_t)Kx * Ky)) != WF_OK) return st;
    if ((st = dalloc(op->A, sizeof(float2) * (size_t)ny * Kx)) != WF_OK) return st;
    if ((st = dalloc(op->twx, sizeof(float2) * Kx)) != WF_OK) return st;
    if ((st = dalloc(op->twy, sizeof(float2) * Ky)) != WF_OK) return st;
    if ((st = dalloc(op->sx, sizeof(float) * nx)) != WF_OK) return st;
    if ((st = dalloc(op->sy, sizeof(float) * ny)) != WF_OK) return st;
    WF_HIP(hipMemsetAsync(op->Y.p, 0, op->Y.bytes, s));
    WF_HIP(hipMemcpyAsync(op->twx.p, twx.data(), sizeof(float2) * Kx, hipMemcpyHostToDevice, s));
    WF_HIP(hipMemcpyAsync(op->twy.p, twy.data(), sizeof(float2) * Ky, hipMemcpyHostToDevice, s));
    WF_HIP(hipMemcpyAsync(op->sx.p, sx.data(), sizeof(float) * nx, hipMemcpyHostToDevice, s));
    WF_HIP(hipMemcpyAsync(op->sy.p, sy.data(), sizeof(float) * ny, hipMemcpyHostToDevice, s));

    op->chans.resize(nchan);
    int64_t off = 0;
    for (int c = 0; c < nchan; ++c) {
      const int64_t Mc = chan_rows ? chan_rows[c] : nrows;
      const double* u = chan_rows ? uvw_m + 3 * off : uvw_m;
      if ((st = build_channel(op, c, u, Mc, freqs_hz[c], op->total_rows, memory_budget_bytes,
                              s)) != WF_OK)
        return st;
      op->total_rows += Mc;
      if (chan_rows) off += Mc;
    }
    for (auto& ch : op->chans) ch.info.nchan = nchan;
    WF_HIP(hipStreamSynchronize(s));
    *out = op;
    guard.op = nullptr;
    return WF_OK;
  } catch (const std::bad_alloc&) {
    return fail(WF_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(WF_EINVAL, e.what());
  }
}

wf_status wf_forward(wf_op* op, const float* d_img, float* d_vis, void* stream) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (!d_img || !d_vis) return fail(WF_EINVAL, "null pointer");
  WF_HIP(hipSetDevice(op->device));
  hipStream_t s = (hipStream_t)stream;
  const int64_t npix = (int64_t)op->shape.nx * op->shape.ny;
  for (size_t c = 0; c < op->chans.size(); ++c) {
    ChanOp& ch = op->chans[c];
    for (int p = 0; p < ch.P; ++p) {
      if (ch.bin_nrows[p] == 0) continue;
      const ColPrune pr = prune_of(op, ch, p);
      if ((st = layer_forward(op, d_img + c * npix, ch.centroids[p], &pr, s)) != WF_OK)
        return st;
      for (int c = 0; c < NCLS; ++c) {
        const int n = ch.cls_nwi[p * NCLS + c];
        if (n == 0) continue;
        WF_HIP(launch_degrid(c, (const WorkItem*)ch.work.p + ch.cls_wi0[p * NCLS + c], n,
                             (const uint32_t*)ch.meta.p, (const uint32_t*)ch.voff.p,
                             (const int32_t*)ch.perm.p, ch.vals.p, op->opt.store,
                             (const float2*)op->X.p, (float2*)d_vis + ch.vis_off, op->Kx,
                             op->Ky, s));
      }
    }
  }
  return WF_OK;
}

wf_status wf_adjoint(wf_op* op, const float* d_vis, float* d_img, void* stream) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (!d_img || !d_vis) return fail(WF_EINVAL, "null pointer");
  WF_HIP(hipSetDevice(op->device));
  hipStream_t s = (hipStream_t)stream;
  const int64_t npix = (int64_t)op->shape.nx * op->shape.ny;
  for (size_t c = 0; c < op->chans.size(); ++c) {
    ChanOp& ch = op->chans[c];
    void* out = (void*)(d_img + 2 * c * npix);
    bool first = true;
    for (int p = 0; p < ch.P; ++p) {
      if (ch.bin_nrows[p] == 0) continue;
      for (int c = 0; c < NCLS; ++c) {
        const int n = ch.cls_nwi[p * NCLS + c];
        if (n == 0) continue;
        WF_HIP(launch_grid(c, (const WorkItem*)ch.work.p + ch.cls_wi0[p * NCLS + c], n,
                           (const uint32_t*)ch.meta.p, (const uint32_t*)ch.voff.p,
                           (const int32_t*)ch.perm.p, ch.vals.p, op->opt.store,
                           (const float2*)d_vis + ch.vis_off, (float2*)op->Y.p, op->Kx,
                           op->Ky, op->win, s));
      }
      const ColPrune pr = prune_of(op, ch, p);
      if ((st = layer_adjoint(op, out, ch.centroids[p], first ? 0 : 1, &pr, s)) != WF_OK)
        return st;
      first = false;
    }
    if (first) WF_HIP(hipMemsetAsync(out, 0, npix * 8, s));
  }
  return WF_OK;
}

wf_status wf_psf_apply(wf_op* op, const float* d_img, float* d_out, void* stream) {
  return psf_common(op, d_img, d_out, stream, false);
}

wf_status wf_psf_apply_re(wf_op* op, const float* d_img, float* d_out, void* stream) {
  return psf_common(op, d_img, d_out, stream, true);
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
    if (row < 0 || row >= ch.nrows) return fail(WF_EINVAL, "row out of range");
    WF_HIP(hipSetDevice(op->device));
    WF_HIP(hipDeviceSynchronize());
    std::vector<int32_t> perm(ch.nrows);
    WF_HIP(hipMemcpy(perm.data(), ch.perm.p, sizeof(int32_t) * ch.nrows, hipMemcpyDeviceToHost));
    int64_t s = -1;
    for (int64_t i = 0; i < ch.nrows; ++i)
      if (perm[i] == row) {
        s = i;
        break;
      }
    if (s < 0) return fail(WF_EINVAL, "row not found");
    uint32_t m, vo;
    WF_HIP(hipMemcpy(&m, (const uint32_t*)ch.meta.p + s, 4, hipMemcpyDeviceToHost));
    WF_HIP(hipMemcpy(&vo, (const uint32_t*)ch.voff.p + s, 4, hipMemcpyDeviceToHost));
    std::vector<WorkItem> wis(ch.nwork);
    WF_HIP(hipMemcpy(wis.data(), ch.work.p, sizeof(WorkItem) * ch.nwork, hipMemcpyDeviceToHost));
    int64_t w = 0;
    for (int64_t i = 0; i < ch.nwork; ++i)
      if (s >= wis[i].row0 && s < wis[i].row0 + wis[i].nrows) {
        w = i;
        break;
      }
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

wf_status wf_layer_grid(wf_op* op, int32_t chan, int32_t bin, const float* d_img,
                        float* d_grid, void* stream) {
  wf_status st = check_op(op);
  if (st != WF_OK) return st;
  if (chan < 0 || chan >= (int)op->chans.size()) return fail(WF_EINVAL, "bad channel");
  const ChanOp& ch = op->chans[chan];
  if (bin < 0 || bin >= ch.P || !d_img || !d_grid) return fail(WF_EINVAL, "bad bin/pointer");
  WF_HIP(hipSetDevice(op->device));
  hipStream_t s = (hipStream_t)stream;
  const int64_t npix = (int64_t)op->shape.nx * op->shape.ny;
  if ((st = layer_forward(op, d_img + chan * npix, ch.centroids[bin], nullptr, s)) != WF_OK)
    return st;
  WF_HIP(launch_strip_to_rowmajor((const float2*)op->X.p, (float2*)d_grid, op->Ky, op->Kx, s));
  return WF_OK;
}

wf_status wf_profile_enable(wf_op* op, int32_t kernel_id, int32_t enable) {
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

wf_status wf_profile_read(wf_op* op, int32_t kernel_id, int64_t* launches, double* total_ms) {
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

wf_status wf_destroy(wf_op* op) {
  if (!op) return fail(WF_EINVAL, "null operator handle");
  destroy_op(op);
  return WF_OK;
}

}  // extern "C"
