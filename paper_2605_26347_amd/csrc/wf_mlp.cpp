// C ABI of the residual-kernel network (include/wf.h, "learned kernels"): parameter
// management, the FP32 training step (forward, loss, backward, Adam) as a sequence of
// the library's matrix-core kernels, the training loop, and inference.
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "mlp_defs.h"
#include "wf_internal.h"

using namespace wf;

namespace {

constexpr int MAX_BATCH = 65536;
constexpr int NT_LAYERS = MLP_LAYERS + 1;

uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

double unit(uint64_t& s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

void free_mlp(wf_mlp* m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  for (DevBuf* b : {&m->params, &m->grad, &m->m, &m->v, &m->wt, &m->xb, &m->tb, &m->P, &m->dP,
                    &m->dA, &m->dB, &m->idx, &m->loss})
    dfree(*b);
  for (int l = 0; l < 4; ++l) {
    dfree(m->H[l]);
    dfree(m->Z[l]);
  }
  delete m;
}

wf_status ensure_batch(wf_mlp* m, int B) {
  if (B <= m->bcap) return WF_OK;
  const int cap = std::max(B, 1024);
  for (DevBuf* b : {&m->xb, &m->tb, &m->P, &m->dP, &m->dA, &m->dB, &m->idx}) dfree(*b);
  for (int l = 0; l < 4; ++l) {
    dfree(m->H[l]);
    dfree(m->Z[l]);
  }
  m->bcap = 0;
  wf_status st;
  const size_t f = sizeof(float);
  if ((st = dalloc(m->xb, f * cap * MLP_IN)) != WF_OK) return st;
  if ((st = dalloc(m->tb, f * cap * MLP_KOUT)) != WF_OK) return st;
  if ((st = dalloc(m->P, f * cap * MLP_OUT)) != WF_OK) return st;
  if ((st = dalloc(m->dP, f * cap * MLP_OUT)) != WF_OK) return st;
  if ((st = dalloc(m->dA, f * cap * MLP_HID)) != WF_OK) return st;
  if ((st = dalloc(m->dB, f * cap * MLP_HID)) != WF_OK) return st;
  if ((st = dalloc(m->idx, sizeof(int32_t) * cap)) != WF_OK) return st;
  for (int l = 0; l < 4; ++l) {
    if ((st = dalloc(m->H[l], f * cap * MLP_HID)) != WF_OK) return st;
    if ((st = dalloc(m->Z[l], f * cap * MLP_HID)) != WF_OK) return st;
  }
  m->bcap = cap;
  return WF_OK;
}

const float* Wp(const wf_mlp* m, int l) { return (const float*)m->params.p + mlp_w_offset(l); }
const float* Bp(const wf_mlp* m, int l) { return (const float*)m->params.p + mlp_b_offset(l); }

// Forward pass of B rows of X; the output layer writes to out (row stride MLP_OUT).
wf_status forward(wf_mlp* m, const float* X, int B, float* out, hipStream_t s) {
  WF_HIP(launch_mlp_gemm(false, false, 1, X, MLP_IN, Wp(m, 0), MLP_HID, (float*)m->H[0].p,
                         MLP_HID, (float*)m->Z[0].p, Bp(m, 0), B, MLP_HID, MLP_IN, s));
  for (int l = 1; l < MLP_LAYERS; ++l)
    WF_HIP(launch_mlp_gemm(false, false, 1, (const float*)m->H[l - 1].p, MLP_HID, Wp(m, l),
                           MLP_HID, (float*)m->H[l].p, MLP_HID, (float*)m->Z[l].p, Bp(m, l), B,
                           MLP_HID, MLP_HID, s));
  WF_HIP(launch_mlp_gemm(false, false, 2, (const float*)m->H[MLP_LAYERS - 1].p, MLP_HID,
                         Wp(m, MLP_LAYERS), MLP_OUT, out, MLP_OUT, nullptr,
                         Bp(m, MLP_LAYERS), B, MLP_OUT, MLP_HID, s));
  return WF_OK;
}

// Loss and gradient (into m->grad) of B rows X, T; loss terms added to loss[2].
wf_status loss_grad(wf_mlp* m, const float* X, const float* T, int B, float* loss,
                    hipStream_t s) {
  wf_status st;
  if ((st = forward(m, X, B, (float*)m->P.p, s)) != WF_OK) return st;
  WF_HIP(launch_mlp_loss((const float*)m->P.p, T, (float*)m->dP.p, B, loss, s));
  float* g = (float*)m->grad.p;
  const int L = MLP_LAYERS;
  // output layer: gW = H^T dP, gb = colsum(dP), dH = dP[:, :450] W[:, :450]^T
  WF_HIP(launch_mlp_gemm(true, false, 0, (const float*)m->H[L - 1].p, MLP_HID,
                         (const float*)m->dP.p, MLP_OUT, g + mlp_w_offset(L), MLP_OUT, nullptr,
                         nullptr, MLP_HID, MLP_OUT, B, s));
  WF_HIP(launch_mlp_colsum((const float*)m->dP.p, MLP_OUT, B, MLP_OUT, g + mlp_b_offset(L), s));
  WF_HIP(launch_mlp_gemm(false, true, 0, (const float*)m->dP.p, MLP_OUT, Wp(m, L), MLP_OUT,
                         (float*)m->dA.p, MLP_HID, nullptr, nullptr, B, MLP_HID, MLP_KOUT, s));
  float* dH = (float*)m->dA.p;
  float* dN = (float*)m->dB.p;
  for (int l = L - 1; l >= 0; --l) {
    WF_HIP(launch_mlp_gelu_bwd(dH, (const float*)m->Z[l].p, (int64_t)B * MLP_HID, s));
    const float* Hp = l == 0 ? X : (const float*)m->H[l - 1].p;
    const int in = mlp_fan_in(l);
    WF_HIP(launch_mlp_gemm(true, false, 0, Hp, in, dH, MLP_HID, g + mlp_w_offset(l), MLP_HID,
                           nullptr, nullptr, in, MLP_HID, B, s));
    WF_HIP(launch_mlp_colsum(dH, MLP_HID, B, MLP_HID, g + mlp_b_offset(l), s));
    if (l > 0) {
      WF_HIP(launch_mlp_gemm(false, true, 0, dH, MLP_HID, Wp(m, l), MLP_HID, dN, MLP_HID,
                             nullptr, nullptr, B, MLP_HID, MLP_HID, s));
      std::swap(dH, dN);
    }
  }
  return WF_OK;
}

wf_status adam(wf_mlp* m, float lr, hipStream_t s) {
  m->t += 1;
  const double c1 = 1.0 - std::pow(0.9, (double)m->t);
  const double c2 = 1.0 - std::pow(0.999, (double)m->t);
  WF_HIP(launch_mlp_adam((float*)m->params.p, (const float*)m->grad.p, (float*)m->m.p,
                         (float*)m->v.p, mlp_num_params(), lr, 0.9f, 0.999f, 1e-8f, (float)c1,
                         (float)c2, s));
  m->wt_dirty = true;
  return WF_OK;
}

KernelParams params_of(const wf_options* opt_in) {
  wf_options o;
  if (opt_in) o = *opt_in;
  else wf_default_options(&o);
  KernelParams kp{};
  kp.alpha = o.alpha;
  kp.eps = o.eps_w;
  kp.beta = o.beta;
  kp.i0beta = i0_series(o.beta);
  kp.J = o.J;
  kp.smax = o.smax;
  kp.o = o.oversample;
  return kp;
}

}  // namespace

namespace wf {

// BF16 inference for the operator build (weights refreshed when stale).
wf_status mlp_infer_bf16(const wf_mlp* m, const float* x, int64_t n, bool split, float* out,
                         hipStream_t s) {
  if (m->wt_dirty) {
    if (!m->wt.p) {
      wf_status st =
          dalloc(m->wt, 2 * sizeof(uint16_t) * (3 * MLP_HID * MLP_HID + 512 * MLP_HID));
      if (st != WF_OK) return st;
    }
    WF_HIP(launch_mlp_prep_bf16((const float*)m->params.p, (uint16_t*)m->wt.p, s));
    m->wt_dirty = false;
  }
  WF_HIP(launch_mlp_infer_bf16(x, n, (const float*)m->params.p, (const uint16_t*)m->wt.p,
                               split, out, s));
  return WF_OK;
}

wf_status mlp_snapshot(const wf_mlp* m, DevBuf& params, DevBuf& wt, hipStream_t s) {
  const size_t pb = sizeof(float) * (size_t)mlp_num_params();
  const size_t wb = 2 * sizeof(uint16_t) * (3 * MLP_HID * MLP_HID + 512 * MLP_HID);
  wf_status st;
  if ((st = dalloc(params, pb)) != WF_OK) return st;
  if ((st = dalloc(wt, wb)) != WF_OK) return st;
  WF_HIP(hipMemcpyAsync(params.p, m->params.p, pb, hipMemcpyDeviceToDevice, s));
  WF_HIP(launch_mlp_prep_bf16((const float*)params.p, (uint16_t*)wt.p, s));
  return WF_OK;
}

}  // namespace wf

extern "C" {

int64_t wf_mlp_num_params(void) { return mlp_num_params(); }

wf_status wf_mlp_create(uint64_t seed, wf_mlp** out) {
  try {
    if (!out) return fail(WF_EINVAL, "out is null");
    *out = nullptr;
    int dev = 0;
    WF_HIP(hipGetDevice(&dev));
    wf_mlp* m = new wf_mlp();
    m->device = dev;
    const int64_t n = mlp_num_params();
    std::vector<float> h(n, 0.f);
    uint64_t st = seed;
    for (int l = 0; l < NT_LAYERS; ++l) {
      const int in = mlp_fan_in(l), fo = mlp_fan_out(l);
      const double lim = 1.0 / std::sqrt((double)in);
      float* w = h.data() + mlp_w_offset(l);
      for (int64_t i = 0; i < (int64_t)in * fo; ++i) w[i] = (float)((2.0 * unit(st) - 1.0) * lim);
    }
    wf_status s2;
    for (DevBuf* b : {&m->params, &m->grad, &m->m, &m->v})
      if ((s2 = dalloc(*b, sizeof(float) * n)) != WF_OK) {
        free_mlp(m);
        return s2;
      }
    if ((s2 = dalloc(m->loss, sizeof(float) * 2)) != WF_OK) {
      free_mlp(m);
      return s2;
    }
    if (hipMemcpy(m->params.p, h.data(), sizeof(float) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(m->m.p, 0, sizeof(float) * n) != hipSuccess ||
        hipMemset(m->v.p, 0, sizeof(float) * n) != hipSuccess ||
        hipMemset(m->grad.p, 0, sizeof(float) * n) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
      free_mlp(m);
      return fail(WF_EHIP, "network parameter upload failed");
    }
    *out = m;
    return WF_OK;
  } catch (const std::bad_alloc&) {
    return fail(WF_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(WF_EINVAL, e.what());
  }
}

static wf_status wf_mlp_destroy_body(wf_mlp* m) {
  if (!m) return fail(WF_EINVAL, "null network handle");
  free_mlp(m);
  return WF_OK;
}

wf_status wf_mlp_destroy(wf_mlp* m) {
  return guarded([&] { return wf_mlp_destroy_body(m); });
}

static wf_status wf_mlp_get_params_body(const wf_mlp* m, float* host, int64_t n) {
  if (!m || !host) return fail(WF_EINVAL, "null pointer");
  if (n != mlp_num_params()) return fail(WF_EINVAL, "parameter count mismatch");
  WF_HIP(hipSetDevice(m->device));
  WF_HIP(hipDeviceSynchronize());
  WF_HIP(hipMemcpy(host, m->params.p, sizeof(float) * n, hipMemcpyDeviceToHost));
  return WF_OK;
}

wf_status wf_mlp_get_params(const wf_mlp* m, float* host, int64_t n) {
  return guarded([&] { return wf_mlp_get_params_body(m, host, n); });
}

static wf_status wf_mlp_set_params_body(wf_mlp* m, const float* host, int64_t n) {
  if (!m || !host) return fail(WF_EINVAL, "null pointer");
  if (n != mlp_num_params()) return fail(WF_EINVAL, "parameter count mismatch");
  WF_HIP(hipSetDevice(m->device));
  WF_HIP(hipDeviceSynchronize());
  WF_HIP(hipMemcpy(m->params.p, host, sizeof(float) * n, hipMemcpyHostToDevice));
  WF_HIP(hipMemset(m->m.p, 0, sizeof(float) * n));
  WF_HIP(hipMemset(m->v.p, 0, sizeof(float) * n));
  WF_HIP(hipDeviceSynchronize());
  m->t = 0;
  m->wt_dirty = true;
  return WF_OK;
}

wf_status wf_mlp_set_params(wf_mlp* m, const float* host, int64_t n) {
  return guarded([&] { return wf_mlp_set_params_body(m, host, n); });
}

static wf_status wf_mlp_inputs_body(const double* d_w, const double* d_L, const double* d_fu,
                                    const double* d_fv, int64_t n, const wf_options* opt,
                                    float* d_x, int32_t* d_nk, void* stream) {
  if (n < 0 || (n > 0 && (!d_w || !d_L || !d_fu || !d_fv || !d_x)))
    return fail(WF_EINVAL, "bad network input arguments");
  WF_HIP(launch_train_inputs(d_w, d_L, d_fu, d_fv, n, params_of(opt), d_x, d_nk,
                             (hipStream_t)stream));
  return WF_OK;
}

wf_status wf_mlp_inputs(const double* d_w, const double* d_L, const double* d_fu,
                        const double* d_fv, int64_t n, const wf_options* opt, float* d_x,
                        int32_t* d_nk, void* stream) {
  return guarded([&] {
    return wf_mlp_inputs_body(d_w, d_L, d_fu, d_fv, n, opt, d_x, d_nk, stream);
  });
}

static wf_status wf_mlp_targets_body(const double* d_w, const double* d_L, int64_t n,
                                     const wf_options* opt, float* d_t, void* stream) {
  if (n < 0 || (n > 0 && (!d_w || !d_L || !d_t)))
    return fail(WF_EINVAL, "bad network target arguments");
  WF_HIP(launch_exact_targets(d_w, d_L, n, params_of(opt), d_t, (hipStream_t)stream));
  return WF_OK;
}

wf_status wf_mlp_targets(const double* d_w, const double* d_L, int64_t n, const wf_options* opt,
                         float* d_t, void* stream) {
  return guarded([&] { return wf_mlp_targets_body(d_w, d_L, n, opt, d_t, stream); });
}

static wf_status wf_mlp_loss_grad_body(wf_mlp* m, const float* d_x, const float* d_t, int32_t batch,
                                       float* d_grad, float* d_loss, void* stream) {
  if (!m || !d_x || !d_t || !d_loss) return fail(WF_EINVAL, "null pointer");
  if (batch < 1 || batch > MAX_BATCH) return fail(WF_EINVAL, "batch must be in [1,65536]");
  WF_HIP(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)stream;
  wf_status st;
  if ((st = ensure_batch(m, batch)) != WF_OK) return st;
  WF_HIP(launch_fill_zero(d_loss, 2, s));
  if ((st = loss_grad(m, d_x, d_t, batch, d_loss, s)) != WF_OK) return st;
  if (d_grad)
    WF_HIP(hipMemcpyAsync(d_grad, m->grad.p, sizeof(float) * mlp_num_params(),
                          hipMemcpyDeviceToDevice, s));
  return WF_OK;
}

wf_status wf_mlp_loss_grad(wf_mlp* m, const float* d_x, const float* d_t, int32_t batch,
                           float* d_grad, float* d_loss, void* stream) {
  return guarded([&] { return wf_mlp_loss_grad_body(m, d_x, d_t, batch, d_grad, d_loss, stream); });
}

static wf_status wf_mlp_adam_step_body(wf_mlp* m, float lr, void* stream) {
  if (!m) return fail(WF_EINVAL, "null network handle");
  WF_HIP(hipSetDevice(m->device));
  return adam(m, lr, (hipStream_t)stream);
}

wf_status wf_mlp_adam_step(wf_mlp* m, float lr, void* stream) {
  return guarded([&] { return wf_mlp_adam_step_body(m, lr, stream); });
}

wf_status wf_mlp_train(wf_mlp* m, const float* d_x, const float* d_t, int64_t n, int32_t batch,
                       int32_t epochs, double lr0, double lr_end, uint64_t seed, float* d_hist,
                       void* stream) {
  try {
    if (!m || !d_x || !d_t) return fail(WF_EINVAL, "null pointer");
    if (batch < 1 || batch > MAX_BATCH || n < batch || epochs < 0 || n > INT32_MAX)
      return fail(WF_EINVAL, "bad batch / example count / epochs");
    if (!(lr0 > 0) || !(lr_end > 0)) return fail(WF_EINVAL, "learning rates must be positive");
    WF_HIP(hipSetDevice(m->device));
    hipStream_t s = (hipStream_t)stream;
    wf_status st;
    if ((st = ensure_batch(m, batch)) != WF_OK) return st;
    DevBuf perm;
    if ((st = dalloc(perm, sizeof(int32_t) * n)) != WF_OK) return st;
    struct Guard {
      DevBuf* b;
      ~Guard() { dfree(*b); }
    } guard{&perm};
    const int64_t steps = n / batch;
    const double total = (double)steps * epochs;
    std::vector<int32_t> idx(n);
    uint64_t rs = seed;
    int64_t t = 0;
    for (int e = 0; e < epochs; ++e) {
      std::iota(idx.begin(), idx.end(), 0);
      for (int64_t i = n - 1; i > 0; --i) {
        const int64_t j = (int64_t)(splitmix64(rs) % (uint64_t)(i + 1));
        std::swap(idx[i], idx[j]);
      }
      WF_HIP(hipStreamSynchronize(s));
      WF_HIP(hipMemcpy(perm.p, idx.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
      float* lossp = d_hist ? d_hist + 2 * e : (float*)m->loss.p;
      WF_HIP(launch_fill_zero(lossp, 2, s));
      for (int64_t k = 0; k < steps; ++k, ++t) {
        WF_HIP(launch_mlp_gather(d_x, MLP_IN, d_t, MLP_KOUT, (const int32_t*)perm.p + k * batch,
                                 batch, (float*)m->xb.p, (float*)m->tb.p, s));
        if ((st = loss_grad(m, (const float*)m->xb.p, (const float*)m->tb.p, batch, lossp, s)) !=
            WF_OK)
          return st;
        const double lr =
            lr_end + 0.5 * (lr0 - lr_end) * (1.0 + std::cos(M_PI * (double)t / total));
        if ((st = adam(m, (float)lr, s)) != WF_OK) return st;
      }
    }
    WF_HIP(hipStreamSynchronize(s));
    return WF_OK;
  } catch (const std::bad_alloc&) {
    return fail(WF_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(WF_EINVAL, e.what());
  }
}

static wf_status wf_mlp_infer_body(wf_mlp* m, const float* d_x, int64_t n, int32_t bf16,
                                   float* d_out, void* stream) {
  if (!m || (n > 0 && (!d_x || !d_out))) return fail(WF_EINVAL, "null pointer");
  if (n < 0) return fail(WF_EINVAL, "negative row count");
  WF_HIP(hipSetDevice(m->device));
  hipStream_t s = (hipStream_t)stream;
  if (bf16 < 0 || bf16 > 2) return fail(WF_EINVAL, "bf16 must be 0, 1 or 2");
  if (bf16) return mlp_infer_bf16(m, d_x, n, bf16 == 2, d_out, s);
  wf_status st;
  const int chunk = (int)std::min<int64_t>(std::max<int64_t>(n, 1), MAX_BATCH);
  if ((st = ensure_batch(m, chunk)) != WF_OK) return st;
  for (int64_t r0 = 0; r0 < n; r0 += chunk) {
    const int B = (int)std::min<int64_t>(chunk, n - r0);
    if ((st = forward(m, d_x + r0 * MLP_IN, B, d_out + r0 * MLP_OUT, s)) != WF_OK) return st;
  }
  return WF_OK;
}

wf_status wf_mlp_infer(wf_mlp* m, const float* d_x, int64_t n, int32_t bf16, float* d_out,
                       void* stream) {
  return guarded([&] { return wf_mlp_infer_body(m, d_x, n, bf16, d_out, stream); });
}

}  // extern "C"
