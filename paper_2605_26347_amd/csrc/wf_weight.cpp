// C ABI of the Briggs robust weights (include/wf.h, wf_briggs_weights): per channel,
// upload the channel's coordinates and natural weights, grid the weight density, reduce
// the two sums that fix f^2, and write the operator weights back to the host.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "wf_internal.h"

using namespace wf;

namespace {

constexpr double C_LIGHT_MS = 299792458.0;

struct Bufs {
  DevBuf uvw, w, flags, W, sums, out;
  ~Bufs() {
    for (DevBuf* b : {&uvw, &w, &flags, &W, &sums, &out}) dfree(*b);
  }
};

}  // namespace

extern "C" wf_status wf_briggs_weights(const double* uvw_m, int64_t nrows,
                                       const int64_t* chan_rows, const double* freqs_hz,
                                       int32_t nchan, wf_image_shape shape, double robust,
                                       const float* natural, const uint8_t* flags, float* out,
                                       void* hip_stream) {
  try {
    if (nrows < 0 || nchan <= 0 || !freqs_hz || !out)
      return fail(WF_EINVAL, "bad row/channel counts or null output");
    if (nrows > 0 && !uvw_m) return fail(WF_EINVAL, "uvw is null");
    if (shape.nx < 1 || shape.ny < 1 || shape.nx > 65536 || shape.ny > 65536)
      return fail(WF_EINVAL, "nx, ny must be in [1, 65536]");
    if (!(shape.cell_rad > 0.0) || !std::isfinite(shape.cell_rad))
      return fail(WF_EINVAL, "cell must be positive");
    if (!std::isfinite(robust)) return fail(WF_EINVAL, "robustness must be finite");
    int64_t total = 0;
    if (chan_rows) {
      for (int c = 0; c < nchan; ++c) {
        if (chan_rows[c] < 0) return fail(WF_EINVAL, "negative channel row count");
        total += chan_rows[c];
      }
      if (total != nrows) return fail(WF_EINVAL, "channel row counts do not sum to nrows");
    }
    const int64_t nvis = chan_rows ? nrows : nrows * (int64_t)nchan;
    for (int c = 0; c < nchan; ++c)
      if (!(freqs_hz[c] > 0) || !std::isfinite(freqs_hz[c]))
        return fail(WF_EINVAL, "frequencies must be positive");
    if (natural)
      for (int64_t k = 0; k < nvis; ++k)
        if (!std::isfinite(natural[k]) || natural[k] < 0.f)
          return fail(WF_EINVAL, "natural weights must be finite and non-negative");
    const double du = 1.0 / (shape.nx * shape.cell_rad);
    const double dv = 1.0 / (shape.ny * shape.cell_rad);
    double fmax = 0;
    for (int c = 0; c < nchan; ++c) fmax = std::max(fmax, freqs_hz[c]);
    // cell indices are formed as 64-bit integers: keep |u / du| far inside that range
    for (int64_t k = 0; k < nrows; ++k) {
      const double a = std::fabs(uvw_m[3 * k]) * fmax / C_LIGHT_MS / du;
      const double b = std::fabs(uvw_m[3 * k + 1]) * fmax / C_LIGHT_MS / dv;
      if (!(a < 1e15) || !(b < 1e15)) return fail(WF_EINVAL, "uvw coordinate out of range");
    }
    hipStream_t s = (hipStream_t)hip_stream;
    int64_t mmax = 0;
    for (int c = 0; c < nchan; ++c) mmax = std::max(mmax, chan_rows ? chan_rows[c] : nrows);
    if (mmax == 0) return WF_OK;
    Bufs B;
    wf_status st;
    const size_t ncell = (size_t)shape.nx * shape.ny;
    if ((st = dalloc(B.uvw, sizeof(double) * 3 * (chan_rows ? mmax : nrows))) != WF_OK) return st;
    if ((st = dalloc(B.W, sizeof(double) * ncell)) != WF_OK) return st;
    if ((st = dalloc(B.sums, 2 * sizeof(double))) != WF_OK) return st;
    if ((st = dalloc(B.out, sizeof(float) * mmax)) != WF_OK) return st;
    if (natural && (st = dalloc(B.w, sizeof(float) * mmax)) != WF_OK) return st;
    if (flags && (st = dalloc(B.flags, mmax)) != WF_OK) return st;
    int64_t off = 0, voff = 0;
    for (int c = 0; c < nchan; ++c) {
      const int64_t Mc = chan_rows ? chan_rows[c] : nrows;
      if (Mc > 0) {
        if (chan_rows || c == 0)
          WF_HIP(hipMemcpyAsync(B.uvw.p, uvw_m + 3 * off, sizeof(double) * 3 * Mc,
                                hipMemcpyHostToDevice, s));
        if (natural)
          WF_HIP(hipMemcpyAsync(B.w.p, natural + voff, sizeof(float) * Mc,
                                hipMemcpyHostToDevice, s));
        if (flags)
          WF_HIP(hipMemcpyAsync(B.flags.p, flags + voff, Mc, hipMemcpyHostToDevice, s));
        WF_HIP(hipMemsetAsync(B.W.p, 0, sizeof(double) * ncell, s));
        WF_HIP(hipMemsetAsync(B.sums.p, 0, 2 * sizeof(double), s));
        const double scale = freqs_hz[c] / C_LIGHT_MS;
        const float* dw = natural ? (const float*)B.w.p : nullptr;
        const uint8_t* df = flags ? (const uint8_t*)B.flags.p : nullptr;
        WF_HIP(launch_density((const double*)B.uvw.p, Mc, scale, du, dv, shape.nx, shape.ny,
                              dw, df, (double*)B.W.p, s));
        WF_HIP(launch_briggs_sums((const double*)B.uvw.p, Mc, scale, du, dv, shape.nx,
                                  shape.ny, dw, df, (const double*)B.W.p, (double*)B.sums.p,
                                  s));
        double sums[2] = {0, 0};
        WF_HIP(hipMemcpyAsync(sums, B.sums.p, sizeof(sums), hipMemcpyDeviceToHost, s));
        WF_HIP(hipStreamSynchronize(s));
        if (sums[0] > 0 && sums[1] > 0) {
          const double a = 5.0 * std::pow(10.0, -robust);
          const double f2 = a * a * sums[1] / sums[0];
          WF_HIP(launch_briggs_out((const double*)B.uvw.p, Mc, scale, du, dv, shape.nx,
                                   shape.ny, dw, df, (const double*)B.W.p, f2,
                                   (float*)B.out.p, s));
          WF_HIP(hipMemcpyAsync(out + voff, B.out.p, sizeof(float) * Mc,
                                hipMemcpyDeviceToHost, s));
          WF_HIP(hipStreamSynchronize(s));
        } else {
          std::memset(out + voff, 0, sizeof(float) * Mc);
        }
      }
      if (chan_rows) off += Mc;
      voff += Mc;
    }
    return WF_OK;
  } catch (const std::bad_alloc&) {
    return fail(WF_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(WF_EINVAL, e.what());
  }
}

extern "C" wf_status wf_briggs_weights_noalloc(const double* d_uvw_m, int64_t nrows,
                                               double freq_hz, wf_image_shape shape,
                                               double robust, const float* d_natural,
                                               const uint8_t* d_flags, float* d_out,
                                               void* hip_stream) {
  try {
    if (nrows < 0) return fail(WF_EINVAL, "negative row count");
    if (nrows > 0 && (!d_uvw_m || !d_out)) return fail(WF_EINVAL, "null uvw or output");
    if (shape.nx < 1 || shape.ny < 1 ||
        (int64_t)shape.nx * shape.ny > (int64_t)WF_BRIGGS_NOALLOC_MAX_CELLS)
      return fail(WF_EINVAL, "nx * ny must be in [1, " +
                                 std::to_string(WF_BRIGGS_NOALLOC_MAX_CELLS) + "]");
    if (!(shape.cell_rad > 0.0) || !std::isfinite(shape.cell_rad))
      return fail(WF_EINVAL, "cell must be positive");
    if (!std::isfinite(robust)) return fail(WF_EINVAL, "robustness must be finite");
    if (!(freq_hz > 0) || !std::isfinite(freq_hz)) return fail(WF_EINVAL, "frequency must be positive");
    if (nrows == 0) return WF_OK;
    double* W = nullptr;
    WF_HIP(briggs_scratch(&W));
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t ncell = (int64_t)shape.nx * shape.ny;
    double* sums = W + ncell;
    // density and sums start at zero (a fill kernel: the call may be captured in a graph)
    WF_HIP(launch_fill_zero(W, 2 * (ncell + 2), s));
    const double du = 1.0 / (shape.nx * shape.cell_rad);
    const double dv = 1.0 / (shape.ny * shape.cell_rad);
    const double scale = freq_hz / C_LIGHT_MS;
    WF_HIP(launch_density(d_uvw_m, nrows, scale, du, dv, shape.nx, shape.ny, d_natural, d_flags,
                          W, s));
    WF_HIP(launch_briggs_sums(d_uvw_m, nrows, scale, du, dv, shape.nx, shape.ny, d_natural,
                              d_flags, W, sums, s));
    const double a = 5.0 * std::pow(10.0, -robust);
    WF_HIP(launch_briggs_out_dev(d_uvw_m, nrows, scale, du, dv, shape.nx, shape.ny, d_natural,
                                 d_flags, W, sums, a * a, d_out, s));
    return WF_OK;
  } catch (const std::bad_alloc&) {
    return fail(WF_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(WF_EINVAL, e.what());
  }
}
