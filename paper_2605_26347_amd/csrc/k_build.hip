// Build of the de-gridding matrix G (workflow stages 2-3 of Sect. 3.5), FP64.
//
// Per visibility row k (one wavefront per row; one launch per class of residual-kernel
// side, whose LDS scratch is sized for that class):
//   * u, v, w in wavelengths = uvw_m * f / c; bin p = nearest w-bin centroid with ties to
//     the lower bin, i.e. the number of bin midpoints below w (Sect. 3.1 w-stacking);
//     residual w_proj = w - w_p;
//   * grid coordinates u_bar = u Kx cell, nearest cell r = floor(u_bar + 1/2);
//   * residual-w kernel (Sect. 3.1 w-projection, Fig. 1): side n_k from the chirp's
//     bandwidth over the padded field; the phase-tapered chirp is sampled on n_k x n_k
//     points over o times the field; a small DFT gives the kernel; the smallest entries
//     holding at most eps of the energy are dropped (a binary search over the energies'
//     bit patterns finds the cut; entries within 1e-9 relative of the smallest kept
//     energy are kept with it) and the kernel is cut to the smallest centred square;
//   * G row (Sect. 3.2): the kernel convolved with the 7 x 7 Kaiser-Bessel taps at the
//     row's fractional grid offset, a dense T x T patch, T = n' + J - 1.
// Decisions that turn floating point into integers (bin, nearest cell, n_k, threshold)
// use only correctly rounded FP64 operations, without contraction, so that they are
// reproducible by any IEEE implementation that performs the same operations.
#include <hip/hip_fp16.h>

#include <float.h>

#include <algorithm>

#include "mlp_defs.h"
#include "wf_internal.h"

namespace wf {

constexpr int MAXNK = 31;
constexpr int MAXT = 37;      // J - 1 + smax <= 37

constexpr int pow2_at_least(int v) {
  int p = 16;
  while (p < v) p <<= 1;
  return p;
}

// Columns of a G patch convolved per step by the large classes (their convolution
// intermediate holds n' x CB values).
constexpr int CB = 6;

// LDS scratch of one row for residual-kernel sides up to NK: the samples / kernel c and
// one region whose users never overlap in time.  Small classes (NK <= 15) keep the DFT
// intermediate t, the sort slots e and the full convolution intermediate t2 there.  The
// large classes, whose scratch limits how many rows are in flight, run the DFT sweeps in
// place (through registers) and convolve CB patch columns at a time, so the region only
// holds t2 for CB columns.  Rows are processed by kernel-side class
// (sides in (nk_lo<NK>, NK]), so that small kernels get a small scratch and many rows
// in flight per compute unit.
template <int NK>
struct KScratch {
  static constexpr bool BIG = NK > 15;
  static constexpr int TM = NK + 14 < MAXT ? NK + 14 : MAXT;  // patch side (J <= 15)
  static constexpr int NS = BIG ? 0 : pow2_at_least(NK * NK);  // sort slots
  static constexpr int UW = BIG ? 2 * NK * CB : (2 * NK * TM > NS ? 2 * NK * TM : NS);
  double2 c[NK * NK];                     // samples, then kernel
  alignas(16) double u[UW];               // small: t, e, t2; large: t2 of CB columns
  double2 roots[NK];                      // exp(-2 pi i m / nk)
  double ku[16], kv[16];                  // Kaiser-Bessel taps (J <= 15)
  __device__ double2* t() { return reinterpret_cast<double2*>(u); }
  __device__ double* e() { return u; }
  __device__ double2* t2() { return reinterpret_cast<double2*>(u); }
};

template <int NK>
constexpr int nk_lo() {
  return NK == 7 ? 0 : NK == 15 ? 7 : NK == 21 ? 15 : 21;
}
__host__ __device__ constexpr int class_of_nk(int nk) {
  return nk <= 7 ? 0 : nk <= 15 ? 1 : nk <= 21 ? 2 : 3;
}

// Workgroups of a launch over n listed rows (grid-stride beyond 2^18).
inline unsigned grid_for(int64_t n) { return (unsigned)(n < 262144 ? n : 262144); }



// 1 / k^2 for the I0 series (k < 128; the series has converged by k ~ 60 for the
// arguments of the Kaiser-Bessel taps, beta <= 2.34 * 15).
struct InvSquares {
  double v[128];
};
constexpr InvSquares make_inv_squares() {
  InvSquares t{};
  t.v[0] = 0.0;
  for (int k = 1; k < 128; ++k) t.v[k] = 1.0 / ((double)k * (double)k);
  return t;
}
__constant__ InvSquares c_inv_k2 = make_inv_squares();

// I0(x) = sum_k (x^2 / 4)^k / (k!)^2, the term ratio q / k^2 taken as q * (1 / k^2) so
// that the loop carries no division (the taps only scale values of G; no integer
// decision depends on them).
__device__ __forceinline__ double dev_i0(double x) {
#pragma clang fp contract(off)
  const double q = 0.25 * x * x;
  double term = 1.0, s = 1.0;
  for (int k = 1; k < 128; ++k) {
    term = term * (q * c_inv_k2.v[k]);
    s += term;
    if (term < 1e-18 * s) break;
  }
  return s;
}

__device__ __forceinline__ double dev_taper(double a_signed, double L) {
#pragma clang fp contract(off)
  const double a = fabs(a_signed);
  const double half = L / 2.0;
  if (a <= half) return 1.0;
  return 0.54 + 0.46 * cos(M_PI * (a - half) / half);
}

__device__ __forceinline__ int dev_nk(double wproj, const KernelParams& kp, bool capped) {
#pragma clang fp contract(off)
  if (wproj == 0.0) return 1;
  const double lp = ((double)kp.o * kp.Lx) / 2.0;
  const double mp = ((double)kp.o * kp.Ly) / 2.0;
  const double nn = sqrt(1.0 - lp * lp - mp * mp);
  const double aw = fabs(wproj);
  const double bx = 2.0 * ((aw * lp) / nn) * ((double)kp.o * kp.Lx);
  const double by = 2.0 * ((aw * mp) / nn) * ((double)kp.o * kp.Ly);
  const double B = bx > by ? bx : by;
  double nkd = 2.0 * ceil((kp.alpha * B) / 2.0) + 1.0;
  if (nkd > 1e6) nkd = 1e6;
  int nk = (int)nkd;
  if (capped && nk > kp.smax) nk = kp.smax;
  return nk;
}

struct RowGeom {
  double wproj, ub, vb;
  int p;
};

__device__ __forceinline__ RowGeom dev_geom(const double* __restrict__ uvw, int64_t k,
                                            double scale, double gsx, double gsy,
                                            const double* __restrict__ mids, int P,
                                            const double* __restrict__ cents) {
#pragma clang fp contract(off)
  RowGeom g;
  const double u = uvw[3 * k] * scale;
  const double v = uvw[3 * k + 1] * scale;
  const double w = uvw[3 * k + 2] * scale;
  int lo = 0, hi = P - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (mids[mid] < w) lo = mid + 1;
    else hi = mid;
  }
  g.p = lo;
  g.wproj = w - cents[lo];
  g.ub = u * gsx;
  g.vb = v * gsy;
  return g;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

template <int NK>
__device__ int wkernel_threshold(int nk, double eps, KScratch<NK>& S, double* dropped);

// Exact residual kernel of side nk with threshold; workgroup = one wavefront.
// Leaves the masked kernel in S.c (nk x nk, [s_v][s_u]); returns h' (kept half-side).
template <int NK>
__device__ int wkernel_row(double wproj, int nk, const KernelParams& kp, KScratch<NK>& S,
                           double* dropped) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x;
  const int nn2 = nk * nk;
  if (nk == 1) {
    if (lane == 0) S.c[0] = make_double2(1.0, 0.0);
    __syncthreads();
    *dropped = 0.0;
    return 0;
  }
  const int h = (nk - 1) / 2;
  for (int m = lane; m < nk; m += 64) {
    double s, c;
    sincospi((double)(-2 * m) / (double)nk, &s, &c);
    S.roots[m] = make_double2(c, s);
  }
  for (int idx = lane; idx < nn2; idx += 64) {
    const int b = idx / nk, a = idx - b * nk;
    const double lpa = ((double)(a - h) * kp.oLx) / (double)nk;
    const double mpb = ((double)(b - h) * kp.oLy) / (double)nk;
    const double L2 = lpa * lpa + mpb * mpb;
    const double n = sqrt(1.0 - L2);
    const double d = -L2 / (1.0 + n);
    const double tap = dev_taper(mpb, kp.Ly) * dev_taper(lpa, kp.Lx);
    const double ph = wproj * (d * tap);
    double s, c;
    sincospi(2.0 * ph, &s, &c);
    S.c[idx] = make_double2(c, -s);   // exp(-2 pi i ph)
  }
  __syncthreads();
  if constexpr (KScratch<NK>::BIG) {
    // t[b][su] = sum_a c[b][a] exp(-2 pi i (su-h)(a-h)/nk), in place: each lane holds its
    // outputs (entries lane + 64 q) in registers until every lane has read its inputs.
    // The root index (su-h)(a-h) mod nk advances by (su-h) mod nk per step of a.
    constexpr int PL = (NK * NK + 63) / 64;
    double2 acc[PL];
#pragma unroll
    for (int q = 0; q < PL; ++q) {
      const int idx = lane + 64 * q;
      if (idx >= nn2) continue;
      const int b = idx / nk, su = idx - b * nk;
      double re = 0.0, im = 0.0;
      const int step = (su - h + nk) % nk;
      int m = ((su - h) * (-h)) % nk;
      if (m < 0) m += nk;
#pragma unroll 4
      for (int a = 0; a < nk; ++a, m = (m + step >= nk ? m + step - nk : m + step)) {
        const double2 r = S.roots[m], x = S.c[b * nk + a];
        re += x.x * r.x - x.y * r.y;
        im += x.x * r.y + x.y * r.x;
      }
      acc[q] = make_double2(re, im);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PL; ++q)
      if (lane + 64 * q < nn2) S.c[lane + 64 * q] = acc[q];
    __syncthreads();
    const double inv = 1.0 / ((double)nk * (double)nk);
#pragma unroll
    for (int q = 0; q < PL; ++q) {
      const int idx = lane + 64 * q;
      if (idx >= nn2) continue;
      const int sv = idx / nk, su = idx - sv * nk;
      double re = 0.0, im = 0.0;
      const int step = (sv - h + nk) % nk;
      int m = ((sv - h) * (-h)) % nk;
      if (m < 0) m += nk;
#pragma unroll 4
      for (int b = 0; b < nk; ++b, m = (m + step >= nk ? m + step - nk : m + step)) {
        const double2 r = S.roots[m], x = S.c[b * nk + su];
        re += r.x * x.x - r.y * x.y;
        im += r.x * x.y + r.y * x.x;
      }
      acc[q] = make_double2(re * inv, im * inv);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PL; ++q)
      if (lane + 64 * q < nn2) S.c[lane + 64 * q] = acc[q];
    __syncthreads();
  } else {
    // t[b][su] = sum_a c[b][a] exp(-2 pi i (su-h)(a-h)/nk); the root index
    // (su-h)(a-h) mod nk advances by (su-h) mod nk per step of a
    for (int idx = lane; idx < nn2; idx += 64) {
      const int b = idx / nk, su = idx - b * nk;
      double re = 0.0, im = 0.0;
      const int step = (su - h + nk) % nk;
      int m = ((su - h) * (-h)) % nk;
      if (m < 0) m += nk;
#pragma unroll 4
      for (int a = 0; a < nk; ++a, m = (m + step >= nk ? m + step - nk : m + step)) {
        const double2 r = S.roots[m], x = S.c[b * nk + a];
        re += x.x * r.x - x.y * r.y;
        im += x.x * r.y + x.y * r.x;
      }
      S.t()[idx] = make_double2(re, im);
    }
    __syncthreads();
    const double inv = 1.0 / ((double)nk * (double)nk);
    for (int idx = lane; idx < nn2; idx += 64) {
      const int sv = idx / nk, su = idx - sv * nk;
      double re = 0.0, im = 0.0;
      const int step = (sv - h + nk) % nk;
      int m = ((sv - h) * (-h)) % nk;
      if (m < 0) m += nk;
#pragma unroll 4
      for (int b = 0; b < nk; ++b, m = (m + step >= nk ? m + step - nk : m + step)) {
        const double2 r = S.roots[m], x = S.t()[b * nk + su];
        re += r.x * x.x - r.y * x.y;
        im += r.x * x.y + r.y * x.x;
      }
      S.c[idx] = make_double2(re * inv, im * inv);
    }
    __syncthreads();
  }
  return wkernel_threshold(nk, kp.eps, S, dropped);
}

// Energy threshold of a kernel in S.c (nk x nk): drop the smallest entries holding at
// most eps of the energy (ties within 1e-9 relative of the smallest kept energy are
// kept), zero them in S.c, and return the half-side of the smallest centred square that
// holds every kept entry.  Workgroup = one wavefront.
//
// In ascending order the dropped entries are the longest prefix whose running sum stays
// at most eps * total, and tau, the smallest kept energy, is the entry after it (the
// largest entry when every prefix stays below).  Small kernels (n_k <= 15) sort their
// energies (a bitonic sort over at most 256 slots in LDS) and scan the prefix sums.
// Larger ones use the equivalent rule without sorting: with G(v) the sum of the energies
// <= v, tau is the smallest energy with G(tau) > eps * total; non-negative doubles order
// like their bit patterns, so a binary search over those patterns finds tau, with the
// energies in registers (lane l holds entries l + 64 q).
// Wave sum of a double, identical in every lane: DPP steps inside each row of 16 lanes
// (quad xor 1, quad xor 2, half-row mirror, row mirror) on both 32-bit halves, then the
// four row sums read back in a fixed order.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_d<0xb1>(v);
  v += dpp_d<0x4e>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  auto row = [&](int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
  };
  return (row(0) + row(16)) + (row(32) + row(48));
}

__device__ __forceinline__ double wave_min_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

template <int NK>
__device__ int wkernel_threshold(int nk, double eps, KScratch<NK>& S, double* dropped) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x;
  const int nn2 = nk * nk;
  const int h = (nk - 1) / 2;
  double tau, tot;
  if constexpr (NK <= 15) {
    // energies, ascending bitonic sort over NS slots (NS = next power of two >= nk^2,
    // +inf padding)
    int NS = 16;
    while (NS < nn2) NS <<= 1;
    for (int i = lane; i < NS; i += 64) {
      if (i < nn2) {
        const double2 v = S.c[i];
        S.e()[i] = v.x * v.x + v.y * v.y;
      } else {
        S.e()[i] = DBL_MAX;
      }
    }
    __syncthreads();
    for (int k = 2; k <= NS; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = lane; i < NS; i += 64) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const bool up = (i & k) == 0;
            const double a = S.e()[i], b = S.e()[ixj];
            if ((a > b) == up) {
              S.e()[i] = b;
              S.e()[ixj] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    // inclusive prefix sums: lane holds slots pl*lane .. pl*lane + pl - 1
    constexpr int PLMAX = KScratch<NK>::NS >= 64 ? KScratch<NK>::NS / 64 : 1;
    const int pl = NS >= 64 ? NS / 64 : 1;
    double loc[PLMAX];
    double run = 0.0;
#pragma unroll
    for (int q = 0; q < PLMAX; ++q) {
      const int i = pl * lane + q;
      const double v = (q < pl && i < nn2) ? S.e()[i] : 0.0;
      run += v;
      loc[q] = run;
    }
    double scan = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double y = __shfl_up(scan, o, 64);
      if (lane >= o) scan += y;
    }
    const double offs = scan - run;
    tot = __shfl(scan, 63, 64);
    const double thr = eps * tot;
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < PLMAX; ++q) {
      const int i = pl * lane + q;
      if (q < pl && i < nn2 && offs + loc[q] <= thr) ++cnt;
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    int jdrop = cnt < nn2 - 1 ? cnt : nn2 - 1;
    tau = S.e()[jdrop];
  } else {
    constexpr int PL = (NK * NK + 63) / 64;
    double en[PL];
    double run = 0.0;
#pragma unroll
    for (int q = 0; q < PL; ++q) {
      const int i = lane + 64 * q;
      double v = 0.0;   // slots beyond nn2 hold no entry (0 adds nothing, is never tau)
      if (i < nn2) {
        const double2 c = S.c[i];
        v = c.x * c.x + c.y * c.y;
      }
      en[q] = v;
      run += v;
    }
    tot = wave_sum_d(run);
    const double thr = eps * tot;
    // largest bit pattern lo with G(lo) <= thr; G(0) = 0 <= thr always
    uint64_t lo = 0, hi = 1ull << 63;
    while (hi - lo > 1) {
      const uint64_t mid = lo + ((hi - lo) >> 1);
      double g = 0.0;
#pragma unroll
      for (int q = 0; q < PL; ++q)
        if ((uint64_t)__double_as_longlong(en[q]) <= mid) g += en[q];
      g = wave_sum_dpp(g);   // identical in every lane: the branch is wave-uniform
      if (g <= thr) lo = mid;
      else hi = mid;
    }
    double tmin = DBL_MAX, tmax = 0.0;
#pragma unroll
    for (int q = 0; q < PL; ++q) {
      if (lane + 64 * q >= nn2) continue;
      if ((uint64_t)__double_as_longlong(en[q]) >= hi) tmin = en[q] < tmin ? en[q] : tmin;
      tmax = en[q] > tmax ? en[q] : tmax;
    }
    tmin = wave_min_d(tmin);
    tmax = wave_max_d(tmax);
    tau = tmin < DBL_MAX ? tmin : tmax;
  }
  const double cut = tau * (1.0 - 1e-9);
  int hp = 0;
  double dsum = 0.0;
  for (int idx = lane; idx < nn2; idx += 64) {
    const double2 v = S.c[idx];
    const double E = v.x * v.x + v.y * v.y;
    if (E >= cut) {
      const int sv = idx / nk, su = idx - sv * nk;
      const int rv = sv > h ? sv - h : h - sv;
      const int ru = su > h ? su - h : h - su;
      const int r = rv > ru ? rv : ru;
      hp = r > hp ? r : hp;
    } else {
      dsum += E;
      S.c[idx] = make_double2(0.0, 0.0);
    }
  }
  hp = wave_max_i(hp);
  dsum = wave_sum_d(dsum);
  *dropped = tot > 0.0 ? dsum / tot : 0.0;
  __syncthreads();
  return hp;
}

// Rows whose kernel comes from the network: side at most the prediction window and the
// cap, not a plain delta, and a predicted log10 error at most logtol.
__device__ __forceinline__ bool use_prediction(const float* pr, int nk_full,
                                               const KernelParams& kp, float logtol) {
  return pr && nk_full > 1 && nk_full <= MLP_SIDE && nk_full <= kp.smax &&
         pr[MLP_KOUT] <= logtol;
}

// Kernel of side nk from the network's prediction: the centre nk x nk of the predicted
// window, cut to the smallest centred square whose outside holds at most eps of the
// energy (whole square rings are dropped; no sort, unlike the exact kernel's per-entry
// threshold, whose zeroed entries the network has learned as near-zero outputs).
template <int NK>
__device__ int predicted_kernel(const float* pr, int nk, const KernelParams& kp, KScratch<NK>& S,
                                double* dropped) {
#pragma clang fp contract(off)
  const int a = (MLP_SIDE - nk) / 2;
  const int h = (nk - 1) / 2;
  double ring[MLP_SIDE / 2 + 1];
#pragma unroll
  for (int r = 0; r <= MLP_SIDE / 2; ++r) ring[r] = 0.0;
  for (int idx = threadIdx.x; idx < nk * nk; idx += 64) {
    const int sv = idx / nk, su = idx - sv * nk;
    const int j = (sv + a) * MLP_SIDE + (su + a);
    const double re = (double)pr[2 * j], im = (double)pr[2 * j + 1];
    S.c[idx] = make_double2(re, im);
    const int rv = sv > h ? sv - h : h - sv;
    const int ru = su > h ? su - h : h - su;
    const int r = rv > ru ? rv : ru;
    const double e = re * re + im * im;
#pragma unroll
    for (int q = 0; q <= MLP_SIDE / 2; ++q)
      if (q == r) ring[q] += e;
  }
  double tot = 0.0;
#pragma unroll
  for (int q = 0; q <= MLP_SIDE / 2; ++q) {
    ring[q] = wave_sum_d(ring[q]);
    tot += ring[q];
  }
  int hp = h;
  double outside = 0.0;
  for (int q = h; q > 0; --q) {
    if (outside + ring[q] > kp.eps * tot) break;
    outside += ring[q];
    hp = q - 1;
  }
  *dropped = tot > 0.0 ? outside / tot : 0.0;
  __syncthreads();
  return hp;
}

template <int NK>
__global__ __launch_bounds__(64, NK <= 15 ? 4 : 1) void k_rowsym(const double* __restrict__ uvw, int64_t r0,
                                               const int32_t* __restrict__ rows, int64_t nl,
                                               double scale, double gsx,
                                               double gsy, const double* __restrict__ mids,
                                               int P, const double* __restrict__ cents, int Kx,
                                               int Ky, int tile, KernelParams kp,
                                               uint64_t* __restrict__ keys,
                                               float* __restrict__ dropped_out, Surrogate sg) {
#pragma clang fp contract(off)
  __shared__ KScratch<NK> S;
  for (int64_t i = blockIdx.x; i < nl; i += gridDim.x) {
    const int64_t k = rows[i];
    const RowGeom g = dev_geom(uvw, k, scale, gsx, gsy, mids, P, cents);
    const int nk_full = dev_nk(g.wproj, kp, false);
    const int nk = nk_full > kp.smax ? kp.smax : nk_full;
    if (nk > NK || nk <= nk_lo<NK>()) {   // class byte disagrees: mark the key invalid
      if (threadIdx.x == 0) keys[k] = ~0ull;
      continue;
    }
    double dropped;
    const float* pr = sg.pred ? sg.pred + (sg.by_slot ? i : k - r0) * MLP_OUT : nullptr;
    const bool usep = use_prediction(pr, nk_full, kp, sg.logtol);
    const int hp = usep ? predicted_kernel(pr, nk, kp, S, &dropped)
                        : wkernel_row(g.wproj, nk, kp, S, &dropped);
    if (usep && threadIdx.x == 0 && sg.used) atomicAdd(sg.used, 1);
    if (threadIdx.x == 0) {
      const int T = 2 * hp + 1 + kp.J - 1;
      const int64_t ru = (int64_t)floor(g.ub + 0.5);
      const int64_t rv = (int64_t)floor(g.vb + 0.5);
      const int64_t rum = ((ru % Kx) + Kx) % Kx;
      const int64_t rvm = ((rv % Ky) + Ky) % Ky;
      const uint64_t tu = (uint64_t)(rum / tile), lu = (uint64_t)(rum % tile);
      const uint64_t tv = (uint64_t)(rvm / tile), lv = (uint64_t)(rvm % tile);
      keys[k] = row_key(g.p, T, (uint32_t)tv, (uint32_t)tu, (uint32_t)lv, (uint32_t)lu);
      const float df = (float)dropped;
      dropped_out[k] = (nk_full > kp.smax) ? -df - 1e-30f : df;
    }
    __syncthreads();
  }
}

template <int STORE>
__device__ __forceinline__ void store_val(void* vals, int64_t i, double re, double im) {
  if constexpr (STORE == WF_STORE_F32) {
    reinterpret_cast<float2*>(vals)[i] = make_float2((float)re, (float)im);
  } else if constexpr (STORE == WF_STORE_F16) {
    reinterpret_cast<__half2*>(vals)[i] = __floats2half2_rn((float)re, (float)im);
  } else {
    // round-to-nearest-even FP32 -> BF16 (finite inputs)
    auto bf = [](float f) -> uint32_t {
      const uint32_t b = __float_as_uint(f);
      return (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
    };
    reinterpret_cast<uint32_t*>(vals)[i] = bf((float)re) | (bf((float)im) << 16);
  }
}

template <int STORE, int NK>
__global__ __launch_bounds__(64, NK <= 15 ? 4 : 1) void k_gbuild(const double* __restrict__ uvw, int64_t s0,
                                               const int32_t* __restrict__ rows, int64_t nl,
                                               const int32_t* __restrict__ perm,
                                               const uint32_t* __restrict__ meta,
                                               const uint32_t* __restrict__ voff,
                                               const int32_t* __restrict__ row_wi,
                                               const WorkItem* __restrict__ wis, double scale,
                                               double gsx, double gsy,
                                               const double* __restrict__ mids, int P,
                                               const double* __restrict__ cents,
                                               KernelParams kp, void* __restrict__ vals,
                                               int64_t vbase, int* __restrict__ mismatch,
                                               Surrogate sg, const float* __restrict__ wts) {
#pragma clang fp contract(off)
  __shared__ KScratch<NK> S;
  const int lane = threadIdx.x;
  const int half = (kp.J - 1) / 2;
  for (int64_t i = blockIdx.x; i < nl; i += gridDim.x) {
    const int64_t s = rows[i];
    const int64_t k = perm[s];
    const RowGeom g = dev_geom(uvw, k, scale, gsx, gsy, mids, P, cents);
    const int nk_full = dev_nk(g.wproj, kp, false);
    const int nk = nk_full > kp.smax ? kp.smax : nk_full;
    if (nk > NK || nk <= nk_lo<NK>()) {   // class byte disagrees: count it, build nothing
      if (lane == 0) atomicAdd(mismatch, 1);
      continue;
    }
    double dropped;
    const float* pr = sg.pred ? sg.pred + (sg.by_slot ? i : s - s0) * MLP_OUT : nullptr;
    const bool usep = use_prediction(pr, nk_full, kp, sg.logtol);
    const int hp = usep ? predicted_kernel(pr, nk, kp, S, &dropped)
                        : wkernel_row(g.wproj, nk, kp, S, &dropped);
    const int h = (nk - 1) / 2;
    const int np = 2 * hp + 1;
    const int T = np + kp.J - 1;
    const int Tm = (int)((meta[s] >> 16) & 0xff);
    // Kaiser-Bessel taps phi(f - d), d = -half..half
    const double fu = g.ub - floor(g.ub + 0.5);
    const double fv = g.vb - floor(g.vb + 0.5);
    if (lane < 2 * kp.J) {
      const int d = (lane % kp.J) - half;
      const double f = lane < kp.J ? fu : fv;
      const double t = f - (double)d;
      const double z = 1.0 - ((2.0 * t) / (double)kp.J) * ((2.0 * t) / (double)kp.J);
      const double val = z >= 0.0 ? dev_i0(kp.beta * sqrt(z)) / kp.i0beta : 0.0;
      if (lane < kp.J) S.ku[lane % kp.J] = val;
      else S.kv[lane % kp.J] = val;
    }
    __syncthreads();
    const int64_t vb = wis[row_wi[s]].voff + voff[s] - vbase;
    const double wk = wts ? (double)wts[k] : 1.0;   // data weight of the row
    bool over = false;
    if constexpr (KScratch<NK>::BIG) {
      // CB patch columns at a time: t2[m][c] = sum_n kern[m][n] ku[au - n] (au = au0 + c,
      // kern = kept centre square of S.c), then G[av][au] = sum_m kv[av - m] t2[m][c]
      for (int au0 = 0; au0 < T; au0 += CB) {
        const int cw = T - au0 < CB ? T - au0 : CB;
        for (int idx = lane; idx < np * cw; idx += 64) {
          const int m = idx / cw, cc = idx - m * cw, au = au0 + cc;
          double re = 0.0, im = 0.0;
          for (int nn = 0; nn < np; ++nn) {
            const int dd = au - nn;
            if (dd >= 0 && dd < kp.J) {
              const double2 c = S.c[(m + h - hp) * nk + (nn + h - hp)];
              re += c.x * S.ku[dd];
              im += c.y * S.ku[dd];
            }
          }
          S.t2()[m * CB + cc] = make_double2(re, im);
        }
        __syncthreads();
        if (T == Tm) {
          for (int idx = lane; idx < T * cw; idx += 64) {
            const int av = idx / cw, cc = idx - av * cw, au = au0 + cc;
            double re = 0.0, im = 0.0;
            for (int m = 0; m < np; ++m) {
              const int dd = av - m;
              if (dd >= 0 && dd < kp.J) {
                const double2 x = S.t2()[m * CB + cc];
                re += S.kv[dd] * x.x;
                im += S.kv[dd] * x.y;
              }
            }
            re *= wk;
            im *= wk;
            if constexpr (STORE == WF_STORE_F16)
              over = over || fabs(re) > 65504.0 || fabs(im) > 65504.0;
            store_val<STORE>(vals, vb + av * T + au, re, im);
          }
        }
        __syncthreads();
      }
      if (T != Tm && lane == 0) atomicAdd(mismatch, 1);
    } else {
      // t2[m][au] = sum_n kern[m][n] ku[au - n], kern = kept centre square of S.c
      for (int idx = lane; idx < np * T; idx += 64) {
        const int m = idx / T, au = idx - m * T;
        double re = 0.0, im = 0.0;
        for (int nn = 0; nn < np; ++nn) {
          const int dd = au - nn;
          if (dd >= 0 && dd < kp.J) {
            const double2 c = S.c[(m + h - hp) * nk + (nn + h - hp)];
            re += c.x * S.ku[dd];
            im += c.y * S.ku[dd];
          }
        }
        S.t2()[idx] = make_double2(re, im);
      }
      __syncthreads();
      if (T == Tm) {
        for (int idx = lane; idx < T * T; idx += 64) {
          const int av = idx / T, au = idx - av * T;
          double re = 0.0, im = 0.0;
          for (int m = 0; m < np; ++m) {
            const int dd = av - m;
            if (dd >= 0 && dd < kp.J) {
              const double2 x = S.t2()[m * T + au];
              re += S.kv[dd] * x.x;
              im += S.kv[dd] * x.y;
            }
          }
          re *= wk;
          im *= wk;
          if constexpr (STORE == WF_STORE_F16) over = over || fabs(re) > 65504.0 || fabs(im) > 65504.0;
          store_val<STORE>(vals, vb + idx, re, im);
        }
      } else if (lane == 0) {
        atomicAdd(mismatch, 1);
      }
    }
    if (over) atomicAdd(mismatch + 1, 1);
    __syncthreads();
  }
}

// Factorised strategy (c), build side: the thresholded residual kernel of each listed
// row (the kept n' x n' centre of c_hat_k, Sect. 3.1), times the row's data weight,
// written in the value format at khat[kabs[s] ..] ([s_v][s_u], row-major).  The kernel
// is built and checked exactly as by k_gbuild; the Kaiser-Bessel convolution is left
// to every apply (k_expand).
template <int STORE, int NK>
__global__ __launch_bounds__(64, NK <= 15 ? 4 : 1) void k_khat(const double* __restrict__ uvw, int64_t s0,
                                               const int32_t* __restrict__ rows, int64_t nl,
                                               const int32_t* __restrict__ perm,
                                               const uint32_t* __restrict__ meta,
                                               const int64_t* __restrict__ kabs, double scale,
                                               double gsx, double gsy,
                                               const double* __restrict__ mids, int P,
                                               const double* __restrict__ cents,
                                               KernelParams kp, void* __restrict__ khat,
                                               float* __restrict__ taps,
                                               int* __restrict__ mismatch, Surrogate sg,
                                               const float* __restrict__ wts) {
#pragma clang fp contract(off)
  __shared__ KScratch<NK> S;
  const int lane = threadIdx.x;
  const int half = (kp.J - 1) / 2;
  for (int64_t i = blockIdx.x; i < nl; i += gridDim.x) {
    const int64_t s = rows[i];
    const int64_t k = perm[s];
    const RowGeom g = dev_geom(uvw, k, scale, gsx, gsy, mids, P, cents);
    const int nk_full = dev_nk(g.wproj, kp, false);
    const int nk = nk_full > kp.smax ? kp.smax : nk_full;
    if (nk > NK || nk <= nk_lo<NK>()) {
      if (lane == 0) atomicAdd(mismatch, 1);
      continue;
    }
    double dropped;
    const float* pr = sg.pred ? sg.pred + (sg.by_slot ? i : s - s0) * MLP_OUT : nullptr;
    const bool usep = use_prediction(pr, nk_full, kp, sg.logtol);
    const int hp = usep ? predicted_kernel(pr, nk, kp, S, &dropped)
                        : wkernel_row(g.wproj, nk, kp, S, &dropped);
    const int h = (nk - 1) / 2;
    const int np = 2 * hp + 1;
    if (np + kp.J - 1 != (int)((meta[s] >> 16) & 0xff)) {
      if (lane == 0) atomicAdd(mismatch, 1);
    } else {
      const double wk = wts ? (double)wts[k] : 1.0;
      const int64_t kb = kabs[s];
      for (int idx = lane; idx < np * np; idx += 64) {
        const int m = idx / np, nn = idx - m * np;
        const double2 c = S.c[(m + h - hp) * nk + (nn + h - hp)];
        store_val<STORE>(khat, kb + idx, c.x * wk, c.y * wk);
      }
      // the row's Kaiser-Bessel taps phi(f - d), d = -half..half, as k_gbuild evaluates
      // them (FP64), rounded to FP32: u taps then v taps
      if (lane < 2 * kp.J) {
        const int d = (lane % kp.J) - half;
        const double f = lane < kp.J ? g.ub - floor(g.ub + 0.5) : g.vb - floor(g.vb + 0.5);
        const double t = f - (double)d;
        const double z = 1.0 - ((2.0 * t) / (double)kp.J) * ((2.0 * t) / (double)kp.J);
        taps[s * 2 * kp.J + lane] = z >= 0.0 ? (float)(dev_i0(kp.beta * sqrt(z)) / kp.i0beta) : 0.f;
      }
    }
    __syncthreads();
  }
}

template <int STORE>
__device__ __forceinline__ float2 load_val(const void* __restrict__ v, int64_t i) {
  if constexpr (STORE == WF_STORE_F32) {
    return reinterpret_cast<const float2*>(v)[i];
  } else if constexpr (STORE == WF_STORE_F16) {
    return __half22float2(reinterpret_cast<const __half2*>(v)[i]);
  } else {
    const uint32_t b = reinterpret_cast<const uint32_t*>(v)[i];
    return make_float2(__uint_as_float(b << 16), __uint_as_float(b & 0xffff0000u));
  }
}

// Factorised strategy (c), apply side: rows of G from the stored kernels,
// G = Kv c Ku^T (Sect. 3.2), Ku / Kv the banded matrices of the Kaiser-Bessel taps at the
// row's fractional grid offset.  The taps were evaluated by the build in FP64 (the
// uvw -> grid map) and stored in FP32, 2J per row (u then v, taps[s 2J ..]); the
// convolution is FP32; values are written in the store format where the value pass
// would write them (item offset + row offset - vbase).
//
// A workgroup is one wavefront and takes rpw <= 64 listed rows at a time (fewer where a
// launch has few rows, so that every SIMD still holds several wavefronts): lane i reads
// the i-th row's words and taps.  The rows are then expanded SL at a time,
// one per slot of TM = NK + JT - 1 lanes (the largest patch side of the class), lane a_u
// of a slot computing patch column a_u: first t[m] = sum_d ku[d] c[m][a_u - d] for the
// kernel rows m (c staged in LDS), then G[a_v][a_u] = sum_d kv[d] t[a_v - d] in registers,
// so that the lanes of a slot write each patch row with consecutive values.  Loops run
// to the largest n' and T among the wavefront's slots.  The next rows' kernels are
// loaded while the current ones are expanded.  JT >= J taps are carried (zero past J).
// over counts values beyond the FP16 range (FP16 store only).
template <int NK, int JT>
struct EScratch {
  static constexpr int NN = NK * NK;
  static constexpr int TM = NK + JT - 1;
  static constexpr int SL = 64 / TM;                   // rows expanded side by side
  static constexpr int CK = (SL * NN + 63) / 64;       // kernel cells per lane and step
  static constexpr int PW = NK + 2 * (JT - 1);         // padded kernel row
  static constexpr int PS = NK * PW;                   // padded kernel of one slot
  // the step's kernels, [slot][s_v][JT - 1 + s_u]: an NK x NK interior (the n' x n'
  // kernel, zero beyond it) between zero margins of JT - 1 cells, so that the taps'
  // reads need no bounds checks
  float2 c[SL * PS];
};

// Raw stored value: two 32-bit words (FP32) or one word of two 16-bit halves.
template <int STORE>
struct KRaw {
  using type = uint32_t;
};
template <>
struct KRaw<WF_STORE_F32> {
  using type = uint2;
};
template <int STORE>
__device__ __forceinline__ typename KRaw<STORE>::type kraw_load(const void* __restrict__ v,
                                                                int64_t i) {
  if constexpr (STORE == WF_STORE_F32) return reinterpret_cast<const uint2*>(v)[i];
  else return reinterpret_cast<const uint32_t*>(v)[i];
}
template <int STORE>
__device__ __forceinline__ float2 kraw_widen(typename KRaw<STORE>::type r) {
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

// Orders one wavefront's LDS accesses: its LDS operations complete in order, so a
// workgroup of one wavefront needs only that the compiler keep them in program order.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_max_u(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return __builtin_amdgcn_readfirstlane(v);
}

template <int STORE, int NK, int JT>
__global__ __launch_bounds__(64) void k_expand(const int32_t* __restrict__ rows, int64_t nl,
                                               const uint32_t* __restrict__ meta,
                                               const uint32_t* __restrict__ voff,
                                               const int32_t* __restrict__ row_wi,
                                               const WorkItem* __restrict__ wis,
                                               KernelParams kp, const void* __restrict__ khat,
                                               const uint32_t* __restrict__ kof,
                                               const float* __restrict__ taps,
                                               void* __restrict__ vals, int64_t vbase,
                                               int rpw, int* __restrict__ over) {
#pragma clang fp contract(off)
  using ES = EScratch<NK, JT>;
  using Raw = typename KRaw<STORE>::type;
  constexpr int NN = ES::NN, TM = ES::TM, SL = ES::SL, CK = ES::CK, PW = ES::PW, PS = ES::PS;
  __shared__ ES S;
  const int lane = threadIdx.x;
  const int slot = lane / TM, au = lane - slot * TM;   // slot == SL: spare lanes
  bool ovf = false;
  for (int64_t b0 = (int64_t)blockIdx.x * rpw; b0 < nl; b0 += (int64_t)gridDim.x * rpw) {
    const int nb = (int)(nl - b0 < rpw ? nl - b0 : rpw);
    // lane i: row b0 + i's patch side, kernel and value offsets, and taps
    int myT = 0;
    uint32_t mykof = 0;
    int64_t myvb = 0;
    float myku[JT], mykv[JT];
#pragma unroll
    for (int d = 0; d < JT; ++d) myku[d] = mykv[d] = 0.f;
    if (lane < nb) {
      const int64_t s = rows[b0 + lane];
      myT = (int)((meta[s] >> 16) & 0xff);
      mykof = kof[s];
      myvb = wis[row_wi[s]].voff + voff[s] - vbase;
      const float* tp = taps + s * 2 * kp.J;
#pragma unroll
      for (int d = 0; d < JT; ++d) {
        if (d < kp.J) {
          myku[d] = tp[d];
          mykv[d] = tp[kp.J + d];
        }
      }
    }
    const int vlo = (int)(uint32_t)(uint64_t)myvb, vhi = (int)(uint32_t)((uint64_t)myvb >> 32);
    // the SL kernels of the step at rb: every interior cell (slot j, row m, column n) of
    // the step is handled by lane (cell % 64), which loads the kernel value there (zero
    // outside the slot's n' x n' kernel) into registers; the cells are then written to
    // LDS.  Slot j's kernel side and offset are wave-uniform.
    Raw cb[CK];
    struct Step {
      int np[SL];
      uint32_t ko[SL];
    };
    auto step_of = [&](int rb) {
      Step st;
#pragma unroll
      for (int j = 0; j < SL; ++j) {
        const int r = rb + j;
        st.np[j] = r < nb ? __builtin_amdgcn_readlane(myT, r & 63) - kp.J + 1 : 0;
        st.ko[j] = r < nb ? (uint32_t)__builtin_amdgcn_readlane((int)mykof, r & 63) : 0u;
      }
      return st;
    };
    // cell i of the step: slot j, kernel row m, column n; its kernel index when inside
    auto cell = [&](const Step& st, int i, int& j, int& m, int& n, int& np, uint32_t& ko) {
      j = i / NN;
      const int e = i - j * NN;
      m = e / NK;
      n = e - m * NK;
      np = st.np[0];
      ko = st.ko[0];
#pragma unroll
      for (int q = 1; q < SL; ++q)
        if (j == q) {
          np = st.np[q];
          ko = st.ko[q];
        }
    };
    auto issue = [&](int rb) {
      const Step st = step_of(rb);
#pragma unroll
      for (int q = 0; q < CK; ++q) {
        const int i = lane + 64 * q;
        int j, m, n, np;
        uint32_t ko;
        cell(st, i, j, m, n, np, ko);
        if (i < SL * NN && m < np && n < np)
          cb[q] = kraw_load<STORE>(khat, (int64_t)ko + m * np + n);
      }
    };
    auto stage = [&](int rb) {
      const Step st = step_of(rb);
#pragma unroll
      for (int q = 0; q < CK; ++q) {
        const int i = lane + 64 * q;
        int j, m, n, np;
        uint32_t ko;
        cell(st, i, j, m, n, np, ko);
        if (i < SL * NN)
          S.c[j * PS + m * PW + (JT - 1) + n] =
              (m < np && n < np) ? kraw_widen<STORE>(cb[q]) : make_float2(0.f, 0.f);
      }
    };
    // the margins stay zero
    for (int i = lane; i < SL * NK * 2 * (JT - 1); i += 64) {
      const int row = i / (2 * (JT - 1)), e = i - row * (2 * (JT - 1));
      S.c[row * PW + (e < JT - 1 ? e : NK + e)] = make_float2(0.f, 0.f);
    }
    issue(0);
    for (int rb = 0; rb < nb; rb += SL) {
      stage(rb);
      wave_lds_sync();
      if (rb + SL < nb) issue(rb + SL);
      // this lane's row (slot) and its words and taps.  Every lane takes part in the
      // cross-lane reads (a lane left out would read nothing to its peers).
      const int r = rb + slot;
      const bool valid = slot < SL && r < nb;
      const int src = valid ? r : 0;
      const int Tsrc = __shfl(myT, src, 64);
      const int T = valid ? Tsrc : 0;
      const int np = valid ? T - kp.J + 1 : 0;
      const int64_t vb = (int64_t)(((uint64_t)(uint32_t)__shfl(vhi, src, 64) << 32) |
                                   (uint64_t)(uint32_t)__shfl(vlo, src, 64));
      float ku[JT], kv[JT];
#pragma unroll
      for (int d = 0; d < JT; ++d) {
        ku[d] = __shfl(myku[d], src, 64);
        kv[d] = __shfl(mykv[d], src, 64);
      }
      const int npmax = wave_max_u(np), Tmax = wave_max_u(T);
      // t[m] = sum_d ku[d] c[m][a_u - d]: reads at a_u - d + JT - 1 in [0, PW) (a_u < TM)
      const float2* c = S.c + (slot < SL ? slot : 0) * PS + au;
      float2 t[NK];
#pragma unroll
      for (int m = 0; m < NK; ++m) {
        t[m] = make_float2(0.f, 0.f);
        if (m < npmax) {
          float re = 0.f, im = 0.f;
#pragma unroll
          for (int d = 0; d < JT; ++d) {
            const float2 v = c[m * PW + (JT - 1 - d)];
            re = fmaf(ku[d], v.x, re);
            im = fmaf(ku[d], v.y, im);
          }
          t[m] = make_float2(re, im);
        }
      }
      // G[a_v][a_u] = sum_d kv[d] t[a_v - d]
      const bool col = valid && au < T;
#pragma unroll
      for (int av = 0; av < TM; ++av) {
        if (av < Tmax) {
          float re = 0.f, im = 0.f;
#pragma unroll
          for (int d = 0; d < JT; ++d) {
            if (av - d >= 0 && av - d < NK) {
              re = fmaf(kv[d], t[av - d].x, re);
              im = fmaf(kv[d], t[av - d].y, im);
            }
          }
          if (col && av < T) {
            if constexpr (STORE == WF_STORE_F16)
              ovf = ovf || fabsf(re) > 65504.f || fabsf(im) > 65504.f;
            store_val<STORE>(vals, vb + (int64_t)av * T + au, (double)re, (double)im);
          }
        }
      }
      wave_lds_sync();   // every read of the step's kernels is done before the next staging
    }
  }
  if (ovf) atomicAdd(over, 1);
}

// Kernel-side class (0: n_k <= 7, 1: <= 15, 2: <= 21, 3: <= 31) of rows [r0, r1) in
// caller order; the same bin and side computation as the build kernels.
__global__ __launch_bounds__(256) void k_row_class(const double* __restrict__ uvw, int64_t r0,
                                                   int64_t r1, double scale, double gsx,
                                                   double gsy, const double* __restrict__ mids,
                                                   int P, const double* __restrict__ cents,
                                                   KernelParams kp, uint8_t* __restrict__ cls) {
#pragma clang fp contract(off)
  for (int64_t k = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < r1;
       k += (int64_t)gridDim.x * blockDim.x) {
    const RowGeom g = dev_geom(uvw, k, scale, gsx, gsy, mids, P, cents);
    const int nk_full = dev_nk(g.wproj, kp, false);
    cls[k] = (uint8_t)class_of_nk(nk_full > kp.smax ? kp.smax : nk_full);
  }
}

// Network inputs of rows [r0, r0 + nr) in caller order (perm null) or of sorted rows
// perm[r0 ..] (field side L, square field).
__global__ __launch_bounds__(256) void k_row_inputs(const double* __restrict__ uvw,
                                                    const int32_t* __restrict__ list,
                                                    const int32_t* __restrict__ perm, int64_t r0,
                                                    int64_t nr, double scale, double gsx,
                                                    double gsy, const double* __restrict__ mids,
                                                    int P, const double* __restrict__ cents,
                                                    KernelParams kp, double L,
                                                    float* __restrict__ x) {
#pragma clang fp contract(off)
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = list ? (int64_t)list[r0 + i] : r0 + i;
    const int64_t k = perm ? (int64_t)perm[s] : s;
    const RowGeom g = dev_geom(uvw, k, scale, gsx, gsy, mids, P, cents);
    const int nk_full = dev_nk(g.wproj, kp, false);
    const double fu = g.ub - floor(g.ub + 0.5);
    const double fv = g.vb - floor(g.vb + 0.5);
    mlp_inputs(g.wproj, L, kp.o, fu, fv, nk_full, x + i * MLP_IN);
  }
}

__device__ __forceinline__ KernelParams with_field(KernelParams kp, double L) {
  kp.Lx = L;
  kp.Ly = L;
  kp.oLx = (double)kp.o * L;
  kp.oLy = (double)kp.o * L;
  return kp;
}

// Training inputs of examples (w_proj, field side L, cell offsets).
__global__ __launch_bounds__(256) void k_train_inputs(const double* __restrict__ w,
                                                      const double* __restrict__ L,
                                                      const double* __restrict__ fu,
                                                      const double* __restrict__ fv, int64_t n,
                                                      KernelParams kp, float* __restrict__ x,
                                                      int32_t* __restrict__ nk_out) {
#pragma clang fp contract(off)
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const KernelParams q = with_field(kp, L[i]);
    const int nk = dev_nk(w[i], q, false);
    mlp_inputs(w[i], L[i], q.o, fu[i], fv[i], nk, x + i * MLP_IN);
    if (nk_out) nk_out[i] = nk;
  }
}

// Training targets: the thresholded exact kernel of each example centred in the 15 x 15
// window (zeros when its side exceeds 15).  One wavefront per example.
__global__ __launch_bounds__(64) void k_exact_targets(const double* __restrict__ w,
                                                      const double* __restrict__ L, int64_t n,
                                                      KernelParams kp, float* __restrict__ t) {
#pragma clang fp contract(off)
  __shared__ KScratch<MLP_SIDE> S;
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const KernelParams q = with_field(kp, L[i]);
    const int nk = dev_nk(w[i], q, false);
    if (nk <= MLP_SIDE) {
      double dropped;
      (void)wkernel_row(w[i], nk, q, S, &dropped);
    }
    const int a = (MLP_SIDE - nk) / 2;
    for (int j = threadIdx.x; j < MLP_SIDE * MLP_SIDE; j += 64) {
      const int sv = j / MLP_SIDE - a, su = j % MLP_SIDE - a;
      double2 v = make_double2(0.0, 0.0);
      if (nk <= MLP_SIDE && sv >= 0 && sv < nk && su >= 0 && su < nk) v = S.c[sv * nk + su];
      t[i * MLP_KOUT + 2 * j] = (float)v.x;
      t[i * MLP_KOUT + 2 * j + 1] = (float)v.y;
    }
    __syncthreads();
  }
}

hipError_t launch_rowsym(const double* uvw, int64_t r0, const ClassSlices& cs, double scale,
                         double gsx, double gsy, const double* mids, int P, const double* cents,
                         int Kx, int Ky, int tile, const KernelParams& kp, uint64_t* keys,
                         float* dropped, const Surrogate& sg, hipStream_t s) {
  // one launch per kernel-side class over that class's rows of the range
#define WF_ROWSYM(NKC, C)                                                                   \
  if (cs.n[C] > 0)                                                                          \
    hipLaunchKernelGGL(k_rowsym<NKC>, dim3(grid_for(cs.n[C])), dim3(64), 0, s, uvw, r0,   \
                       cs.rows[C], cs.n[C], scale, gsx, gsy, mids, P, cents, Kx, Ky, tile,  \
                       kp, keys, dropped, sg);
  WF_ROWSYM(7, 0)
  WF_ROWSYM(15, 1)
  WF_ROWSYM(21, 2)
  WF_ROWSYM(31, 3)
#undef WF_ROWSYM
  return hipGetLastError();
}

template <int STORE>
void launch_gbuild_classes(hipStream_t s, const double* uvw, int64_t s0, const ClassSlices& cs,
                           const int32_t* perm, const uint32_t* meta, const uint32_t* voff,
                           const int32_t* row_wi, const WorkItem* wi, double scale, double gsx,
                           double gsy, const double* mids, int P, const double* cents,
                           const KernelParams& kp, void* vals, int64_t vbase, int* mismatch,
                           const Surrogate& sg, const float* wts) {
  // one launch per kernel-side class over that class's rows of the range
#define WF_GBUILD(NKC, C)                                                                     \
  if (cs.n[C] > 0)                                                                            \
    hipLaunchKernelGGL((k_gbuild<STORE, NKC>), dim3(grid_for(cs.n[C])), dim3(64), 0, s, uvw,  \
                       s0, cs.rows[C], cs.n[C], perm, meta, voff, row_wi, wi, scale, gsx, gsy, \
                       mids, P, cents, kp, vals, vbase, mismatch, sg, wts);
  WF_GBUILD(7, 0)
  WF_GBUILD(15, 1)
  WF_GBUILD(21, 2)
  WF_GBUILD(31, 3)
#undef WF_GBUILD
}

hipError_t launch_gbuild(const double* uvw, int64_t s0, const ClassSlices& cs,
                         const int32_t* perm, const uint32_t* meta, const uint32_t* voff,
                         const int32_t* row_wi, const WorkItem* wi, double scale, double gsx,
                         double gsy, const double* mids, int P, const double* cents,
                         const KernelParams& kp, void* vals, int64_t vbase, wf_store store,
                         int* mismatch, const Surrogate& sg, const float* wts, hipStream_t s) {
  switch (store) {
    case WF_STORE_F32:
      launch_gbuild_classes<WF_STORE_F32>(s, uvw, s0, cs, perm, meta, voff, row_wi, wi, scale,
                                          gsx, gsy, mids, P, cents, kp, vals, vbase, mismatch,
                                          sg, wts);
      break;
    case WF_STORE_F16:
      launch_gbuild_classes<WF_STORE_F16>(s, uvw, s0, cs, perm, meta, voff, row_wi, wi, scale,
                                          gsx, gsy, mids, P, cents, kp, vals, vbase, mismatch,
                                          sg, wts);
      break;
    default:
      launch_gbuild_classes<WF_STORE_BF16>(s, uvw, s0, cs, perm, meta, voff, row_wi, wi, scale,
                                           gsx, gsy, mids, P, cents, kp, vals, vbase, mismatch,
                                           sg, wts);
      break;
  }
  return hipGetLastError();
}

template <int STORE>
void launch_khat_classes(hipStream_t s, const double* uvw, int64_t s0, const ClassSlices& cs,
                         const int32_t* perm, const uint32_t* meta, const int64_t* kabs,
                         double scale, double gsx, double gsy, const double* mids, int P,
                         const double* cents, const KernelParams& kp, void* khat, float* taps,
                         int* mismatch, const Surrogate& sg, const float* wts) {
#define WF_KHAT(NKC, C)                                                                      \
  if (cs.n[C] > 0)                                                                           \
    hipLaunchKernelGGL((k_khat<STORE, NKC>), dim3(grid_for(cs.n[C])), dim3(64), 0, s, uvw,   \
                       s0, cs.rows[C], cs.n[C], perm, meta, kabs, scale, gsx, gsy, mids, P,  \
                       cents, kp, khat, taps, mismatch, sg, wts);
  WF_KHAT(7, 0)
  WF_KHAT(15, 1)
  WF_KHAT(21, 2)
  WF_KHAT(31, 3)
#undef WF_KHAT
}

hipError_t launch_khat(const double* uvw, int64_t s0, const ClassSlices& cs, const int32_t* perm,
                       const uint32_t* meta, const int64_t* kabs, double scale, double gsx,
                       double gsy, const double* mids, int P, const double* cents,
                       const KernelParams& kp, void* khat, float* taps, wf_store store,
                       int* mismatch, const Surrogate& sg, const float* wts, hipStream_t s) {
  switch (store) {
    case WF_STORE_F32:
      launch_khat_classes<WF_STORE_F32>(s, uvw, s0, cs, perm, meta, kabs, scale, gsx, gsy, mids,
                                        P, cents, kp, khat, taps, mismatch, sg, wts);
      break;
    case WF_STORE_F16:
      launch_khat_classes<WF_STORE_F16>(s, uvw, s0, cs, perm, meta, kabs, scale, gsx, gsy, mids,
                                        P, cents, kp, khat, taps, mismatch, sg, wts);
      break;
    default:
      launch_khat_classes<WF_STORE_BF16>(s, uvw, s0, cs, perm, meta, kabs, scale, gsx, gsy,
                                         mids, P, cents, kp, khat, taps, mismatch, sg, wts);
      break;
  }
  return hipGetLastError();
}

template <int STORE, int JT>
void launch_expand_classes(hipStream_t s, const ExpSlices& cs, const uint32_t* meta,
                           const uint32_t* voff, const int32_t* row_wi, const WorkItem* wi,
                           const KernelParams& kp, const void* khat, const uint32_t* kof,
                           const float* taps, void* vals, int64_t vbase, int* over) {
  // one launch per kept-kernel side class; a workgroup expands rpw listed rows per step,
  // rpw chosen for about 8192 wavefronts per launch (eight per SIMD) and at least one
  // row per slot
#define WF_EXPAND(NKC, C)                                                                     \
  if (cs.n[C] > 0) {                                                                          \
    const int rpw = (int)std::min<int64_t>(                                                   \
        64, std::max<int64_t>(EScratch<NKC, JT>::SL, (cs.n[C] + 8191) / 8192));              \
    hipLaunchKernelGGL((k_expand<STORE, NKC, JT>), dim3(grid_for((cs.n[C] + rpw - 1) / rpw)), \
                       dim3(64), 0, s, cs.rows[C], cs.n[C], meta, voff, row_wi, wi, kp, khat,   \
                       kof, taps, vals, vbase, rpw, over);                                    \
  }
  WF_EXPAND(3, 0)
  WF_EXPAND(7, 1)
  WF_EXPAND(11, 2)
  WF_EXPAND(15, 3)
  WF_EXPAND(21, 4)
  WF_EXPAND(31, 5)
#undef WF_EXPAND
}

template <int STORE>
void launch_expand_store(hipStream_t s, const ExpSlices& cs, const uint32_t* meta,
                         const uint32_t* voff, const int32_t* row_wi, const WorkItem* wi,
                         const KernelParams& kp, const void* khat, const uint32_t* kof,
                         const float* taps, void* vals, int64_t vbase, int* over) {
  if (kp.J <= 7)
    launch_expand_classes<STORE, 7>(s, cs, meta, voff, row_wi, wi, kp, khat, kof, taps, vals,
                                    vbase, over);
  else
    launch_expand_classes<STORE, 15>(s, cs, meta, voff, row_wi, wi, kp, khat, kof, taps, vals,
                                     vbase, over);
}

hipError_t launch_expand(const ExpSlices& cs, const uint32_t* meta, const uint32_t* voff,
                         const int32_t* row_wi, const WorkItem* wi, const KernelParams& kp,
                         const void* khat, const uint32_t* kof, const float* taps, void* vals,
                         int64_t vbase, wf_store store, int* over, hipStream_t s) {
  switch (store) {
    case WF_STORE_F32:
      launch_expand_store<WF_STORE_F32>(s, cs, meta, voff, row_wi, wi, kp, khat, kof, taps, vals,
                                        vbase, over);
      break;
    case WF_STORE_F16:
      launch_expand_store<WF_STORE_F16>(s, cs, meta, voff, row_wi, wi, kp, khat, kof, taps, vals,
                                        vbase, over);
      break;
    default:
      launch_expand_store<WF_STORE_BF16>(s, cs, meta, voff, row_wi, wi, kp, khat, kof, taps,
                                         vals, vbase, over);
      break;
  }
  return hipGetLastError();
}

ClassSlices slice_classes(const RowClasses& rc, int64_t lo, int64_t hi) {
  ClassSlices cs{};
  for (int c = 0; c < 4; ++c) {
    const int32_t* b = rc.h.data() + rc.off[c];
    const int32_t* e = rc.h.data() + rc.off[c + 1];
    const int64_t i0 = std::lower_bound(b, e, (int32_t)lo) - b;
    const int64_t i1 = std::lower_bound(b, e, (int32_t)std::min<int64_t>(hi, INT32_MAX)) - b;
    cs.rows[c] = rc.d + rc.off[c] + i0;
    cs.n[c] = i1 - i0;
  }
  return cs;
}

hipError_t launch_row_class(const double* uvw, int64_t r0, int64_t r1, double scale, double gsx,
                            double gsy, const double* mids, int P, const double* cents,
                            const KernelParams& kp, uint8_t* cls, hipStream_t s) {
  const int64_t n = r1 - r0;
  if (n <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_row_class, dim3((unsigned)nb), dim3(256), 0, s, uvw, r0, r1, scale, gsx,
                     gsy, mids, P, cents, kp, cls);
  return hipGetLastError();
}


hipError_t launch_row_inputs(const double* uvw, const int32_t* list, const int32_t* perm,
                             int64_t r0, int64_t nr,
                             double scale, double gsx, double gsy, const double* mids, int P,
                             const double* cents, const KernelParams& kp, double L, float* x,
                             hipStream_t s) {
  if (nr <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((nr + 255) / 256, 16384);
  hipLaunchKernelGGL(k_row_inputs, dim3((unsigned)nb), dim3(256), 0, s, uvw, list, perm, r0, nr,
                     scale, gsx, gsy, mids, P, cents, kp, L, x);
  return hipGetLastError();
}

hipError_t launch_train_inputs(const double* w, const double* L, const double* fu,
                               const double* fv, int64_t n, const KernelParams& kp, float* x,
                               int32_t* nk, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_train_inputs, dim3((unsigned)nb), dim3(256), 0, s, w, L, fu, fv, n, kp,
                     x, nk);
  return hipGetLastError();
}

hipError_t launch_exact_targets(const double* w, const double* L, int64_t n,
                                const KernelParams& kp, float* t, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)(n < 262144 ? n : 262144);
  hipLaunchKernelGGL(k_exact_targets, dim3(blocks), dim3(64), 0, s, w, L, n, kp, t);
  return hipGetLastError();
}

}  // namespace wf
