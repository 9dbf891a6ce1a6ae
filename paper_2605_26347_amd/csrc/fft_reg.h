// Register-resident radix-16/32 FFT passes for CDNA (wave64), used by the row passes of
// the oversampled 2-D DFT F (Sect. 3.2, eq. 6) at the long row lengths.
//
// A length-N transform runs as three Stockham passes of radices R1, R2, R3
// (N = R1 R2 R3, each at most 32).  A thread holds E = N / NT elements and performs
// E / R butterflies per pass entirely in registers; between passes the data crosses
// LDS once.  The first pass reads its inputs straight from global memory (with the
// image-domain modulation fused in) and the last pass writes its outputs, which come
// out in natural order, straight to global memory.  Pass with radix R and sub-transform
// length Ns: butterfly j in [0, N/R) reads x[j + r N/R], multiplies input r by
// W_{Ns R}^{r (j mod Ns)}, does an R-point DFT and writes output r to
// ((j / Ns) Ns R + j mod Ns) + r Ns.
// R-point DFTs of 16 and 32 points are Cooley-Tukey products of the 2/4/8-point ones
// with their inner twiddles as compile-time constants (cos and sin of k pi / 16 from
// their Taylor series, evaluated in double precision by the compiler).
#pragma once

#include <hip/hip_runtime.h>

#include "fft_lds.h"

namespace wf {

namespace twc {
constexpr double PI = 3.14159265358979323846264338327950288;
// sin and cos of x in [-pi, pi] from their Taylor series (terms to x^49: below 1e-17)
constexpr double tsin(double x) {
  double term = x, sum = x;
  for (int i = 1; i < 25; ++i) {
    term *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double tcos(double x) {
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 25; ++i) {
    term *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
    sum += term;
  }
  return sum;
}
// angle 2 pi m / n reduced to [-pi, pi]
constexpr double ang(int m, int n) {
  const int r = ((m % n) + n) % n;
  const double a = 2.0 * PI * (double)r / (double)n;
  return a > PI ? a - 2.0 * PI : a;
}
}  // namespace twc

// exp(-2 pi i m / n) (forward) or its conjugate (inverse), rounded to FP32
template <int M, int N, bool INV>
struct Twiddle {
  static constexpr float c = (float)twc::tcos(twc::ang(M, N));
  static constexpr float s = (float)(INV ? twc::tsin(twc::ang(M, N)) : -twc::tsin(twc::ang(M, N)));
};

template <int M, int N, bool INV>
__device__ __forceinline__ float2 twiddle_const(float2 a) {
  if constexpr (((M % N) + N) % N == 0) {
    return a;
  } else if constexpr (4 * (((M % N) + N) % N) == N) {  // -i (forward) / +i (inverse)
    return rot90<INV>(a);
  } else if constexpr (2 * (((M % N) + N) % N) == N) {
    return make_float2(-a.x, -a.y);
  } else {
    constexpr float c = Twiddle<M, N, INV>::c, s = Twiddle<M, N, INV>::s;
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

template <int R, bool INV>
__device__ __forceinline__ void dft_reg(float2* v);

// Cooley-Tukey R = A B: x[B n1 + n2] -> A-point DFTs over n1, twiddles W_R^{n2 k1},
// B-point DFTs over n2 -> X[k1 + A k2].
template <int A, int B, bool INV>
struct CT {
  template <int K1, int N2>
  static __device__ __forceinline__ void tw(float2 (&t)[A * B]) {
    t[K1 * B + N2] = twiddle_const<K1 * N2, A * B, INV>(t[K1 * B + N2]);
    if constexpr (N2 + 1 < B) {
      tw<K1, N2 + 1>(t);
    } else if constexpr (K1 + 1 < A) {
      tw<K1 + 1, 0>(t);
    }
  }
  static __device__ __forceinline__ void run(float2* v) {
    float2 t[A * B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      float2 s[A];
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) s[n1] = v[B * n1 + n2];
      dft_reg<A, INV>(s);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) t[k1 * B + n2] = s[k1];
    }
    tw<0, 0>(t);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      float2 s[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) s[n2] = t[k1 * B + n2];
      dft_reg<B, INV>(s);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = s[k2];
    }
  }
};

template <int R, bool INV>
__device__ __forceinline__ void dft_reg(float2* v) {
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v);
  else if constexpr (R == 8) dft8<INV>(v);
  else if constexpr (R == 16) CT<4, 4, INV>::run(v);
  else CT<8, 4, INV>::run(v);
}

// The three radices of a length-N row transform and its thread count.
template <int N>
struct RowPlan {
  static constexpr int R1 = N >= 8192 ? 32 : 16;
  static constexpr int R2 = N >= 16384 ? 32 : 16;
  static constexpr int R3 = N / (R1 * R2);
  static constexpr int E = R1 > R2 ? (R1 > R3 ? R1 : R3) : (R2 > R3 ? R2 : R3);
  static constexpr int NT = N / E;
};

// Whether element q = j + r S (j < S) of a pass lies in a needed column strip of mask m
// (strip q / 16).  When a step of S covers at most 32 strips, all lanes' strips of one r
// share one mask word, so that word is one uniform load per r instead of a load per
// element.
template <int S>
__device__ __forceinline__ bool strip_on(const uint32_t* __restrict__ m, int j, int r) {
  constexpr int SS = S / 16;
  if constexpr (SS <= 32) {
    static_assert(32 % SS == 0, "strips per step must divide a mask word");
    const uint32_t w = m[(r * SS) >> 5];
    return (w >> (((r * SS) & 31) + (j >> 4))) & 1u;
  } else {
    const int st = (j >> 4) + r * SS;
    return (m[st >> 5] >> (st & 31)) & 1u;
  }
}

// LDS slot of element idx: one float2 of padding after every 32, so that the strided
// writes of the first pass (stride R1 elements) spread over the banks.
__device__ __forceinline__ int lds_slot(int idx) { return idx + (idx >> 5); }
template <int N>
constexpr int lds_elems() {
  return N + N / 32;
}

// One middle pass over the line in buf: inputs from LDS, outputs to LDS (all inputs are
// read before the barrier, outputs written after it).  The butterflies of a thread are
// j = tid + b NT; several lines may share the block, each with its own NT threads.
template <int N, int R, int NS, int NT, bool INV>
__device__ __forceinline__ void reg_pass_lds(float2* buf, const float2* __restrict__ tw,
                                             int tid) {
  constexpr int B = (N / R) / NT;
  float2 v[B][R];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = tid + b * NT;
#pragma unroll
    for (int r = 0; r < R; ++r) v[b][r] = buf[lds_slot(j + r * (N / R))];
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = tid + b * NT;
    const int kk = j & (NS - 1);
    const int step = kk * (N / (NS * R));
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const float2 t = tw[r * step];
      v[b][r] = INV ? cmulc(v[b][r], t) : cmul(v[b][r], t);
    }
    dft_reg<R, INV>(v[b]);
    const int d = (j - kk) * R + kk;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[lds_slot(d + r * NS)] = v[b][r];
  }
  __syncthreads();
}

// Cross-lane exchange through LDS in two halves, the real parts and then the imaginary
// parts, so that a line occupies N floats of LDS instead of N complex values.  out[k]
// goes to slot oslot(k) and in[k] comes from slot islot(k); the block's threads pass the
// four barriers together (the last one lets the next exchange reuse the buffer).
// The slots are functions of (k, tid); they are computed afresh for the second half
// (the empty asm hides that tid is unchanged) instead of being held in registers across
// it.
template <int KO, int KI, typename OS, typename IS>
__device__ __forceinline__ void xchg_split(float* buf, int tid, const float2 (&out)[KO],
                                           OS&& oslot, float2 (&in)[KI], IS&& islot) {
  int t = tid;
#pragma unroll
  for (int k = 0; k < KO; ++k) buf[oslot(k, t)] = out[k].x;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KI; ++k) in[k].x = buf[islot(k, t)];
  __syncthreads();
  asm volatile("" : "+v"(t));
#pragma unroll
  for (int k = 0; k < KO; ++k) buf[oslot(k, t)] = out[k].y;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KI; ++k) in[k].y = buf[islot(k, t)];
  __syncthreads();
}

// The same exchange with complex values in one go (N complex values of LDS per line).
template <int KO, int KI, typename OS, typename IS>
__device__ __forceinline__ void xchg_full(float2* buf, int tid, const float2 (&out)[KO],
                                          OS&& oslot, float2 (&in)[KI], IS&& islot) {
#pragma unroll
  for (int k = 0; k < KO; ++k) buf[oslot(k, tid)] = out[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KI; ++k) in[k] = buf[islot(k, tid)];
  __syncthreads();
}

// Whether a transform of length N exchanges its lines as floats (xchg_split): from 8192
// points on, where a complex line's LDS, not its registers, limits the lines per compute
// unit; shorter lines fit by registers already and would only pay the extra barriers.
template <int N>
constexpr bool line_split() {
  return N >= 8192;
}
// LDS of one line in bytes.
template <int N>
constexpr size_t line_lds_bytes() {
  return (size_t)lds_elems<N>() * (line_split<N>() ? sizeof(float) : sizeof(float2));
}

// The middle of a row transform, the line crossing LDS twice (xchg_split or xchg_full as
// line_split says; buf is the line, in floats or complex values accordingly).  v1 holds
// the first pass's outputs of the thread's butterflies j = tid + b NT (output r of
// butterfly j belongs at position j R1 + r); the second pass (radix R2, sub-transform
// length R1, twiddles from tw) runs in registers between the two exchanges; v3 receives
// the third pass's inputs x[j + r R1 R2].
template <int N, bool INV>
__device__ __forceinline__ void row_middle(void* buf, const float2 (&v1)[N / RowPlan<N>::NT],
                                           float2 (&v3)[N / RowPlan<N>::NT],
                                           const float2* __restrict__ tw, int tid) {
  using RP = RowPlan<N>;
  constexpr int R1 = RP::R1, R2 = RP::R2, R3 = RP::R3, NT = RP::NT, E = N / NT;
  constexpr int B2 = (N / R2) / NT;
  static_assert(((N / R1) / NT) * R1 == E && B2 * R2 == E && ((N / R3) / NT) * R3 == E,
                "every pass holds E elements per thread");
  float2 v2[E];
  auto xchg = [&](const float2(&o)[E], auto&& os, float2(&in)[E], auto&& is) {
    if constexpr (line_split<N>())
      xchg_split(reinterpret_cast<float*>(buf), tid, o, os, in, is);
    else
      xchg_full(reinterpret_cast<float2*>(buf), tid, o, os, in, is);
  };
  xchg(
      v1,
      [](int k, int t) {
        const int b = k / R1, r = k - b * R1;
        return lds_slot((t + b * NT) * R1 + r);
      },
      v2,
      [](int k, int t) {
        const int b = k / R2, r = k - b * R2;
        return lds_slot(t + b * NT + r * (N / R2));
      });
#pragma unroll
  for (int b = 0; b < B2; ++b) {
    const int j = tid + b * NT;
    const int kk = j & (R1 - 1);
    const int step = kk * (N / (R1 * R2));
#pragma unroll
    for (int r = 1; r < R2; ++r) {
      const float2 t = tw[r * step];
      v2[b * R2 + r] = INV ? cmulc(v2[b * R2 + r], t) : cmul(v2[b * R2 + r], t);
    }
    dft_reg<R2, INV>(v2 + b * R2);
  }
  xchg(
      v2,
      [](int k, int t) {
        const int b = k / R2, r = k - b * R2;
        const int j = t + b * NT, kk = j & (R1 - 1);
        return lds_slot((j - kk) * R2 + kk + r * R1);
      },
      v3,
      [](int k, int t) {
        const int b = k / R3, r = k - b * R3;
        return lds_slot(t + b * NT + r * (R1 * R2));
      });
}

}  // namespace wf
