// LDS-resident complex FFTs for CDNA (wave64), used by the row and column passes of
// the oversampled 2-D DFT F (Sect. 3.2, eq. 6).
//
// Stockham auto-sort formulation, mixed radix (one radix-2 or radix-4 stage when
// log2 N is not a multiple of 3, then radix-8 stages).  Stage with radix R and current
// sub-transform length Ns: butterfly j in [0, N/R) reads x[j + r N/R], multiplies
// input r by W_{Ns R}^{r (j mod Ns)}, does an R-point DFT and writes output r to
// ((j / Ns) Ns R + j mod Ns) + r Ns.  Every thread loads all of its butterflies into
// registers before the block-wide barrier, so each stage runs in place in one buffer.
// Twiddles come from a table tw[m] = exp(-2 pi i m / N), m < N, built on the host in
// FP64 and rounded to FP32; the inverse transform uses their conjugates.
#pragma once

#include <hip/hip_runtime.h>

namespace wf {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2* v) {
  float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  float2 a2 = cadd(v[1], v[3]), a3 = rot90<INV>(csub(v[1], v[3]));
  v[0] = cadd(a0, a2);
  v[2] = csub(a0, a2);
  v[1] = cadd(a1, a3);
  v[3] = csub(a1, a3);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  const float h = 0.70710678118654752440f;
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  // o[k] *= W8^k (forward W8 = exp(-i pi/4))
  float2 o1 = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                  : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
  float2 o2 = rot90<INV>(o[2]);
  float2 o3 = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                  : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(float2* v) {
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v);
  else dft8<INV>(v);
}

// One Stockham stage over B lines of length N (line stride S elements) held in LDS.
template <int N, int R, int NT, int B, bool INV>
__device__ __forceinline__ void stockham_stage(float2* buf, int S, int Ns,
                                               const float2* __restrict__ tw) {
  constexpr int NB = N / R;
  constexpr int TOT = NB * B;
  constexpr int PER = (TOT + NT - 1) / NT;
  float2 v[PER][R];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int b = threadIdx.x + k * NT;
    if ((TOT % NT) == 0 || b < TOT) {
      const int line = b / NB, j = b - line * NB;
      const float2* L = buf + line * S;
#pragma unroll
      for (int r = 0; r < R; ++r) v[k][r] = L[j + r * NB];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int b = threadIdx.x + k * NT;
    if ((TOT % NT) == 0 || b < TOT) {
      const int line = b / NB, j = b - line * NB;
      const int kk = j & (Ns - 1);
      if (Ns > 1) {
        const int step = kk * (N / (Ns * R));
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 t = tw[r * step];
          v[k][r] = INV ? cmulc(v[k][r], t) : cmul(v[k][r], t);
        }
      }
      dftR<R, INV>(v[k]);
      float2* L = buf + line * S;
      const int d = (j - kk) * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) L[d + r * Ns] = v[k][r];
    }
  }
  __syncthreads();
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// In-place FFT of B lines of length N in LDS.  Caller must __syncthreads() before
// (data written) -- the first stage's loads happen before its barrier.
template <int N, int NT, int B, bool INV>
__device__ __forceinline__ void fft_lines(float2* buf, int S, const float2* __restrict__ tw) {
  constexpr int L2 = ilog2(N);
  constexpr int n8 = L2 / 3;
  constexpr int rem = L2 - 3 * n8;
  int Ns = 1;
  if constexpr (rem == 1) {
    stockham_stage<N, 2, NT, B, INV>(buf, S, Ns, tw);
    Ns *= 2;
  } else if constexpr (rem == 2) {
    stockham_stage<N, 4, NT, B, INV>(buf, S, Ns, tw);
    Ns *= 4;
  }
#pragma unroll
  for (int s = 0; s < n8; ++s) {
    stockham_stage<N, 8, NT, B, INV>(buf, S, Ns, tw);
    Ns *= 8;
  }
}

// Map workgroup ids so that each XCD (workgroups are dealt round-robin over 8 XCDs)
// receives one contiguous range of logical ids: neighbouring logical work then runs
// concurrently on one L2.  Bijective for any count.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, k = b >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

}  // namespace wf
