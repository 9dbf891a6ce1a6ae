// Row and column passes of F and F^dag with the image-domain work fused in
// (Sect. 3.2, eq. 6; Sect. 3.3, eq. 8):
//   forward rows : x (.) Z_p, zero-pad to Kx, FFT of the ny image rows      -> A
//   forward cols : zero-pad to Ky, FFT of every column                     -> X
//   inverse cols : inverse FFT of every column, keep the ny image rows     -> A
//                  (and clear Y behind the read, ready for the next gridding)
//   inverse rows : inverse FFT of the ny rows, crop to nx, (.) conj(Z_p),
//                  store or accumulate the sum over w-layers (eq. 7)
// Pruning to the bin's active uv support (the discrete Fourier modes its rows touch, plus
// a one-tile halo): the forward column pass writes X only inside needed tiles, the inverse
// column pass reads (and clears) Y only there, and both row passes touch only the column
// strips that hold needed tiles; everything else is known to be unused or zero.  Null
// masks mean the full grid.
// Z_p = grid correction x w-layer: s_i s_j exp(-2 pi i w_p (n-1)) / n with the phase
// computed in FP64 (n - 1 = -(l^2+m^2)/(1+n) avoids cancellation), reduced to
// [-1/2, 1/2) cycles in FP64 and only then rounded to FP32 for sincospi.
#include <mutex>
#include <vector>

#include "fft_lds.h"
#include "fft_reg.h"
#include "wf_internal.h"

namespace wf {

// n - 1 = sqrt(1 - r2) - 1 for r2 = l^2 + m^2 in FP64.  Inside r2 < 1/20 (fields up to
// about 25 degrees across) the binomial series of sqrt(1 - x) - 1 to x^12, whose
// coefficients are exact dyadic fractions, in Horner form: the next term is below 1e-17
// of the result, so it matches -r2 / (1 + sqrt(1 - r2)) to FP64 rounding, at a dozen
// fused multiply-adds instead of a square root and a division.
__device__ __forceinline__ double nm1_of(double r2) {
  if (r2 < 0.05) {
    double p = -29393.0 / 4194304.0;
    p = fma(p, r2, -4199.0 / 524288.0);
    p = fma(p, r2, -2431.0 / 262144.0);
    p = fma(p, r2, -715.0 / 65536.0);
    p = fma(p, r2, -429.0 / 32768.0);
    p = fma(p, r2, -33.0 / 2048.0);
    p = fma(p, r2, -21.0 / 1024.0);
    p = fma(p, r2, -7.0 / 256.0);
    p = fma(p, r2, -5.0 / 128.0);
    p = fma(p, r2, -1.0 / 16.0);
    p = fma(p, r2, -1.0 / 8.0);
    p = fma(p, r2, -0.5);
    return p * r2;
  }
  return -r2 / (1.0 + sqrt(1.0 - r2));
}

__device__ __forceinline__ float2 zvalue(int i, int j, int nx, int ny, double cell, double wp,
                                         float sxi, float syj) {
  const double l = (double)(i - nx / 2) * cell;
  const double m = (double)(j - ny / 2) * cell;
  const double r2 = l * l + m * m;
  const double d = nm1_of(r2);
  const double n = 1.0 + d;
  double cyc = -wp * d;
  cyc -= rint(cyc);
  float s, c;
  sincospif((float)(2.0 * cyc), &s, &c);
  const float a = sxi * syj / (float)n;
  return make_float2(a * c, a * s);
}

// Z_p = s(l) s(m) / n exp(-2 i pi w_p (n - 1)) split by n - 1 = -(l^2 + m^2)/2 + D(r2),
// r2 = l^2 + m^2, D = -r2^2/8 - r2^3/16 - 5 r2^4/128 - 7 r2^5/256 - ...:
//   Z_p = C_p(l) R_p(m) exp(i theta) / n,  C_p(l) = s(l) exp(i pi w_p l^2) (a per-bin table
//   of the image columns, FP64 phase at build), R_p(m) = s(m) exp(i pi w_p m^2) (FP64
//   phase once per row), theta = -2 pi w_p D(r2).
// Where r2 <= 1/100 over the image and |theta| <= 1/4 (the table exists only then), D and
// 1/n = 1 + r2/2 + 3 r2^2/8 + ... are FP32 series truncated below 1e-9 relative, and
// exp(i theta) its Taylor series to theta^7 (error below 1e-9): each factor carries an
// FP32 rounding error, a few 1e-7 in all, like the FP32 sine and cosine of the direct form.
struct ChirpRow {
  float2 R;      // s(m) exp(i pi w_p m^2)
  float m2;      // m^2
  float kth;     // -2 pi w_p
  float cellf;
  int hx;        // nx / 2
};

__device__ __forceinline__ ChirpRow chirp_row(int j, int nx, int ny, double cell, double wp,
                                              float syj) {
  ChirpRow c;
  const double m = (double)(j - ny / 2) * cell;
  double cyc = 0.5 * wp * (m * m);
  cyc -= rint(cyc);
  float sn, cs;
  sincospif((float)(2.0 * cyc), &sn, &cs);
  c.R = make_float2(syj * cs, syj * sn);
  c.m2 = (float)(m * m);
  c.kth = (float)(-2.0 * M_PI * wp);
  c.cellf = (float)cell;
  c.hx = nx / 2;
  return c;
}

__device__ __forceinline__ float2 zvalue_tab(const ChirpRow& c, int i, float2 ci) {
  const float li = (float)(i - c.hx) * c.cellf;
  const float r2 = fmaf(li, li, c.m2);
  const float dl = -(r2 * r2) * fmaf(r2, fmaf(r2, fmaf(r2, 7.f / 256.f, 5.f / 128.f),
                                               1.f / 16.f), 1.f / 8.f);
  const float th = c.kth * dl;
  const float t2 = th * th;
  const float ct = fmaf(t2, fmaf(t2, fmaf(t2, -1.f / 720.f, 1.f / 24.f), -0.5f), 1.f);
  const float st = th * fmaf(t2, fmaf(t2, fmaf(t2, -1.f / 5040.f, 1.f / 120.f), -1.f / 6.f),
                             1.f);
  const float inv_n =
      fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, 35.f / 128.f, 5.f / 16.f), 3.f / 8.f), 0.5f), 1.f);
  const float2 a = make_float2(ci.x * ct - ci.y * st, ci.x * st + ci.y * ct);
  const float2 b = make_float2(a.x * c.R.x - a.y * c.R.y, a.x * c.R.y + a.y * c.R.x);
  return make_float2(b.x * inv_n, b.y * inv_n);
}

// C_p(l_i) = s(l_i) exp(i pi w_p l_i^2), i < nx: FP64 phase reduced to one cycle, FP64 sine
// and cosine.
__global__ __launch_bounds__(256) void k_chirp_table(float2* __restrict__ ct, int nx,
                                                     double cell, double wp,
                                                     const float* __restrict__ sx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx) return;
  const double l = (double)(i - nx / 2) * cell;
  double cyc = 0.5 * wp * (l * l);
  cyc -= rint(cyc);
  double sn, cs;
  sincospi(2.0 * cyc, &sn, &cs);
  ct[i] = make_float2((float)(sx[i] * cs), (float)(sx[i] * sn));
}

__device__ __forceinline__ bool bit_set(const uint32_t* __restrict__ m, int i) {
  return (m[i >> 5] >> (i & 31)) & 1u;
}

// Geometry of the pruning masks: tile bitmap [Ky/tile][Kx/tile] and strip bitmap
// [Kx/16], both as packed 32-bit words.
struct Masks {
  const uint32_t* strip;  // null: all strips needed
  const uint32_t* tile;   // null: all tiles needed
  const int32_t* groups;  // null: column groups 0..n-1
  int tiles_x;
  int tsh;                // log2(tile)
};

template <int N>
constexpr int row_threads() {
  return N / 16 < 64 ? 64 : (N / 16 > 1024 ? 1024 : N / 16);
}
template <int N>
constexpr int col_width() {
  return (16384 / N) > 16 ? 16 : (16384 / N);
}
template <int N>
constexpr int col_threads() {
  return (col_width<N>() * N) / 16 < 64 ? 64
         : ((col_width<N>() * N) / 16 > 1024 ? 1024 : (col_width<N>() * N) / 16);
}

template <int N, int NT>
__global__ __launch_bounds__(NT) void k_fwd_rows(const float* __restrict__ img,
                                                 float2* __restrict__ A,
                                                 const float2* __restrict__ tw,
                                                 const float* __restrict__ sx,
                                                 const float* __restrict__ sy, int nx, int ny,
                                                 double cell, double wp,
                                                 const uint32_t* __restrict__ smask) {
  extern __shared__ float2 buf[];
  const int j = blockIdx.x;
  const float syj = sy[j];
  for (int t = threadIdx.x; t < N - nx; t += NT) buf[nx / 2 + t] = make_float2(0.f, 0.f);
  const float* row = img + (int64_t)j * nx;
  for (int i = threadIdx.x; i < nx; i += NT) {
    const float v = row[i];
    const float2 z = zvalue(i, j, nx, ny, cell, wp, sx[i], syj);
    buf[(i - nx / 2) & (N - 1)] = make_float2(v * z.x, v * z.y);
  }
  __syncthreads();
  fft_lines<N, NT, 1, false>(buf, N, tw);
  for (int q = threadIdx.x; q < N; q += NT)
    if (!smask || bit_set(smask, q >> 4)) A[strip_index(j, q, ny)] = buf[q];
}

template <int N, int NT>
__global__ __launch_bounds__(NT) void k_inv_rows(const float2* __restrict__ A,
                                                 void* __restrict__ out,
                                                 const float2* __restrict__ tw,
                                                 const float* __restrict__ sx,
                                                 const float* __restrict__ sy, int nx, int ny,
                                                 double cell, double wp, int mode,
                                                 const uint32_t* __restrict__ smask) {
  extern __shared__ float2 buf[];
  const int j = blockIdx.x;
  for (int q = threadIdx.x; q < N; q += NT)
    buf[q] = (!smask || bit_set(smask, q >> 4)) ? A[strip_index(j, q, ny)]
                                                : make_float2(0.f, 0.f);
  __syncthreads();
  fft_lines<N, NT, 1, true>(buf, N, tw);
  const float syj = sy[j];
  for (int i = threadIdx.x; i < nx; i += NT) {
    const float2 v = buf[(i - nx / 2) & (N - 1)];
    const float2 z = zvalue(i, j, nx, ny, cell, wp, sx[i], syj);
    const float2 r = cmulc(v, z);
    const int64_t o = (int64_t)j * nx + i;
    if (mode < 2) {
      float2* po = reinterpret_cast<float2*>(out) + o;
      if (mode == 1) {
        const float2 p = *po;
        *po = make_float2(p.x + r.x, p.y + r.y);
      } else {
        *po = r;
      }
    } else {
      float* po = reinterpret_cast<float*>(out) + o;
      *po = (mode == 3) ? (*po + r.x) : r.x;
    }
  }
}

// Row passes at the long lengths (N = 2048 .. 16384): three register-resident passes
// (fft_reg.h).  Since N = 2 nx, input r of a first-pass butterfly holds an image pixel
// exactly when r < R1/4 (pixel q + nx/2) or r >= 3 R1/4 (pixel q - 3 nx/2), and output r
// of a last-pass butterfly lands inside the crop under the same rule with R3: the zero
// half of the padded row and the discarded half of the inverse are skipped at compile
// time.
// With a sweep's layer table sl, workgroup (row, layer) takes the layer's grid, mask and
// centroid from sl[blockIdx.y] and its channel's image from img (all channels' images).
template <int N>
__global__ __launch_bounds__(RowPlan<N>::NT) __attribute__((amdgpu_waves_per_eu(4))) void k_fwd_rows_reg(
    const float* __restrict__ img, float2* __restrict__ A, const float2* __restrict__ tw,
    const float* __restrict__ sx, const float* __restrict__ sy, int nx, int ny, double cell,
    double wp, const uint32_t* __restrict__ smask, const SweepLayer* __restrict__ sl,
    const float2* __restrict__ ctab) {
  using RP = RowPlan<N>;
  constexpr int R1 = RP::R1, R2 = RP::R2, R3 = RP::R3, NT = RP::NT;
  extern __shared__ float2 buf[];
  const int jr = blockIdx.x;
  if (sl) {
    const SweepLayer& L = sl[blockIdx.y];
    img += (int64_t)L.chan * nx * ny;
    A = L.A;
    wp = L.wp;
    smask = L.smask;
    ctab = L.ctab;
  }
  const float syj = sy[jr];
  const float* __restrict__ row = img + (int64_t)jr * nx;
  float2 v1[N / NT];
  {
    constexpr int B = (N / R1) / NT;
    // the modulation of the lane's pixels, one uniform branch for the whole row (a
    // branch per pixel would keep the loads of different pixels from overlapping)
    auto pix = [&](int b, int r) {
      const int q = threadIdx.x + b * NT + r * (N / R1);
      return r < R1 / 4 ? q + nx / 2 : q - 3 * (nx / 2);
    };
    float2 zr[B][R1 / 2];
    if (ctab) {
      const ChirpRow cr = chirp_row(jr, nx, ny, cell, wp, syj);
#pragma unroll
      for (int b = 0; b < B; ++b)
#pragma unroll
        for (int r = 0; r < R1; ++r)
          if (r < R1 / 4 || r >= 3 * R1 / 4) {
            const int i = pix(b, r);
            zr[b][r < R1 / 4 ? r : r - R1 / 2] = zvalue_tab(cr, i, ctab[i]);
          }
    } else {
#pragma unroll
      for (int b = 0; b < B; ++b)
#pragma unroll
        for (int r = 0; r < R1; ++r)
          if (r < R1 / 4 || r >= 3 * R1 / 4) {
            const int i = pix(b, r);
            zr[b][r < R1 / 4 ? r : r - R1 / 2] = zvalue(i, jr, nx, ny, cell, wp, sx[i], syj);
          }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      float2* v = v1 + b * R1;
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        if (r < R1 / 4 || r >= 3 * R1 / 4) {
          const float x = row[pix(b, r)];
          const float2 z = zr[b][r < R1 / 4 ? r : r - R1 / 2];
          v[r] = make_float2(x * z.x, x * z.y);
        } else {
          v[r] = make_float2(0.f, 0.f);
        }
      }
      dft_reg<R1, false>(v);
    }
  }
  float2 v3[N / NT];
  row_middle<N, false>(buf, v1, v3, tw, threadIdx.x);
  {
    // the thread index taken afresh (the empty asm hides that it is unchanged) rather
    // than held through the exchanges; a wave-uniform row base and 32-bit strip offsets
    // (a grid holds at most 2^27 elements)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    float2* __restrict__ arow = A + (int64_t)jr * SW;
    constexpr int NS = R1 * R2;
    constexpr int B = (N / R3) / NT;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = tid + b * NT;
      float2* v = v3 + b * R3;
#pragma unroll
      for (int r = 1; r < R3; ++r) v[r] = cmul(v[r], tw[r * j]);
      dft_reg<R3, false>(v);
#pragma unroll
      for (int r = 0; r < R3; ++r) {
        const int q = j + r * NS;
        if (!smask || strip_on<NS>(smask, j, r)) arow[(q >> 4) * ny * SW + (q & (SW - 1))] = v[r];
      }
    }
  }
}

template <int N>
__global__ __launch_bounds__(RowPlan<N>::NT) __attribute__((amdgpu_waves_per_eu(3))) void k_inv_rows_reg(
    const float2* __restrict__ A, void* __restrict__ out, const float2* __restrict__ tw,
    const float* __restrict__ sx, const float* __restrict__ sy, int nx, int ny, double cell,
    double wp, int mode, const uint32_t* __restrict__ smask, const float2* __restrict__ ctab) {
  using RP = RowPlan<N>;
  constexpr int R1 = RP::R1, R2 = RP::R2, R3 = RP::R3, NT = RP::NT;
  extern __shared__ float2 buf[];
  const int jr = blockIdx.x;
  constexpr int NS3 = R1 * R2;
  constexpr int B3 = (N / R3) / NT;
  float2 v1[N / NT];
  {
    constexpr int B = (N / R1) / NT;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = threadIdx.x + b * NT;
      float2* v = v1 + b * R1;
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int q = j + r * (N / R1);
        v[r] = (!smask || strip_on<N / R1>(smask, j, r)) ? A[strip_index(jr, q, ny)]
                                                         : make_float2(0.f, 0.f);
      }
      dft_reg<R1, true>(v);
    }
  }
  float2 v3[N / NT];
  row_middle<N, true>(buf, v1, v3, tw, threadIdx.x);
  const float syj = sy[jr];
  {
    constexpr int NS = R1 * R2;
    constexpr int B = (N / R3) / NT;
    // the modulation of the lane's output pixels, one uniform branch for the row
    auto pix = [&](int b, int r) {
      const int q = threadIdx.x + b * NT + r * NS;
      return r < R3 / 4 ? q + nx / 2 : q - 3 * (nx / 2);
    };
    const ChirpRow cr = chirp_row(jr, nx, ny, cell, wp, syj);
#pragma unroll
    for (int b = 0; b < B; ++b) {
      // one group's modulations at a time (registers), one uniform branch per group
      float2 zr[R3 / 2];
      if (ctab) {
#pragma unroll
        for (int r = 0; r < R3; ++r)
          if (r < R3 / 4 || r >= 3 * R3 / 4) {
            const int i = pix(b, r);
            zr[r < R3 / 4 ? r : r - R3 / 2] = zvalue_tab(cr, i, ctab[i]);
          }
      } else {
#pragma unroll
        for (int r = 0; r < R3; ++r)
          if (r < R3 / 4 || r >= 3 * R3 / 4) {
            const int i = pix(b, r);
            zr[r < R3 / 4 ? r : r - R3 / 2] = zvalue(i, jr, nx, ny, cell, wp, sx[i], syj);
          }
      }
      const int j = threadIdx.x + b * NT;
      // the previous image sum of the real-part accumulate mode, requested before this
      // group's transform so that its latency hides behind it (per group: registers)
      float prev[R3 / 2];
      if (mode == 3) {
#pragma unroll
        for (int r = 0; r < R3; ++r)
          if (r < R3 / 4 || r >= 3 * R3 / 4) {
            const int q = j + r * NS3;
            const int i = r < R3 / 4 ? q + nx / 2 : q - 3 * (nx / 2);
            prev[r < R3 / 4 ? r : r - R3 / 2] =
                reinterpret_cast<const float*>(out)[(int64_t)jr * nx + i];
          }
      }
      float2* v = v3 + b * R3;
#pragma unroll
      for (int r = 1; r < R3; ++r) v[r] = cmulc(v[r], tw[r * j]);
      dft_reg<R3, true>(v);
#pragma unroll
      for (int r = 0; r < R3; ++r) {
        if (r < R3 / 4 || r >= 3 * R3 / 4) {
          const int q = j + r * NS;
          const int i = r < R3 / 4 ? q + nx / 2 : q - 3 * (nx / 2);
          const float2 c = cmulc(v[r], zr[r < R3 / 4 ? r : r - R3 / 2]);
          const int64_t o = (int64_t)jr * nx + i;
          if (mode < 2) {
            float2* po = reinterpret_cast<float2*>(out) + o;
            if (mode == 1) {
              const float2 p = *po;
              *po = make_float2(p.x + c.x, p.y + c.y);
            } else {
              *po = c;
            }
          } else {
            float* po = reinterpret_cast<float*>(out) + o;
            *po = (mode == 3) ? (prev[r < R3 / 4 ? r : r - R3 / 2] + c.x) : c.x;
          }
        }
      }
    }
  }
}

// Inverse row pass of a sweep: workgroup (row jr, channel c = c0 + y) transforms row jr of every
// layer of channel c in turn (chan_layers[c] = first layer, count) and accumulates
// conj(Z_p) F^dag ... in registers, then writes the channel's image row once (complex, or
// its real part): the sum over w-layers (eq. 7) needs no read-modify-write and no
// atomics.  With stamps, the channel's last workgroup records the device clock.
template <int N>
__global__ __launch_bounds__(RowPlan<N>::NT) void k_inv_rows_sweep(
    const SweepLayer* __restrict__ sl, const int2* __restrict__ chan_layers, int c0,
    void* __restrict__ out, const float2* __restrict__ tw, const float* __restrict__ sx,
    const float* __restrict__ sy, int nx, int ny, double cell, int real_out,
    unsigned long long* __restrict__ stamps, int* __restrict__ done) {
  using RP = RowPlan<N>;
  constexpr int R1 = RP::R1, R2 = RP::R2, R3 = RP::R3, NT = RP::NT;
  constexpr int NS3 = R1 * R2;
  constexpr int B3 = (N / R3) / NT;
  extern __shared__ float2 buf[];
  const int jr = blockIdx.x, c = c0 + (int)blockIdx.y;
  const int2 cl = chan_layers[c];
  const float syj = sy[jr];
  float2 acc[B3][R3 / 2];
#pragma unroll
  for (int b = 0; b < B3; ++b)
#pragma unroll
    for (int r = 0; r < R3 / 2; ++r) acc[b][r] = make_float2(0.f, 0.f);
  for (int li = cl.x; li < cl.x + cl.y; ++li) {
    const SweepLayer& L = sl[li];
    const float2* __restrict__ A = L.A;
    const uint32_t* __restrict__ smask = L.smask;
    float2 v1[N / NT];
    {
      constexpr int B = (N / R1) / NT;
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int j = threadIdx.x + b * NT;
        float2* v = v1 + b * R1;
#pragma unroll
        for (int r = 0; r < R1; ++r) {
          const int q = j + r * (N / R1);
          v[r] = (!smask || strip_on<N / R1>(smask, j, r)) ? A[strip_index(jr, q, ny)]
                                                           : make_float2(0.f, 0.f);
        }
        dft_reg<R1, true>(v);
      }
    }
    float2 v3[N / NT];
    row_middle<N, true>(buf, v1, v3, tw, threadIdx.x);
#pragma unroll
    for (int b = 0; b < B3; ++b) {
      const int j = threadIdx.x + b * NT;
      float2* v = v3 + b * R3;
#pragma unroll
      for (int r = 1; r < R3; ++r) v[r] = cmulc(v[r], tw[r * j]);
      dft_reg<R3, true>(v);
#pragma unroll
      for (int r = 0; r < R3; ++r) {
        if (r < R3 / 4 || r >= 3 * R3 / 4) {
          const int q = j + r * NS3;
          const int i = r < R3 / 4 ? q + nx / 2 : q - 3 * (nx / 2);
          const float2 z = zvalue(i, jr, nx, ny, cell, L.wp, sx[i], syj);
          const float2 t = cmulc(v[r], z);
          float2& a = acc[b][r < R3 / 4 ? r : r - R3 / 2];
          a = make_float2(a.x + t.x, a.y + t.y);
        }
      }
    }
  }
  const int64_t base = (int64_t)c * nx * ny + (int64_t)jr * nx;
#pragma unroll
  for (int b = 0; b < B3; ++b) {
    const int j = threadIdx.x + b * NT;
#pragma unroll
    for (int r = 0; r < R3; ++r) {
      if (r < R3 / 4 || r >= 3 * R3 / 4) {
        const int q = j + r * NS3;
        const int i = r < R3 / 4 ? q + nx / 2 : q - 3 * (nx / 2);
        const float2 a = acc[b][r < R3 / 4 ? r : r - R3 / 2];
        if (real_out) reinterpret_cast<float*>(out)[base + i] = a.x;
        else reinterpret_cast<float2*>(out)[base + i] = a;
      }
    }
  }
  if (stamps) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0 && atomicAdd(done + c, 1) == (int)gridDim.x - 1) {
      stamps[c] = wall_clock64();
      atomicExch(done + c, 0);
    }
  }
}

// Column passes at the long lengths (N = 2048 .. 16384), register-resident like the row
// passes: CW columns of one strip per workgroup, NT threads per column, interleaved so
// that the CW columns of one grid row are read and written by neighbouring lanes.  The
// needed tiles of the group's column of tiles are copied into LDS flags once, so that no
// element waits on a mask load.  Since N = 2 ny, the zero half of each forward column and
// the discarded half of each inverse column follow the same compile-time rule as rows.
template <int N>
struct ColPlan {
  static constexpr int CW = (16384 / N) > 16 ? 16 : (16384 / N);
  static constexpr int NTC = RowPlan<N>::NT;   // threads per column
  static constexpr int NT = CW * NTC;
  // The CW columns of one grid row sit on neighbouring lanes.  An LDS access of 64 lanes
  // is served in halves of 32 lanes, i.e. 32 / CW consecutive elements of each of CW
  // lines: lines 32 / CW elements apart beyond their padded length (which is a multiple
  // of 32) put those CW runs on disjoint banks.
  static constexpr int LS = lds_elems<N>() + 32 / CW;
  // CW lines of LS complex values, or of LS floats where lines cross LDS in halves
  // (xchg_split, line_split), then the tile flags
  static constexpr size_t lds_bytes() {
    return (size_t)CW * LS * (line_split<N>() ? sizeof(float) : sizeof(float2)) + N / 8;
  }
};

// Flags of the needed tiles of column-tile ct (one byte per row of tiles; all ones when
// there is no mask).
__device__ __forceinline__ void load_tile_flags(uint8_t* flags, const Masks& mk, int N, int ct,
                                                int nthreads) {
  const int nty = (N >> mk.tsh) > 0 ? (N >> mk.tsh) : 1;
  for (int t = threadIdx.x; t < nty; t += nthreads)
    flags[t] = mk.tile ? (uint8_t)bit_set(mk.tile, t * mk.tiles_x + ct) : (uint8_t)1;
}

// Needed-tile bits of a forward column pass's outputs.  The last pass writes outputs
// j + r NS (j < NS = R1 R2, r < R3), whose tile rows are t0 + r S with t0 = j >> tsh and
// S = NS >> tsh (a mask's tile, at most 128, never exceeds NS): entry t0 holds bit r for
// each r, so that a butterfly reads one word instead of R3 flags.  Without a mask every
// entry a butterfly can read (one when tsh exceeds the line) has every bit set.
template <int N>
__device__ __forceinline__ void load_out_tile_bits(uint32_t* bits, const Masks& mk, int ct,
                                                   int nthreads) {
  constexpr int NS = RowPlan<N>::R1 * RowPlan<N>::R2, R3 = RowPlan<N>::R3;
  static_assert(R3 <= 32, "one word per entry");
  const int S = (NS >> mk.tsh) > 0 ? (NS >> mk.tsh) : 1;
  for (int t0 = threadIdx.x; t0 < S; t0 += nthreads) {
    uint32_t m = 0xffffffffu;
    if (mk.tile) {
      m = 0;
      for (int r = 0; r < R3; ++r)
        m |= (uint32_t)bit_set(mk.tile, (t0 + r * S) * mk.tiles_x + ct) << r;
    }
    bits[t0] = m;
  }
}

// With a sweep's layer table sl, workgroup i takes (layer, column group) pairs[i].
template <int N>
__global__ __launch_bounds__(ColPlan<N>::NT) __attribute__((amdgpu_waves_per_eu(4))) void k_fwd_cols_reg(const float2* __restrict__ A,
                                                                 float2* __restrict__ X,
                                                                 const float2* __restrict__ tw,
                                                                 int ny, Masks mk,
                                                                 const SweepLayer* __restrict__ sl,
                                                                 const int2* __restrict__ pairs) {
  using RP = RowPlan<N>;
  constexpr int R1 = RP::R1, R2 = RP::R2, R3 = RP::R3;
  constexpr int CW = ColPlan<N>::CW, NTC = ColPlan<N>::NTC, NT = ColPlan<N>::NT;
  constexpr int LS = ColPlan<N>::LS;
  extern __shared__ float2 buf[];
  // CW lines of LS floats (split exchange) or complex values, then the output tile bits
  constexpr bool SPLIT = line_split<N>();
  uint32_t* omask = SPLIT ? reinterpret_cast<uint32_t*>(reinterpret_cast<float*>(buf) + CW * LS)
                          : reinterpret_cast<uint32_t*>(buf + CW * LS);
  const int gi = xcd_remap(blockIdx.x, gridDim.x);
  int g;
  if (sl) {
    const int2 pr = pairs[gi];
    const SweepLayer& L = sl[pr.x];
    A = L.A;
    X = L.X;
    mk.tile = L.tile;
    g = pr.y;
  } else {
    g = mk.groups ? mk.groups[gi] : gi;
  }
  const int q0 = g * CW;
  const int strip = q0 >> 4, c0 = q0 & (SW - 1);
  const int c = threadIdx.x % CW, tj = threadIdx.x / CW;
  void* line = SPLIT ? (void*)(reinterpret_cast<float*>(buf) + c * LS) : (void*)(buf + c * LS);
  // the bits are read after the exchanges' barriers only
  load_out_tile_bits<N>(omask, mk, q0 >> mk.tsh, NT);
  // wave-uniform bases and 32-bit element offsets (a strip holds at most 16 N elements)
  const float2* __restrict__ src = A + ((int64_t)strip * ny) * SW + c0;
  float2 v1[N / NTC];
  {
    constexpr int B = (N / R1) / NTC;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = tj + b * NTC;
      float2* v = v1 + b * R1;
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int q = j + r * (N / R1);
        if (r < R1 / 4 || r >= 3 * R1 / 4) {
          const int jrow = r < R1 / 4 ? q + N / 4 : q - 3 * (N / 4);
          v[r] = src[jrow * SW + c];
        } else {
          v[r] = make_float2(0.f, 0.f);
        }
      }
      dft_reg<R1, false>(v);
    }
  }
  float2 v3[N / NTC];
  row_middle<N, false>(line, v1, v3, tw, tj);
  float2* __restrict__ dst = X + ((int64_t)strip * N) * SW + c0;
  {
    // the lane's column and butterfly index are taken afresh from the thread index (the
    // empty asm hides that it is unchanged) rather than held through the exchanges
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int cl = tid % CW, tl = tid / CW;
    constexpr int NS = R1 * R2;
    constexpr int B = (N / R3) / NTC;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = tl + b * NTC;
      float2* v = v3 + b * R3;
#pragma unroll
      for (int r = 1; r < R3; ++r) v[r] = cmul(v[r], tw[r * j]);
      dft_reg<R3, false>(v);
      const uint32_t need = omask[j >> mk.tsh];
#pragma unroll
      for (int r = 0; r < R3; ++r) {
        if ((need >> r) & 1u) dst[(j + r * NS) * SW + cl] = v[r];
      }
    }
  }
}

template <int N>
__global__ __launch_bounds__(ColPlan<N>::NT) __attribute__((amdgpu_waves_per_eu(4))) void k_inv_cols_reg(float2* __restrict__ Y,
                                                                 float2* __restrict__ A,
                                                                 const float2* __restrict__ tw,
                                                                 int ny, Masks mk,
                                                                 const SweepLayer* __restrict__ sl,
                                                                 const int2* __restrict__ pairs) {
  using RP = RowPlan<N>;
  constexpr int R1 = RP::R1, R2 = RP::R2, R3 = RP::R3;
  constexpr int CW = ColPlan<N>::CW, NTC = ColPlan<N>::NTC, NT = ColPlan<N>::NT;
  constexpr int LS = ColPlan<N>::LS;
  extern __shared__ float2 buf[];
  // CW lines of LS floats (split exchange) or complex values, then the tile flags
  constexpr bool SPLIT = line_split<N>();
  uint8_t* tflag = SPLIT ? reinterpret_cast<uint8_t*>(reinterpret_cast<float*>(buf) + CW * LS)
                         : reinterpret_cast<uint8_t*>(buf + CW * LS);
  const int gi = xcd_remap(blockIdx.x, gridDim.x);
  int g;
  if (sl) {
    const int2 pr = pairs[gi];
    const SweepLayer& L = sl[pr.x];
    Y = L.Y;
    A = L.A;
    mk.tile = L.tile;
    g = pr.y;
  } else {
    g = mk.groups ? mk.groups[gi] : gi;
  }
  const int q0 = g * CW;
  const int strip = q0 >> 4, c0 = q0 & (SW - 1);
  const int c = threadIdx.x % CW, tj = threadIdx.x / CW;
  void* line = SPLIT ? (void*)(reinterpret_cast<float*>(buf) + c * LS) : (void*)(buf + c * LS);
  load_tile_flags(tflag, mk, N, q0 >> mk.tsh, NT);
  __syncthreads();
  // Y is read only inside needed tiles and cleared behind the read, ready for the next
  // gridding; elsewhere it is zero already
  float2* __restrict__ src = Y + ((int64_t)strip * N) * SW + c0 + c;
  float2 v1[N / NTC];
  {
    constexpr int B = (N / R1) / NTC;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = tj + b * NTC;
      float2* v = v1 + b * R1;
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int q = j + r * (N / R1);
        v[r] = make_float2(0.f, 0.f);
        if (tflag[q >> mk.tsh]) {
          v[r] = src[(int64_t)q * SW];
          src[(int64_t)q * SW] = make_float2(0.f, 0.f);
        }
      }
      dft_reg<R1, true>(v);
    }
  }
  float2 v3[N / NTC];
  row_middle<N, true>(line, v1, v3, tw, tj);
  float2* __restrict__ dst = A + ((int64_t)strip * ny) * SW + c0 + c;
  {
    constexpr int NS = R1 * R2;
    constexpr int B = (N / R3) / NTC;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = tj + b * NTC;
      float2* v = v3 + b * R3;
#pragma unroll
      for (int r = 1; r < R3; ++r) v[r] = cmulc(v[r], tw[r * j]);
      dft_reg<R3, true>(v);
#pragma unroll
      for (int r = 0; r < R3; ++r) {
        if (r < R3 / 4 || r >= 3 * R3 / 4) {
          const int q = j + r * NS;
          const int jrow = r < R3 / 4 ? q + N / 4 : q - 3 * (N / 4);
          dst[(int64_t)jrow * SW] = v[r];
        }
      }
    }
  }
}

// Column passes: CW adjacent columns of one strip per workgroup, lines padded by one
// element in LDS so that the strip-order global accesses (column index fastest) hit
// distinct banks.
template <int N, int NT, int CW>
__global__ __launch_bounds__(NT) void k_fwd_cols(const float2* __restrict__ A,
                                                 float2* __restrict__ X,
                                                 const float2* __restrict__ tw, int ny,
                                                 Masks mk) {
  extern __shared__ float2 buf[];
  constexpr int S = N + 1;
  const int gi = xcd_remap(blockIdx.x, gridDim.x);
  const int g = mk.groups ? mk.groups[gi] : gi;
  const int q0 = g * CW;
  const int strip = q0 >> 4, c0 = q0 & (SW - 1);
  const int nz = N - ny;
  for (int t = threadIdx.x; t < CW * nz; t += NT) {
    const int c = t / nz, r = t - c * nz;
    buf[c * S + ny / 2 + r] = make_float2(0.f, 0.f);
  }
  const float2* src = A + ((int64_t)strip * ny) * SW + c0;
  for (int t = threadIdx.x; t < CW * ny; t += NT) {
    const int jr = t / CW, c = t - jr * CW;
    buf[c * S + ((jr - ny / 2) & (N - 1))] = src[(int64_t)jr * SW + c];
  }
  __syncthreads();
  fft_lines<N, NT, CW, false>(buf, S, tw);
  float2* dst = X + ((int64_t)strip * N) * SW + c0;
  for (int t = threadIdx.x; t < CW * N; t += NT) {
    const int qv = t / CW, c = t - qv * CW;
    if (!mk.tile || bit_set(mk.tile, (qv >> mk.tsh) * mk.tiles_x + ((q0 + c) >> mk.tsh)))
      dst[(int64_t)qv * SW + c] = buf[c * S + qv];
  }
}

template <int N, int NT, int CW>
__global__ __launch_bounds__(NT) void k_inv_cols(float2* __restrict__ Y, float2* __restrict__ A,
                                                 const float2* __restrict__ tw, int ny,
                                                 Masks mk) {
  extern __shared__ float2 buf[];
  constexpr int S = N + 1;
  const int gi = xcd_remap(blockIdx.x, gridDim.x);
  const int g = mk.groups ? mk.groups[gi] : gi;
  const int q0 = g * CW;
  const int strip = q0 >> 4, c0 = q0 & (SW - 1);
  float2* src = Y + ((int64_t)strip * N) * SW + c0;
  for (int t = threadIdx.x; t < CW * N; t += NT) {
    const int qv = t / CW, c = t - qv * CW;
    float2* p = src + (int64_t)qv * SW + c;
    if (!mk.tile || bit_set(mk.tile, (qv >> mk.tsh) * mk.tiles_x + ((q0 + c) >> mk.tsh))) {
      buf[c * S + qv] = *p;
      *p = make_float2(0.f, 0.f);
    } else {
      buf[c * S + qv] = make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  fft_lines<N, NT, CW, true>(buf, S, tw);
  float2* dst = A + ((int64_t)strip * ny) * SW + c0;
  for (int t = threadIdx.x; t < CW * ny; t += NT) {
    const int jr = t / CW, c = t - jr * CW;
    dst[(int64_t)jr * SW + c] = buf[c * S + ((jr - ny / 2) & (N - 1))];
  }
}

__global__ void k_strip_to_rowmajor(const float2* __restrict__ src, float2* __restrict__ dst,
                                    int R, int Q) {
  const int64_t n = (int64_t)R * Q;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(t / Q), q = (int)(t - (int64_t)r * Q);
    dst[t] = src[strip_index(r, q, R)];
  }
}

// ------------------------------------------------------------------ launchers

// Raise a kernel's dynamic LDS limit once per (kernel, device, size), so that launches
// issued later (also inside a stream capture) make no attribute call.
template <typename K>
static hipError_t set_lds(K kern, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  struct Done {
    const void* k;
    int dev;
    size_t bytes;
  };
  static std::mutex mu;
  static std::vector<Done> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const void* k = reinterpret_cast<const void*>(kern);
  std::lock_guard<std::mutex> lock(mu);
  for (const Done& d : done)
    if (d.k == k && d.dev == dev && d.bytes >= bytes) return hipSuccess;
  e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) done.push_back(Done{k, dev, bytes});
  return e;
}

#define WF_FOR_SIZES(X) \
  X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192) X(16384)

template <int N>
static hipError_t launch_fwd_rows_reg(const float* img, float2* A, const float2* tw,
                                      const float* sx, const float* sy, int nx, int ny,
                                      double cell, double wp, const uint32_t* smask,
                                      const float2* ctab, hipStream_t s) {
  const size_t lds = line_lds_bytes<N>();
  hipError_t e = set_lds(k_fwd_rows_reg<N>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fwd_rows_reg<N>), dim3(ny), dim3(RowPlan<N>::NT), lds, s, img, A, tw,
                     sx, sy, nx, ny, cell, wp, smask, nullptr, ctab);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_inv_rows_reg(const float2* A, void* out, const float2* tw,
                                      const float* sx, const float* sy, int nx, int ny,
                                      double cell, double wp, int mode, const uint32_t* smask,
                                      const float2* ctab, hipStream_t s) {
  const size_t lds = line_lds_bytes<N>();
  hipError_t e = set_lds(k_inv_rows_reg<N>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_inv_rows_reg<N>), dim3(ny), dim3(RowPlan<N>::NT), lds, s, A, out, tw,
                     sx, sy, nx, ny, cell, wp, mode, smask, ctab);
  return hipGetLastError();
}

hipError_t launch_chirp_table(float2* ct, int nx, double cell, double wp, const float* sx,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_chirp_table, dim3((nx + 255) / 256), dim3(256), 0, s, ct, nx, cell, wp,
                     sx);
  return hipGetLastError();
}

hipError_t launch_fwd_rows(const float* img, float2* A, const float2* tw, const float* sx,
                           const float* sy, int nx, int ny, int Kx, double cell, double wp,
                           const uint32_t* smask, const float2* ctab, hipStream_t s) {
  if (Kx == 2 * nx) {
    switch (Kx) {
      case 2048: return launch_fwd_rows_reg<2048>(img, A, tw, sx, sy, nx, ny, cell, wp, smask, ctab, s);
      case 4096: return launch_fwd_rows_reg<4096>(img, A, tw, sx, sy, nx, ny, cell, wp, smask, ctab, s);
      case 8192: return launch_fwd_rows_reg<8192>(img, A, tw, sx, sy, nx, ny, cell, wp, smask, ctab, s);
      case 16384: return launch_fwd_rows_reg<16384>(img, A, tw, sx, sy, nx, ny, cell, wp, smask, ctab, s);
      default: break;
    }
  }
  switch (Kx) {
#define C(N)                                                                              \
  case N: {                                                                               \
    constexpr int NT = row_threads<N>();                                                  \
    const size_t lds = (size_t)N * sizeof(float2);                                        \
    hipError_t e = set_lds(k_fwd_rows<N, NT>, lds);                                       \
    if (e != hipSuccess) return e;                                                        \
    hipLaunchKernelGGL((k_fwd_rows<N, NT>), dim3(ny), dim3(NT), lds, s, img, A, tw, sx,  \
                       sy, nx, ny, cell, wp, smask);                                      \
    return hipGetLastError();                                                             \
  }
    WF_FOR_SIZES(C)
#undef C
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_inv_rows(const float2* A, void* out, const float2* tw, const float* sx,
                           const float* sy, int nx, int ny, int Kx, double cell, double wp,
                           int mode, const uint32_t* smask, const float2* ctab,
                           hipStream_t s) {
  if (Kx == 2 * nx) {
    switch (Kx) {
      case 2048: return launch_inv_rows_reg<2048>(A, out, tw, sx, sy, nx, ny, cell, wp, mode, smask, ctab, s);
      case 4096: return launch_inv_rows_reg<4096>(A, out, tw, sx, sy, nx, ny, cell, wp, mode, smask, ctab, s);
      case 8192: return launch_inv_rows_reg<8192>(A, out, tw, sx, sy, nx, ny, cell, wp, mode, smask, ctab, s);
      case 16384: return launch_inv_rows_reg<16384>(A, out, tw, sx, sy, nx, ny, cell, wp, mode, smask, ctab, s);
      default: break;
    }
  }
  switch (Kx) {
#define C(N)                                                                              \
  case N: {                                                                               \
    constexpr int NT = row_threads<N>();                                                  \
    const size_t lds = (size_t)N * sizeof(float2);                                        \
    hipError_t e = set_lds(k_inv_rows<N, NT>, lds);                                       \
    if (e != hipSuccess) return e;                                                        \
    hipLaunchKernelGGL((k_inv_rows<N, NT>), dim3(ny), dim3(NT), lds, s, A, out, tw, sx,  \
                       sy, nx, ny, cell, wp, mode, smask);                                \
    return hipGetLastError();                                                             \
  }
    WF_FOR_SIZES(C)
#undef C
    default:
      return hipErrorInvalidValue;
  }
}

template <int N, bool INV>
static hipError_t launch_cols_reg(float2* in, float2* out, const float2* tw, int ny, int Kx,
                                  const ColPrune* pr, hipStream_t s) {
  constexpr int CW = ColPlan<N>::CW;
  if (Kx % CW != 0) return hipErrorInvalidValue;
  const size_t lds = ColPlan<N>::lds_bytes();
  Masks mk{nullptr, nullptr, nullptr, 1, 0};
  int ng = Kx / CW;
  if (pr) {
    mk = Masks{pr->strip, pr->tile, pr->groups, pr->tiles_x, pr->tsh};
    ng = pr->ngroups;
  }
  if (!pr || !pr->tile) {   // no mask: one row of tiles of any side
    mk.tsh = 30;
  }
  if (ng == 0) return hipSuccess;
  hipError_t e;
  if constexpr (INV) {
    e = set_lds(k_inv_cols_reg<N>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_inv_cols_reg<N>), dim3(ng), dim3(ColPlan<N>::NT), lds, s, in, out, tw,
                       ny, mk, nullptr, nullptr);
  } else {
    e = set_lds(k_fwd_cols_reg<N>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fwd_cols_reg<N>), dim3(ng), dim3(ColPlan<N>::NT), lds, s,
                       (const float2*)in, out, tw, ny, mk, nullptr, nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_fwd_cols(const float2* A, float2* X, const float2* tw, int ny, int Kx,
                           int Ky, const ColPrune* pr, hipStream_t s) {
  if (Ky == 2 * ny) {
    float2* a = const_cast<float2*>(A);
    switch (Ky) {
      case 2048: return launch_cols_reg<2048, false>(a, X, tw, ny, Kx, pr, s);
      case 4096: return launch_cols_reg<4096, false>(a, X, tw, ny, Kx, pr, s);
      case 8192: return launch_cols_reg<8192, false>(a, X, tw, ny, Kx, pr, s);
      case 16384: return launch_cols_reg<16384, false>(a, X, tw, ny, Kx, pr, s);
      default: break;
    }
  }
  switch (Ky) {
#define C(N)                                                                              \
  case N: {                                                                               \
    constexpr int CW = col_width<N>();                                                    \
    constexpr int NT = col_threads<N>();                                                  \
    if (Kx % CW != 0) return hipErrorInvalidValue;                                        \
    const size_t lds = (size_t)CW * (N + 1) * sizeof(float2);                             \
    hipError_t e = set_lds(k_fwd_cols<N, NT, CW>, lds);                                   \
    if (e != hipSuccess) return e;                                                        \
    Masks mk{nullptr, nullptr, nullptr, 1, 0};                                            \
    int ng = Kx / CW;                                                                     \
    if (pr) {                                                                             \
      mk = Masks{pr->strip, pr->tile, pr->groups, pr->tiles_x, pr->tsh};                  \
      ng = pr->ngroups;                                                                   \
    }                                                                                     \
    if (ng == 0) return hipSuccess;                                                       \
    hipLaunchKernelGGL((k_fwd_cols<N, NT, CW>), dim3(ng), dim3(NT), lds, s, A, X, tw, ny, \
                       mk);                                                               \
    return hipGetLastError();                                                             \
  }
    WF_FOR_SIZES(C)
#undef C
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_inv_cols(float2* Y, float2* A, const float2* tw, int ny, int Kx, int Ky,
                           const ColPrune* pr, hipStream_t s) {
  if (Ky == 2 * ny) {
    switch (Ky) {
      case 2048: return launch_cols_reg<2048, true>(Y, A, tw, ny, Kx, pr, s);
      case 4096: return launch_cols_reg<4096, true>(Y, A, tw, ny, Kx, pr, s);
      case 8192: return launch_cols_reg<8192, true>(Y, A, tw, ny, Kx, pr, s);
      case 16384: return launch_cols_reg<16384, true>(Y, A, tw, ny, Kx, pr, s);
      default: break;
    }
  }
  switch (Ky) {
#define C(N)                                                                              \
  case N: {                                                                               \
    constexpr int CW = col_width<N>();                                                    \
    constexpr int NT = col_threads<N>();                                                  \
    if (Kx % CW != 0) return hipErrorInvalidValue;                                        \
    const size_t lds = (size_t)CW * (N + 1) * sizeof(float2);                             \
    hipError_t e = set_lds(k_inv_cols<N, NT, CW>, lds);                                   \
    if (e != hipSuccess) return e;                                                        \
    Masks mk{nullptr, nullptr, nullptr, 1, 0};                                            \
    int ng = Kx / CW;                                                                     \
    if (pr) {                                                                             \
      mk = Masks{pr->strip, pr->tile, pr->groups, pr->tiles_x, pr->tsh};                  \
      ng = pr->ngroups;                                                                   \
    }                                                                                     \
    if (ng == 0) return hipSuccess;                                                       \
    hipLaunchKernelGGL((k_inv_cols<N, NT, CW>), dim3(ng), dim3(NT), lds, s, Y, A, tw, ny, \
                       mk);                                                               \
    return hipGetLastError();                                                             \
  }
    WF_FOR_SIZES(C)
#undef C
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_strip_to_rowmajor(const float2* src, float2* dst, int R, int Q,
                                    hipStream_t s) {
  const int64_t n = (int64_t)R * Q;
  const int blocks = (int)((n + 255) / 256 > 65536 ? 65536 : (n + 255) / 256);
  hipLaunchKernelGGL(k_strip_to_rowmajor, dim3(blocks), dim3(256), 0, s, src, dst, R, Q);
  return hipGetLastError();
}

// ------------------------------------------------------------------ sweep stages
// One launch per stage over every layer of a sweep (grid sides 2048 .. 16384, Kx = 2 nx,
// Ky = 2 ny).  Layer tables and pairs are device arrays built by the host.

hipError_t launch_sweep_fwd_rows(const float* img, const SweepLayer* sl, int nlayers,
                                 const float2* tw, const float* sx, const float* sy, int nx,
                                 int ny, int Kx, double cell, hipStream_t s) {
  if (nlayers <= 0) return hipSuccess;
  switch (Kx) {
#define C(NN)                                                                               \
  case NN: {                                                                                \
    const size_t lds = line_lds_bytes<NN>();                                            \
    hipError_t e = set_lds(k_fwd_rows_reg<NN>, lds);                                        \
    if (e != hipSuccess) return e;                                                          \
    hipLaunchKernelGGL((k_fwd_rows_reg<NN>), dim3(ny, nlayers), dim3(RowPlan<NN>::NT), lds, \
                       s, img, nullptr, tw, sx, sy, nx, ny, cell, 0.0, nullptr, sl,        \
                       nullptr);                                                            \
    return hipGetLastError();                                                               \
  }
    C(2048) C(4096) C(8192) C(16384)
#undef C
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_sweep_cols(bool inverse, const SweepLayer* sl, const int2* pairs, int npairs,
                             const float2* tw, int ny, int Ky, int tsh, int tiles_x,
                             hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  Masks mk{nullptr, nullptr, nullptr, tiles_x, tsh};
  switch (Ky) {
#define C(NN)                                                                                 \
  case NN: {                                                                                  \
    const size_t lds = ColPlan<NN>::lds_bytes();                                       \
    hipError_t e;                                                                             \
    if (inverse) {                                                                            \
      e = set_lds(k_inv_cols_reg<NN>, lds);                                                   \
      if (e != hipSuccess) return e;                                                          \
      hipLaunchKernelGGL((k_inv_cols_reg<NN>), dim3(npairs), dim3(ColPlan<NN>::NT), lds, s,   \
                         nullptr, nullptr, tw, ny, mk, sl, pairs);                            \
    } else {                                                                                  \
      e = set_lds(k_fwd_cols_reg<NN>, lds);                                                   \
      if (e != hipSuccess) return e;                                                          \
      hipLaunchKernelGGL((k_fwd_cols_reg<NN>), dim3(npairs), dim3(ColPlan<NN>::NT), lds, s,   \
                         nullptr, nullptr, tw, ny, mk, sl, pairs);                            \
    }                                                                                         \
    return hipGetLastError();                                                                 \
  }
    C(2048) C(4096) C(8192) C(16384)
#undef C
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_sweep_inv_rows(const SweepLayer* sl, const int2* chan_layers, int c0,
                                 int nchan, void* out, bool real_out, const float2* tw,
                                 const float* sx,
                                 const float* sy, int nx, int ny, int Kx, double cell,
                                 unsigned long long* stamps, int* done, hipStream_t s) {
  if (nchan <= 0) return hipSuccess;
  switch (Kx) {
#define C(NN)                                                                                \
  case NN: {                                                                                 \
    const size_t lds = line_lds_bytes<NN>();                                            \
    hipError_t e = set_lds(k_inv_rows_sweep<NN>, lds);                                       \
    if (e != hipSuccess) return e;                                                           \
    hipLaunchKernelGGL((k_inv_rows_sweep<NN>), dim3(ny, nchan), dim3(RowPlan<NN>::NT), lds,  \
                       s, sl, chan_layers, c0, out, tw, sx, sy, nx, ny, cell,              \
                       real_out ? 1 : 0, stamps, done);                                      \
    return hipGetLastError();                                                                \
  }
    C(2048) C(4096) C(8192) C(16384)
#undef C
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace wf
