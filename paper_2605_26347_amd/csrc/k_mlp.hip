// Kernels of the residual-kernel network (not part of the paper): FP32 training on the
// matrix cores (GEMMs with fused bias / GELU epilogues, GELU backward, column sums,
// loss, Adam) and fused BF16 inference.
//
// GEMM tiles: a workgroup of four wavefronts computes a 64 x 64 block of C, each
// wavefront one 32 x 32 quadrant with v_mfma_f32_32x32x2f32 (lane l supplies
// A[l % 32][l / 32] and B[l / 32][l % 32] of a 32 x 2 x 32 step; accumulator element i
// of lane l is C[8 (i / 4) + 4 (l / 32) + i % 4][l % 32]).  Operands are staged through
// LDS in chunks of 32 along K, k-major, so that both operands are read as 32
// consecutive floats per half-wave.
//
// Inference: one workgroup of four wavefronts carries 64 rows through the whole network
// with the activations in LDS as BF16.  The first layer (5 inputs) runs in FP32 so that
// the inputs keep their precision; the hidden and output layers use
// v_mfma_f32_32x32x16_bf16 (lane l supplies A[l % 32][8 (l / 32) .. + 7] and
// B[8 (l / 32) .. + 7][l % 32]) with FP32 accumulation, weights read from a transposed
// BF16 copy that stays resident in L2.  Plain BF16 operands leave a relative output error
// near 1e-3; the split form (hi + lo BF16 parts, three products per step) brings it to
// the FP32 level at three times the matrix-core work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "mlp_defs.h"
#include "wf_internal.h"

namespace wf {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.7071067811865475f));
}
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.7071067811865475f)) +
         z * 0.3989422804014327f * __expf(-0.5f * z * z);
}

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t b = __float_as_uint(f);
  return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

constexpr int GT = 64;   // C tile side
constexpr int GK = 32;   // K chunk

// C[M x N] = op(A)[M x K] op(B)[K x N]; EPI 0: C = acc; 1: Z = acc + bias, C = gelu(Z);
// 2: C = acc + bias; 3: C += acc atomically (split K: blockIdx.z takes K range
// [z kc, (z + 1) kc)).  op(A) = A^T when TA (A stored [K x M]), likewise for B.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const float* __restrict__ A, int lda,
                                              const float* __restrict__ B, int ldb,
                                              float* __restrict__ C, int ldc,
                                              float* __restrict__ Z,
                                              const float* __restrict__ bias, int M, int N,
                                              int K, int kc) {
  __shared__ float As[GK][GT + 4];
  __shared__ float Bs[GK][GT + 4];
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int kb = blockIdx.z * kc;
  const int ke = min(K, kb + kc);
  f32x16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  for (int k0 = kb; k0 < ke; k0 += GK) {
    for (int i = tid; i < GT * GK; i += 256) {
      int m, k;
      if (TA) {
        k = i / GT;
        m = i - k * GT;
      } else {
        m = i / GK;
        k = i - m * GK;
      }
      const int gm = m0 + m, gk = k0 + k;
      float v = 0.f;
      if (gm < M && gk < ke) v = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      As[k][m] = v;
    }
    for (int i = tid; i < GT * GK; i += 256) {
      int n, k;
      if (TB) {
        n = i / GK;
        k = i - n * GK;
      } else {
        k = i / GT;
        n = i - k * GT;
      }
      const int gn = n0 + n, gk = k0 + k;
      float v = 0.f;
      if (gn < N && gk < ke) v = TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
      Bs[k][n] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; kk += 2) {
      const float a = As[kk + (lane >> 5)][wm * 32 + (lane & 31)];
      const float b = Bs[kk + (lane >> 5)][wn * 32 + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int col = n0 + wn * 32 + (lane & 31);
  if (col >= N) return;
  const float bb = (EPI == 1 || EPI == 2) ? bias[col] : 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = m0 + wm * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
    if (row >= M) continue;
    const float v = acc[i] + bb;
    if (EPI == 1) {
      Z[(int64_t)row * ldc + col] = v;
      C[(int64_t)row * ldc + col] = gelu(v);
    } else if (EPI == 3) {
      atomicAdd(&C[(int64_t)row * ldc + col], v);
    } else {
      C[(int64_t)row * ldc + col] = v;
    }
  }
}

__global__ __launch_bounds__(256) void k_gelu_bwd(float* __restrict__ dH,
                                                  const float* __restrict__ Z, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dH[i] *= gelu_grad(Z[i]);
}

// db[c] += sum over rows [256 blockIdx.y, 256 blockIdx.y + 256) of D[r][c] (D [rows x N],
// row stride ld; db cleared by the caller); 64 columns per block, four row phases
// reduced in LDS.
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ D, int ld, int rows,
                                                int N, float* __restrict__ db) {
  __shared__ float part[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
  const int r0 = blockIdx.y * 256, r1 = min(rows, r0 + 256);
  float s = 0.f;
  if (c < N)
    for (int r = r0 + ph; r < r1; r += 4) s += D[(int64_t)r * ld + c];
  part[ph][threadIdx.x & 63] = s;
  __syncthreads();
  if (ph == 0 && c < N)
    atomicAdd(&db[c], (part[0][threadIdx.x] + part[1][threadIdx.x]) +
                          (part[2][threadIdx.x] + part[3][threadIdx.x]));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Loss of one batch, one wavefront per example: dP = 2 (P - T) / B on the kernel
// outputs, 2 (e - log10(max(r, 1e-8))) / B on the error output with r held constant;
// loss[0] += kernel loss, loss[1] += error-output loss.
__global__ __launch_bounds__(64) void k_loss(const float* __restrict__ P,
                                             const float* __restrict__ T, float* __restrict__ dP,
                                             int B, float* __restrict__ loss) {
  const int b = blockIdx.x, lane = threadIdx.x;
  const float* p = P + (int64_t)b * MLP_OUT;
  const float* t = T + (int64_t)b * MLP_KOUT;
  float* d = dP + (int64_t)b * MLP_OUT;
  const float inv = 2.0f / (float)B;
  float s = 0.f, st = 0.f;
  for (int j = lane; j < MLP_KOUT; j += 64) {
    const float e = p[j] - t[j];
    s += e * e;
    st += t[j] * t[j];
    d[j] = inv * e;
  }
  s = wave_sum(s);
  st = wave_sum(st);
  if (lane == 0) {
    const float r = sqrtf(s) / fmaxf(sqrtf(st), 1e-30f);
    const float tgt = log10f(fmaxf(r, 1e-8f));
    const float e = p[MLP_KOUT] - tgt;
    d[MLP_KOUT] = inv * e;
    atomicAdd(&loss[0], s / (float)B);
    atomicAdd(&loss[1], e * e / (float)B);
  }
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Minibatch gather of rows idx[0..B) of X [n x cx] and T [n x ct].
__global__ __launch_bounds__(256) void k_gather(const float* __restrict__ X, int cx,
                                                const float* __restrict__ T, int ct,
                                                const int32_t* __restrict__ idx, int B,
                                                float* __restrict__ xb, float* __restrict__ tb) {
  const int b = blockIdx.x;
  const int64_t r = idx[b];
  for (int j = threadIdx.x; j < cx; j += blockDim.x) xb[(int64_t)b * cx + j] = X[r * cx + j];
  for (int j = threadIdx.x; j < ct; j += blockDim.x) tb[(int64_t)b * ct + j] = T[r * ct + j];
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int64_t WT_HALF = 3LL * MLP_HID * MLP_HID + 512LL * MLP_HID;

// Transposed BF16 copies of the hidden and output weights: layer l = 1..4 goes to
// wt + (l - 1) * 256 * 256 as [n][k] (the output layer padded to 512 rows of zeros); the
// second half holds the residuals w - bf16(w), also in BF16 (the low parts of the split
// operands).
__global__ __launch_bounds__(256) void k_prep_bf16(const float* __restrict__ params,
                                                   uint16_t* __restrict__ wt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < WT_HALF;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int l = i < 3LL * MLP_HID * MLP_HID ? 1 + (int)(i / (MLP_HID * MLP_HID)) : 4;
    const int64_t base = (int64_t)(l - 1) * MLP_HID * MLP_HID;
    const int64_t j = i - base;
    const int n = (int)(j / MLP_HID), k = (int)(j - (int64_t)n * MLP_HID);
    const int fo = mlp_fan_out(l);
    const float w = n < fo ? params[mlp_w_offset(l) + (int64_t)k * fo + n] : 0.f;
    const uint16_t hi = to_bf16(w);
    wt[i] = hi;
    wt[WT_HALF + i] = to_bf16(w - from_bf16(hi));
  }
}

constexpr int IR = 64;               // rows per inference workgroup
constexpr int HS = MLP_HID + 8;      // LDS row stride (bf16 elements)

// SPLIT: every operand is carried as a high BF16 part and a BF16 residual, and each
// product as hi*hi + hi*lo + lo*hi (three BF16 matrix-core steps, FP32 accumulation):
// about 16 significant bits instead of 8.
// GELU for inference: z Phi(z) with erf from Abramowitz & Stegun 7.1.26 (absolute error
// below 1.5e-7, far under the BF16 products' rounding), branch-free: one reciprocal and
// one exponential instead of the library erf's two-range evaluation.
__device__ __forceinline__ float gelu_infer(float z) {
  const float x = fabsf(z) * 0.7071067811865475f;
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * x);
  float p = 1.061405429f;
  p = fmaf(p, t, -1.453152027f);
  p = fmaf(p, t, 1.421413741f);
  p = fmaf(p, t, -0.284496736f);
  p = fmaf(p, t, 0.254829592f);
  const float e = 1.0f - p * t * __expf(-x * x);   // erf(|z| / sqrt 2)
  return 0.5f * z * (1.0f + copysignf(e, z));
}

template <bool SPLIT>
__global__ __launch_bounds__(256, 2) void k_infer_bf16(const float* __restrict__ x, int64_t n,
                                                    const float* __restrict__ params,
                                                    const uint16_t* __restrict__ wt,
                                                    float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) uint16_t H[(SPLIT ? 2 : 1) * IR * HS];
  uint16_t* Hl = H + IR * HS;
  const int64_t r0 = (int64_t)blockIdx.x * IR;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  auto put = [&](int row, int col, float v) {
    const uint16_t hi = to_bf16(v);
    H[row * HS + col] = hi;
    if (SPLIT) Hl[row * HS + col] = to_bf16(v - from_bf16(hi));
  };
  // layer 0 in FP32: thread tid owns hidden unit tid; the tile's inputs are staged in
  // LDS once (rows past n read as zero and are never written out)
  {
    __shared__ float xs[IR * MLP_IN];
    for (int i = tid; i < IR * MLP_IN; i += 256) {
      const int64_t row = r0 + i / MLP_IN;
      xs[i] = row < n ? x[r0 * MLP_IN + i] : 0.f;
    }
    float w[MLP_IN];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) w[i] = params[(int64_t)i * MLP_HID + tid];
    const float b0 = params[mlp_b_offset(0) + tid];
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < IR; ++r) {
      float z = b0;
#pragma unroll
      for (int i = 0; i < MLP_IN; ++i) z += xs[r * MLP_IN + i] * w[i];
      put(r, tid, gelu_infer(z));
    }
  }
  __syncthreads();
  const int am = lane & 31, ak = 8 * (lane >> 5);
  // layers 1..4: wave wv computes NB column tiles starting at column wv * 32 * NB
  auto layer = [&](const uint16_t* W, int col0, auto nbt,
                   f32x16 (&acc)[2][decltype(nbt)::value]) {
    constexpr int NB = decltype(nbt)::value;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;
    // the weights (L2-resident) of step k0 + 16 are requested before the products of
    // step k0, so that their latency hides behind the matrix-core work
    bf16x8 fb[NB], lb[NB];
    auto load_b = [&](int k0, bf16x8 (&b0)[NB], bf16x8 (&b1)[NB]) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int64_t o = (int64_t)(col0 + wv * 32 * NB + b * 32 + am) * MLP_HID + k0 + ak;
        b0[b] = *reinterpret_cast<const bf16x8*>(&W[o]);
        if (SPLIT) b1[b] = *reinterpret_cast<const bf16x8*>(&W[WT_HALF + o]);
      }
    };
    load_b(0, fb, lb);
#pragma unroll 2
    for (int k0 = 0; k0 < MLP_HID; k0 += 16) {
      bf16x8 fa[2], la[2], nfb[NB], nlb[NB];
      if (k0 + 16 < MLP_HID) load_b(k0 + 16, nfb, nlb);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int o = (a * 32 + am) * HS + k0 + ak;
        fa[a] = *reinterpret_cast<const bf16x8*>(&H[o]);
        if (SPLIT) la[a] = *reinterpret_cast<const bf16x8*>(&Hl[o]);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
          if (SPLIT) {
            acc[a][b] =
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], lb[b], acc[a][b], 0, 0, 0);
            acc[a][b] =
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(la[a], fb[b], acc[a][b], 0, 0, 0);
          }
        }
      if (k0 + 16 < MLP_HID) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          fb[b] = nfb[b];
          if (SPLIT) lb[b] = nlb[b];
        }
      }
    }
  };
  for (int l = 1; l < MLP_LAYERS; ++l) {
    f32x16 acc[2][2];
    layer(wt + (int64_t)(l - 1) * MLP_HID * MLP_HID, 0, std::integral_constant<int, 2>{}, acc);
    __syncthreads();
    const float* bias = params + mlp_b_offset(l);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = wv * 64 + b * 32 + am;
      const float bb = bias[col];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int i = 0; i < 16; ++i)
          put(a * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3), col,
              gelu_infer(acc[a][b][i] + bb));
    }
    __syncthreads();
  }
  // output layer in two halves of 256 columns (451 real): in half h, wave wv computes
  // columns [256 h + 64 wv, 256 h + 64 wv + 64), so that the accumulators of one half
  // (64 registers) leave room for two waves per SIMD
  const float* bias = params + mlp_b_offset(MLP_LAYERS);
  for (int h = 0; h < 2; ++h) {
    f32x16 acc[2][2];
    layer(wt + 3LL * MLP_HID * MLP_HID, 256 * h, std::integral_constant<int, 2>{}, acc);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = 256 * h + wv * 64 + b * 32 + am;
      if (col >= MLP_OUT) continue;
      const float bb = bias[col];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int64_t row = r0 + a * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
          if (row < n) out[row * MLP_OUT + col] = acc[a][b][i] + bb;
        }
    }
  }
}

unsigned grid_for(int64_t n, int64_t cap = 8192) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

}  // namespace

hipError_t launch_mlp_gemm(bool ta, bool tb, int epi, const float* A, int lda, const float* B,
                           int ldb, float* C, int ldc, float* Z, const float* bias, int M,
                           int N, int K, hipStream_t s) {
  // transposed-A products (weight gradients: small M x N, K = batch) split K over up to
  // 64 workgroup layers and add into a cleared C
  int splits = 1, kc = K;
  if (ta) {
    splits = std::max(1, std::min(64, K / 256));
    kc = ((K + splits - 1) / splits + GK - 1) / GK * GK;
    splits = (K + kc - 1) / kc;
    if (epi != 0) return hipErrorInvalidValue;
    hipError_t e = launch_fill_zero(C, (int64_t)M * ldc, s);
    if (e != hipSuccess) return e;
    epi = 3;
  }
  const dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, splits);
#define G(TA, TB, E)                                                                   \
  if (ta == TA && tb == TB && epi == E) {                                              \
    hipLaunchKernelGGL((k_gemm<TA, TB, E>), grid, dim3(256), 0, s, A, lda, B, ldb, C, \
                       ldc, Z, bias, M, N, K, kc);                                     \
    return hipGetLastError();                                                          \
  }
  G(false, false, 1)
  G(false, false, 2)
  G(true, false, 3)
  G(false, true, 0)
#undef G
  return hipErrorInvalidValue;
}

hipError_t launch_mlp_gelu_bwd(float* dH, const float* Z, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_gelu_bwd, dim3(grid_for(n)), dim3(256), 0, s, dH, Z, n);
  return hipGetLastError();
}

hipError_t launch_mlp_colsum(const float* D, int ld, int rows, int N, float* db,
                             hipStream_t s) {
  hipError_t e = launch_fill_zero(db, N, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3((N + 63) / 64, (rows + 255) / 256), dim3(256), 0, s, D, ld,
                     rows, N, db);
  return hipGetLastError();
}

hipError_t launch_mlp_loss(const float* P, const float* T, float* dP, int B, float* loss,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_loss, dim3(B), dim3(64), 0, s, P, T, dP, B, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                           float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_gather(const float* X, int cx, const float* T, int ct,
                             const int32_t* idx, int B, float* xb, float* tb, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(B), dim3(256), 0, s, X, cx, T, ct, idx, B, xb, tb);
  return hipGetLastError();
}

hipError_t launch_mlp_prep_bf16(const float* params, uint16_t* wt, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_bf16, dim3(1024), dim3(256), 0, s, params, wt);
  return hipGetLastError();
}

hipError_t launch_mlp_infer_bf16(const float* x, int64_t n, const float* params,
                                 const uint16_t* wt, bool split, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + IR - 1) / IR;
  if (split)
    hipLaunchKernelGGL(k_infer_bf16<true>, dim3((unsigned)nb), dim3(256), 0, s, x, n, params, wt,
                       out);
  else
    hipLaunchKernelGGL(k_infer_bf16<false>, dim3((unsigned)nb), dim3(256), 0, s, x, n, params,
                       wt, out);
  return hipGetLastError();
}

}  // namespace wf
