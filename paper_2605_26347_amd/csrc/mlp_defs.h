// Inputs and outputs of the residual-kernel network (not part of the paper): a
// multilayer perceptron that predicts the thresholded residual-w Fourier kernel of
// Sect. 3.1 from per-row inputs, with one extra output that predicts log10 of its own
// relative L2 error.  Shared by the build kernels and the network kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace wf {

constexpr int MLP_IN = 5;                          // network inputs per row
constexpr int MLP_HID = 256;                       // hidden width
constexpr int MLP_LAYERS = 4;                      // hidden layers (exact GELU)
constexpr int MLP_SIDE = 15;                       // predicted kernel window side
constexpr int MLP_KOUT = 2 * MLP_SIDE * MLP_SIDE;  // 450 kernel outputs (re, im)
constexpr int MLP_OUT = MLP_KOUT + 1;              // + error output
constexpr double MLP_LREF = 0.06981317007977318;   // 4 degrees in radians

// Network inputs of one row: w_proj (o L)^2 / 4, L / L_ref, the row's offsets from its
// nearest grid cell (cells), and n_k / 15 for the uncapped kernel side n_k (a function
// of w_proj and L, given so that the network can follow the kernel's jumps where the
// sampled side changes).  L = nx cell, square fields.
__host__ __device__ inline void mlp_inputs(double wproj, double L, int o, double fu, double fv,
                                           int nk, float* x) {
  const double oL = (double)o * L;
  x[0] = (float)(wproj * oL * oL / 4.0);
  x[1] = (float)(L / MLP_LREF);
  x[2] = (float)fu;
  x[3] = (float)fv;
  x[4] = (float)((double)nk / 15.0);
}

// Flat parameter vector: for each layer W [in x out] row-major, then b [out].
__host__ __device__ inline int mlp_fan_in(int l) { return l == 0 ? MLP_IN : MLP_HID; }
__host__ __device__ inline int mlp_fan_out(int l) { return l == MLP_LAYERS ? MLP_OUT : MLP_HID; }
__host__ __device__ inline int64_t mlp_w_offset(int l) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += (int64_t)mlp_fan_in(i) * mlp_fan_out(i) + mlp_fan_out(i);
  return o;
}
__host__ __device__ inline int64_t mlp_b_offset(int l) {
  return mlp_w_offset(l) + (int64_t)mlp_fan_in(l) * mlp_fan_out(l);
}
__host__ __device__ inline int64_t mlp_num_params() { return mlp_w_offset(MLP_LAYERS + 1); }

}  // namespace wf
