// Small device helpers: wavefront/workgroup reductions (64-wide waves).
#pragma once

#include <hip/hip_runtime.h>

namespace npfem {

constexpr int kWave = 64;

// Butterfly sum over the 64 lanes of a wave. Every lane ends with the same
// value bit for bit (each stage adds the same two operands in either order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return v;
}

// Workgroup sum of NV doubles; red must hold NV * (blockDim.x / 64) doubles of
// LDS. All threads return identical totals (fixed summation order). Contains
// two barriers; call from uniform control flow.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
  const int nw = blockDim.x / kWave;
  const int w = threadIdx.x / kWave;
  const int l = threadIdx.x % kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (l == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i * nw + w] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += red[i * nw + k];
    v[i] = s;
  }
}

__device__ __forceinline__ float block_max(float v, float* red) {
  const int nw = blockDim.x / kWave;
  const int w = threadIdx.x / kWave;
  const int l = threadIdx.x % kWave;
  v = wave_max(v);
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  float s = red[0];
  for (int k = 1; k < nw; ++k) s = fmaxf(s, red[k]);
  return s;
}

template <typename T>
__device__ __forceinline__ bool finite_val(T x) {
  return isfinite(x);
}

}  // namespace npfem
