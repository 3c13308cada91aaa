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

// Row shift of a double across the lanes of a 16-lane row (DPP row_shr:n);
// lanes whose source lies before the row start read 0.
template <int N>
__device__ __forceinline__ double dpp_row_shr(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x110 | N, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x110 | N, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Wave-wide sum: inclusive scans of each 16-lane row (shifts 1, 2, 4, 8),
// then the four row totals (lanes 15, 31, 47, 63) in a fixed order. Every
// lane receives the same value; the order does not depend on the data.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_row_shr<1>(v);
  v += dpp_row_shr<2>(v);
  v += dpp_row_shr<4>(v);
  v += dpp_row_shr<8>(v);
  return (read_lane(v, 15) + read_lane(v, 31)) + (read_lane(v, 47) + read_lane(v, 63));
}

__device__ __forceinline__ double wave_max_dpp(double v) {
  v = fmax(v, dpp_row_shr<1>(v));
  v = fmax(v, dpp_row_shr<2>(v));
  v = fmax(v, dpp_row_shr<4>(v));
  v = fmax(v, dpp_row_shr<8>(v));
  return fmax(fmax(read_lane(v, 15), read_lane(v, 31)), fmax(read_lane(v, 47), read_lane(v, 63)));
}

// Workgroup sums of NS doubles and, if WITH_MAX, the maximum of one more,
// with a single barrier. red holds 2 * (NS + 1) * (blockDim.x / 64) doubles
// and is used as two halves: consecutive calls must alternate buf (0, 1), so
// that a call never overwrites the half that the previous call is still
// reading. Identical totals in every thread. Call from uniform control flow.
// The max input must be >= 0 (lanes with no data contribute 0).
// block_sum_max in two halves around a barrier the caller provides: the
// waves' partials are written by block_sum_max_write and combined, after any
// barrier, by block_sum_max_read (same arithmetic, same totals).
template <int NS, bool WITH_MAX>
__device__ __forceinline__ void block_sum_max_write(double (&v)[NS], double& mx, double* red,
                                                    int buf) {
  constexpr int NV = NS + (WITH_MAX ? 1 : 0);
  const int nw = blockDim.x / kWave;
  const int w = threadIdx.x / kWave;
  const int l = threadIdx.x % kWave;
  double* r = red + (size_t)buf * (NS + 1) * nw;
#pragma unroll
  for (int i = 0; i < NS; ++i) v[i] = wave_sum_dpp(v[i]);
  if (WITH_MAX) mx = wave_max_dpp(mx);
  if (l == 0) {
#pragma unroll
    for (int i = 0; i < NS; ++i) r[w * NV + i] = v[i];
    if (WITH_MAX) r[w * NV + NS] = mx;
  }
}

template <int NS, bool WITH_MAX>
__device__ __forceinline__ void block_sum_max_read(double (&v)[NS], double& mx, const double* red,
                                                   int buf) {
  constexpr int NV = NS + (WITH_MAX ? 1 : 0);
  const int nw = blockDim.x / kWave;
  const double* r = red + (size_t)buf * (NS + 1) * nw;
#pragma unroll
  for (int i = 0; i < NS; ++i) v[i] = 0.0;
  if (WITH_MAX) mx = 0.0;
  for (int k = 0; k < nw; ++k) {
#pragma unroll
    for (int i = 0; i < NS; ++i) v[i] += r[k * NV + i];
    if (WITH_MAX) mx = fmax(mx, r[k * NV + NS]);
  }
}

template <int NS, bool WITH_MAX>
__device__ __forceinline__ void block_sum_max(double (&v)[NS], double& mx, double* red, int buf) {
  block_sum_max_write<NS, WITH_MAX>(v, mx, red, buf);
  __syncthreads();
  block_sum_max_read<NS, WITH_MAX>(v, mx, red, buf);
}

// Float row shift (DPP row_shr:n), 0 where the source lies before the row.
template <int N>
__device__ __forceinline__ float dpp_row_shr_f(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 | N, 0xf, 0xf, false));
}

// Workgroup maxima of NV non-negative floats with a single barrier (DPP row
// maxima, then the four row results of each wave, then the waves' results
// through red, NV * (blockDim.x / 64) floats). The caller makes sure that no
// thread still reads red from an earlier use. Every thread returns the
// maxima. Call from uniform control flow.
template <int NV>
__device__ __forceinline__ void block_max_n(float (&v)[NV], float* red) {
  const int nw = blockDim.x / kWave;
  const int w = threadIdx.x / kWave;
  const int l = threadIdx.x % kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    float x = v[i];
    x = fmaxf(x, dpp_row_shr_f<1>(x));
    x = fmaxf(x, dpp_row_shr_f<2>(x));
    x = fmaxf(x, dpp_row_shr_f<4>(x));
    x = fmaxf(x, dpp_row_shr_f<8>(x));
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 15));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 31));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 47));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
    v[i] = fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
  }
  if (l == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[w * NV + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    float m = 0.f;
    for (int k = 0; k < nw; ++k) m = fmaxf(m, red[k * NV + i]);
    v[i] = m;
  }
}

template <typename T>
__device__ __forceinline__ bool finite_val(T x) {
  return isfinite(x);
}

}  // namespace npfem
