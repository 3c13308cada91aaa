// One-time FP64 work per (mesh class, time step): explicit inverse of the SPD
// system matrix on the GPU and its conversion to the stored operator.
//
// Inverse: in-place Gauss-Jordan sweeps without pivoting (stable for SPD
// matrices, where every pivot is a positive Schur complement). Sweep k maps
//   a_kk <- 1/a_kk, a_kj <- a_kj/a_kk, a_ik <- -a_ik/a_kk,
//   a_ij <- a_ij - a_ik a_kj / a_kk        (i, j != k)
// and after all n sweeps the matrix holds A^-1. Row and column k are copied
// out before each sweep so the update reads unmodified values.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "npfem_internal.h"

namespace npfem {

__global__ void gj_extract(const double* __restrict__ A, int n, int ld, int k,
                           double* __restrict__ rowk, double* __restrict__ colk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    rowk[i] = A[(size_t)k * ld + i];
    colk[i] = A[(size_t)i * ld + k];
  }
}

__global__ void gj_sweep(double* __restrict__ A, int n, int ld, int k,
                         const double* __restrict__ rowk, const double* __restrict__ colk,
                         int* fail) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n) return;
  const double p = rowk[k];
  if (!(p > 0.0)) {
    if (i == 0 && j == 0) atomicOr(fail, 1);
    return;
  }
  const double ip = 1.0 / p;
  double* a = A + (size_t)i * ld + j;
  if (i == k) {
    *a = (j == k) ? ip : rowk[j] * ip;
  } else if (j == k) {
    *a = -colk[i] * ip;
  } else {
    *a -= colk[i] * rowk[j] * ip;
  }
}

hipError_t launch_spd_inverse(double* A, int n, int ld, double* scratch, int* pivot_fail,
                              hipStream_t st) {
  double* rowk = scratch;
  double* colk = scratch + n;
  const int tb = 256;
  const dim3 g1((n + tb - 1) / tb);
  const dim3 g2((n + tb - 1) / tb, n);
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(gj_extract, g1, dim3(tb), 0, st, A, n, ld, k, rowk, colk);
    hipLaunchKernelGGL(gj_sweep, g2, dim3(tb), 0, st, A, n, ld, k, rowk, colk, pivot_fail);
  }
  return hipGetLastError();
}

// max |(m/h^2) Ainv - I| over the n x n block (one workgroup, fixed order).
__global__ void __launch_bounds__(1024) max_abs_split_kernel(const double* __restrict__ Ainv, int n,
                                                             int ld, double inv_hm,
                                                             double* __restrict__ out) {
  __shared__ double red[1024];
  double mx = 0.0;
  const size_t total = (size_t)n * n;
  for (size_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int i = (int)(idx / n), j = (int)(idx % n);
    const double b = Ainv[(size_t)i * ld + j] * inv_hm - (i == j ? 1.0 : 0.0);
    mx = fmax(mx, fabs(b));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_max_abs_split(const double* Ainv, int n, int Npad, double hm, double* out,
                                hipStream_t st) {
  hipLaunchKernelGGL(max_abs_split_kernel, dim3(1), dim3(1024), 0, st, Ainv, n, Npad, 1.0 / hm,
                     out);
  return hipGetLastError();
}

// kind 0: FP32 copy; 1: FP64 copy; 2/3: Bt = ((m/h^2) Ainv - I) / beta in
// BF16/FP16 (round to nearest even). Padding entries stay zero.
template <typename O>
__global__ void convert_kernel(const double* __restrict__ Ainv, int Npad, double inv_hm,
                               double inv_beta, int split, O* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)Npad * Npad;
  if (idx >= total) return;
  double v = Ainv[idx];
  if (split) {
    const int i = (int)(idx / Npad), j = (int)(idx % Npad);
    v = (v * inv_hm - ((i == j && v != 0.0) ? 1.0 : 0.0)) * inv_beta;
  }
  out[idx] = O(v);
}

template <>
__global__ void convert_kernel<__bf16>(const double* __restrict__ Ainv, int Npad, double inv_hm,
                                       double inv_beta, int split, __bf16* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)Npad * Npad;
  if (idx >= total) return;
  double v = Ainv[idx];
  if (split) {
    const int i = (int)(idx / Npad), j = (int)(idx % Npad);
    v = (v * inv_hm - ((i == j && v != 0.0) ? 1.0 : 0.0)) * inv_beta;
  }
  out[idx] = __bf16((float)v);
}

template <>
__global__ void convert_kernel<_Float16>(const double* __restrict__ Ainv, int Npad, double inv_hm,
                                         double inv_beta, int split, _Float16* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)Npad * Npad;
  if (idx >= total) return;
  double v = Ainv[idx];
  if (split) {
    const int i = (int)(idx / Npad), j = (int)(idx % Npad);
    v = (v * inv_hm - ((i == j && v != 0.0) ? 1.0 : 0.0)) * inv_beta;
  }
  out[idx] = (_Float16)(float)v;
}

// A^-1 - s I in FP32 (nonzero diagonal entries only: padding stays zero).
// Near rest A^-1 ~ s I with s = h^2/m, and the rest, the coupling the
// constraints add, is ~1e-4 of it: an FP32 copy of A^-1 itself keeps only
// ~3 digits of that part, this one all of FP32's.
__global__ void convert_offdiag_kernel(const double* __restrict__ Ainv, int Npad, double s,
                                       float* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)Npad * Npad;
  if (idx >= total) return;
  double v = Ainv[idx];
  const int i = (int)(idx / Npad), j = (int)(idx % Npad);
  if (i == j && v != 0.0) v -= s;
  out[idx] = (float)v;
}

hipError_t launch_convert_offdiag(const double* Ainv, int Npad, double s, float* out,
                                  hipStream_t st) {
  const size_t total = (size_t)Npad * Npad;
  hipLaunchKernelGGL(convert_offdiag_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     st, Ainv, Npad, s, out);
  return hipGetLastError();
}

hipError_t launch_convert_operator(int kind, const double* Ainv, int Npad, double hm, double beta,
                                   void* out, hipStream_t st) {
  const size_t total = (size_t)Npad * Npad;
  const dim3 grid((unsigned)((total + 255) / 256));
  const double ib = beta > 0.0 ? 1.0 / beta : 0.0;
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(convert_kernel<float>, grid, dim3(256), 0, st, Ainv, Npad, 1.0 / hm, 1.0,
                         0, static_cast<float*>(out));
      break;
    case 1:
      hipLaunchKernelGGL(convert_kernel<double>, grid, dim3(256), 0, st, Ainv, Npad, 1.0 / hm,
                         1.0, 0, static_cast<double*>(out));
      break;
    case 2:
      hipLaunchKernelGGL(convert_kernel<__bf16>, grid, dim3(256), 0, st, Ainv, Npad, 1.0 / hm, ib,
                         1, static_cast<__bf16*>(out));
      break;
    case 3:
      hipLaunchKernelGGL(convert_kernel<_Float16>, grid, dim3(256), 0, st, Ainv, Npad, 1.0 / hm,
                         ib, 1, static_cast<_Float16*>(out));
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace npfem
