// Immersed-boundary transfer between a periodic fluid grid and the membrane
// vertices: velocity interpolation at the vertices and force spreading onto
// the grid, with Peskin's 4-point regularised delta function (the IBM
// couples the solids to the fluid through interpolation kernels,
// Introduction).
//
// Grid node (i, j, k) sits at o + dx (i, j, k); fields are SoA
// [3][nx ny nz] with flat index i + nx (j + ny k); indices wrap
// periodically. A vertex's global position is its cell's FP64 origin plus
// its cell-local coordinates, formed in FP64 (the grid coordinate of a vertex
// in a domain of hundreds of cells keeps FP32 resolution only relative to
// the origin). With s = (X - o)/dx, r = s - floor(s) and
// q = sqrt(1 + 4r - 4r^2), the weights of the nodes floor(s) - 1 .. + 2 are
//   ((3 - 2r - q), (3 - 2r + q), (1 + 2r + q), (1 + 2r - q)) / 8
// (phi at distances r + 1, r, 1 - r, 2 - r; they sum to 1).
//
// Spreading is made bitwise reproducible with fixed-point atomics: every
// contribution F phi phi phi / dx^3 is rounded to an integer multiple of 1/S
// and added with 64-bit integer atomics (integer addition is associative,
// so the order of the atomics does not matter), then the sums are converted
// back. S is a power of two chosen from max |F| so that no node sum can
// exceed 2^62 / S: with n vertices and |phi phi phi| <= 1/8,
//   S = 2^floor(log2(2^62 / (n max|F| / (8 dx^3)))),
// which keeps ~40 bits below the largest possible contribution. A cell's
// contributions are first summed in LDS over the box of nodes its vertices
// reach (ibm_spread_box_kernel), then added to the grid once per node.
#include <algorithm>
#include <cmath>

#include "device_utils.h"
#include "npfem_internal.h"

namespace npfem {

template <typename T>
__device__ __forceinline__ void peskin4(double s, int& i0, T (&w)[4]) {
  const double fl = floor(s);
  i0 = (int)fl - 1;
  const T r = T(s - fl);
  const T q = sqrt(T(1) + T(4) * r - T(4) * r * r);
  w[0] = (T(3) - T(2) * r - q) * T(0.125);
  w[1] = (T(3) - T(2) * r + q) * T(0.125);
  w[2] = (T(1) + T(2) * r + q) * T(0.125);
  w[3] = (T(1) + T(2) * r - q) * T(0.125);
}

__device__ __forceinline__ int wrap(int i, int n) {
  const int m = i % n;
  return m < 0 ? m + n : m;
}

// One workgroup per cell of a class, one thread per vertex.
template <typename T>
__global__ void __launch_bounds__(256) ibm_interpolate_kernel(
    ClassSlice<T> cs, const T* __restrict__ pos, long long sumN,
    const double* __restrict__ origins, const T* __restrict__ u, IbmGrid g,
    T* __restrict__ out) {
  const int lc = blockIdx.x;
  const int cell = cs.cell0 + lc;
  const int N = cs.cv.N;
  const long long vb = cs.vert0 + (long long)lc * N;
  const double ox = origins[3 * cell], oy = origins[3 * cell + 1], oz = origins[3 * cell + 2];
  const long long nn = (long long)g.nx * g.ny * g.nz;
  const double idx = 1.0 / g.dx;
  for (int v = threadIdx.x; v < N; v += blockDim.x) {
    const long long e = vb + v;
    int i0, j0, k0;
    T wx[4], wy[4], wz[4];
    peskin4<T>((ox + (double)pos[e] - g.ox) * idx, i0, wx);
    peskin4<T>((oy + (double)pos[sumN + e] - g.oy) * idx, j0, wy);
    peskin4<T>((oz + (double)pos[2 * sumN + e] - g.oz) * idx, k0, wz);
    int ii[4], jj[4], kk[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      ii[a] = wrap(i0 + a, g.nx);
      jj[a] = wrap(j0 + a, g.ny);
      kk[a] = wrap(k0 + a, g.nz);
    }
    T acc[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const long long row = (long long)g.nx * (jj[b] + (long long)g.ny * kk[c]);
        const T wbc = wy[b] * wz[c];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const long long n = row + ii[a];
          const T wt = wx[a] * wbc;
          acc[0] += wt * u[n];
          acc[1] += wt * u[nn + n];
          acc[2] += wt * u[2 * nn + n];
        }
      }
    }
    out[e] = acc[0];
    out[sumN + e] = acc[1];
    out[2 * sumN + e] = acc[2];
  }
}

// max |F| over the class's vertices into *mx (bit pattern of a non-negative
// double: integer order equals value order); non-finite forces set the
// status flag (and are left out).
template <typename T>
__global__ void __launch_bounds__(256) ibm_maxabs_kernel(ClassSlice<T> cs,
                                                         const T* __restrict__ f, long long sumN,
                                                         unsigned long long* __restrict__ mx,
                                                         int* status) {
  const int N = cs.cv.N;
  const long long vb = cs.vert0 + (long long)blockIdx.x * N;
  double m = 0.0;
  int bad = 0;
  for (int v = threadIdx.x; v < N; v += blockDim.x) {
    const long long e = vb + v;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double a = fabs((double)f[d * sumN + e]);
      if (isfinite(a)) m = fmax(m, a);
      else bad = 1;
    }
  }
  m = wave_max_dpp(m);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(mx, (unsigned long long)__double_as_longlong(m));
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(status, ST_NONFINITE);
}

__device__ __forceinline__ double ibm_scale(const unsigned long long* mx, double n_total,
                                            double dx) {
  const double m = __longlong_as_double((long long)*mx);
  if (!(m > 0.0)) return 1.0;
  const double cmax = n_total * m / (8.0 * dx * dx * dx);
  const int e = (int)floor(log2(ldexp(1.0, 62) / cmax));
  return ldexp(1.0, max(-1000, min(1000, e)));
}

// Spreading, one workgroup per cell. The cell's vertices touch a box of grid
// nodes (their supports), which the workgroup sums with 64-bit LDS atomics
// and then adds to the grid with one global atomic per touched node and
// component (instead of one per vertex, node and component). The box is
// found from the vertices' lowest and highest support nodes; a box beyond
// the LDS budget, or a non-finite or far-off coordinate, sends the cell's
// contributions to the grid directly, one global atomic each. The same
// integers either way, so the same (bitwise) result.
constexpr int kIbmBoxNodes = 2688;  // 3 x 8 bytes each: 63 KB of LDS

__device__ __forceinline__ double block_min_d(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < (int)blockDim.x / kWave; ++w) r = fmin(r, red[w]);
  return r;
}

template <typename T>
__global__ void __launch_bounds__(256) ibm_spread_box_kernel(
    ClassSlice<T> cs, const T* __restrict__ pos, long long sumN,
    const double* __restrict__ origins, const T* __restrict__ f, IbmGrid g,
    const unsigned long long* __restrict__ mx, double n_total,
    unsigned long long* __restrict__ acc) {
  __shared__ unsigned long long box[3 * kIbmBoxNodes];
  __shared__ double red[256 / kWave];
  const int lc = blockIdx.x;
  const int cell = cs.cell0 + lc;
  const int N = cs.cv.N;
  const long long vb = cs.vert0 + (long long)lc * N;
  const double ox = origins[3 * cell], oy = origins[3 * cell + 1], oz = origins[3 * cell + 2];
  const long long nn = (long long)g.nx * g.ny * g.nz;
  const double idx = 1.0 / g.dx;
  const double S = ibm_scale(mx, n_total, g.dx) / (g.dx * g.dx * g.dx);
  // the cell's support box: lowest and highest floor of the grid coordinate
  // per axis (unwrapped node units)
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int bad = 0;
  for (int v = threadIdx.x; v < N; v += blockDim.x) {
    const long long e = vb + v;
    const double sv[3] = {(ox + (double)pos[e] - g.ox) * idx, (oy + (double)pos[sumN + e] - g.oy) * idx,
                          (oz + (double)pos[2 * sumN + e] - g.oz) * idx};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double fl = floor(sv[d]);
      if (!(fabs(fl) < 1e9)) {
        bad = 1;
      } else {
        lo[d] = fmin(lo[d], fl);
        hi[d] = fmax(hi[d], fl);
      }
    }
  }
  bool fits = !__syncthreads_or(bad);  // (uniform)
  int b0[3] = {0, 0, 0}, bn[3] = {4, 4, 4};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double l = block_min_d(lo[d], red), h = -block_min_d(-hi[d], red);
    if (fits && h - l + 4.0 <= (double)kIbmBoxNodes) {
      b0[d] = (int)l - 1;  // the lowest support node, floor - 1
      bn[d] = (int)(h - l) + 4;
    } else {
      fits = false;
    }
  }
  const long long vol = (long long)bn[0] * bn[1] * bn[2];
  fits = fits && vol <= kIbmBoxNodes;
  if (fits) {
    for (int i = threadIdx.x; i < 3 * vol; i += blockDim.x) box[i] = 0ull;
    __syncthreads();
  }
  for (int v = threadIdx.x; v < N; v += blockDim.x) {
    const long long e = vb + v;
    int i0, j0, k0;
    double wx[4], wy[4], wz[4];
    peskin4<double>((ox + (double)pos[e] - g.ox) * idx, i0, wx);
    peskin4<double>((oy + (double)pos[sumN + e] - g.oy) * idx, j0, wy);
    peskin4<double>((oz + (double)pos[2 * sumN + e] - g.oz) * idx, k0, wz);
    const double fs[3] = {(double)f[e] * S, (double)f[sumN + e] * S, (double)f[2 * sumN + e] * S};
    // the box holds every support by construction; checked all the same
    const bool inb = fits && (unsigned)(i0 - b0[0]) <= (unsigned)(bn[0] - 4) &&
                     (unsigned)(j0 - b0[1]) <= (unsigned)(bn[1] - 4) &&
                     (unsigned)(k0 - b0[2]) <= (unsigned)(bn[2] - 4);
    for (int c = 0; c < 4; ++c) {
      for (int b = 0; b < 4; ++b) {
        const double wbc = wy[b] * wz[c];
        const long long row = inb ? (long long)bn[0] * ((j0 + b - b0[1]) + (long long)bn[1] * (k0 + c - b0[2]))
                                  : (long long)g.nx * (wrap(j0 + b, g.ny) + (long long)g.ny * wrap(k0 + c, g.nz));
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const double wt = wx[a] * wbc;
          if (inb) {
            const long long n = row + (i0 + a - b0[0]);
#pragma unroll
            for (int d = 0; d < 3; ++d)
              atomicAdd(box + d * vol + n, (unsigned long long)llrint(wt * fs[d]));
          } else {
            const long long n = row + wrap(i0 + a, g.nx);
#pragma unroll
            for (int d = 0; d < 3; ++d)
              atomicAdd(acc + d * nn + n, (unsigned long long)llrint(wt * fs[d]));
          }
        }
      }
    }
  }
  if (!fits) return;
  __syncthreads();
  for (long long i = threadIdx.x; i < vol; i += blockDim.x) {
    const int a = (int)(i % bn[0]);
    const int b = (int)((i / bn[0]) % bn[1]);
    const int c = (int)(i / ((long long)bn[0] * bn[1]));
    const long long n = wrap(b0[0] + a, g.nx) +
                        (long long)g.nx * (wrap(b0[1] + b, g.ny) + (long long)g.ny * wrap(b0[2] + c, g.nz));
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const unsigned long long v = box[d * vol + i];
      if (v) atomicAdd(acc + d * nn + n, v);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) ibm_convert_kernel(const unsigned long long* __restrict__ acc,
                                                          long long count,
                                                          const unsigned long long* __restrict__ mx,
                                                          double n_total, double dx,
                                                          T* __restrict__ out) {
  const double iS = 1.0 / ibm_scale(mx, n_total, dx);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = T((double)(long long)acc[i] * iS);
}

__global__ void __launch_bounds__(256) ibm_zero_kernel(unsigned long long* __restrict__ p,
                                                       long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

template <typename T>
hipError_t launch_ibm_interpolate(const ClassSlice<T>& cs, const T* pos, long long sumN,
                                  const double* origins, const T* u, const IbmGrid& g, T* out,
                                  hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  hipLaunchKernelGGL(ibm_interpolate_kernel<T>, dim3(cs.n_cells), dim3(256), 0, st, cs, pos, sumN,
                     origins, u, g, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ibm_maxabs(const ClassSlice<T>& cs, const T* f, long long sumN,
                             unsigned long long* mx, int* status, hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  hipLaunchKernelGGL(ibm_maxabs_kernel<T>, dim3(cs.n_cells), dim3(256), 0, st, cs, f, sumN, mx,
                     status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ibm_spread(const ClassSlice<T>& cs, const T* pos, long long sumN,
                             const double* origins, const T* f, const IbmGrid& g,
                             const unsigned long long* mx, double n_total,
                             unsigned long long* acc, hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  hipLaunchKernelGGL(ibm_spread_box_kernel<T>, dim3(cs.n_cells), dim3(256), 0, st, cs, pos, sumN,
                     origins, f, g, mx, n_total, acc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ibm_convert(const unsigned long long* acc, long long count,
                              const unsigned long long* mx, double n_total, double dx, T* out,
                              hipStream_t st) {
  const int blocks = (int)std::min<long long>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(ibm_convert_kernel<T>, dim3(std::max(blocks, 1)), dim3(256), 0, st, acc,
                     count, mx, n_total, dx, out);
  return hipGetLastError();
}

hipError_t launch_ibm_zero(unsigned long long* p, long long count, hipStream_t st) {
  const int blocks = (int)std::min<long long>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(ibm_zero_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, st, p, count);
  return hipGetLastError();
}

#define NPFEM_INST(T)                                                                             \
  template hipError_t launch_ibm_interpolate<T>(const ClassSlice<T>&, const T*, long long,        \
                                                const double*, const T*, const IbmGrid&, T*,     \
                                                hipStream_t);                                    \
  template hipError_t launch_ibm_maxabs<T>(const ClassSlice<T>&, const T*, long long,             \
                                           unsigned long long*, int*, hipStream_t);              \
  template hipError_t launch_ibm_spread<T>(const ClassSlice<T>&, const T*, long long,             \
                                           const double*, const T*, const IbmGrid&,              \
                                           const unsigned long long*, double,                    \
                                           unsigned long long*, hipStream_t);                    \
  template hipError_t launch_ibm_convert<T>(const unsigned long long*, long long,                 \
                                            const unsigned long long*, double, double, T*,       \
                                            hipStream_t);
NPFEM_INST(float)
NPFEM_INST(double)
#undef NPFEM_INST

}  // namespace npfem
