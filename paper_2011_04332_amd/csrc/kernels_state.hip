// Streaming kernels around the PD iterations: predict, update, the
// refinement residual and per-cell volumes.
//
// Layouts: the caller's state is SoA [3][sumN]; the solver's column buffers
// hold one column per (cell, coordinate) of Npad entries (rows >= N are zero),
// so that the global step is a plain GEMM over 3 * cells columns.
#include <algorithm>
#include <mutex>

#include "device_utils.h"
#include "npfem_internal.h"

namespace npfem {

// Predict (start of a time step, delta form). With s = x + h v + (h^2/m) f:
//   cterm  = (m/h^2)(s - x) = (m/h) v + f   (constant over the PD iterations)
//   delta0 = (s - x)/(1 + alpha h)          (q^0 = s; with mass-proportional
//            damping alpha the minimiser of the inertia and damping terms)
// Rows per thread in predict and update (a 656-row RBC column in one pass
// of 256 threads).
constexpr int kStateRows = 3;

template <typename T>
__global__ void __launch_bounds__(256) predict_kernel(ClassSlice<T> cs, const T* __restrict__ pos,
                                                      const T* __restrict__ vel,
                                                      const T* __restrict__ force, long long sumN,
                                                      T* __restrict__ delta, T* __restrict__ cterm,
                                                      int* status, double h, double alpha) {
  const int lc = blockIdx.x;
  const int N = cs.cv.N, Npad = cs.cv.Npad;
  const long long vb = cs.vert0 + (long long)lc * N;
  const long long cb = cs.elem0 + 3LL * lc * Npad;
  const double m = (double)cs.mass;
  const double mh = m / h, hm = h * h / m, ds = 1.0 / (1.0 + alpha * h);
  int bad = 0;
  // kStateRows rows per thread with all their loads in flight (clamped
  // addresses; rows past N are written as zeros)
  for (int v0 = threadIdx.x; v0 < Npad; v0 += kStateRows * blockDim.x) {
    T x[kStateRows][3], u[kStateRows][3], f[kStateRows][3];
#pragma unroll
    for (int r = 0; r < kStateRows; ++r) {
      const int v = min(v0 + r * (int)blockDim.x, N - 1);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        x[r][d] = pos[d * sumN + vb + v];
        u[r][d] = vel[d * sumN + vb + v];
        f[r][d] = force[d * sumN + vb + v];
      }
    }
#pragma unroll
    for (int r = 0; r < kStateRows; ++r) {
      const int v = v0 + r * (int)blockDim.x;
      if (v >= Npad) break;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        T c = T(0), dl = T(0);
        if (v < N) {
          bad |= !(isfinite(x[r][d]) && isfinite(u[r][d]) && isfinite(f[r][d]));
          const double cd = mh * (double)u[r][d] + (double)f[r][d];
          c = T(cd);
          dl = T((h * (double)u[r][d] + hm * (double)f[r][d]) * ds);
        }
        cterm[cb + d * Npad + v] = c;
        delta[cb + d * Npad + v] = dl;
      }
    }
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(status, ST_NONFINITE);
}

// Update (end of a time step): x <- x + delta, v <- delta / h.
template <typename T>
__global__ void __launch_bounds__(256) update_kernel(ClassSlice<T> cs, T* __restrict__ pos,
                                                     T* __restrict__ vel, long long sumN,
                                                     const T* __restrict__ delta, double h) {
  const int lc = blockIdx.x;
  const int N = cs.cv.N, Npad = cs.cv.Npad;
  const long long vb = cs.vert0 + (long long)lc * N;
  const long long cb = cs.elem0 + 3LL * lc * Npad;
  const double ih = 1.0 / h;
  for (int v0 = threadIdx.x; v0 < N; v0 += kStateRows * blockDim.x) {
    T dl[kStateRows][3], x[kStateRows][3];
#pragma unroll
    for (int r = 0; r < kStateRows; ++r) {
      const int v = min(v0 + r * (int)blockDim.x, N - 1);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        dl[r][d] = delta[cb + d * Npad + v];
        x[r][d] = pos[d * sumN + vb + v];
      }
    }
#pragma unroll
    for (int r = 0; r < kStateRows; ++r) {
      const int v = v0 + r * (int)blockDim.x;
      if (v >= N) break;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        pos[d * sumN + vb + v] = x[r][d] + dl[r][d];
        vel[d * sumN + vb + v] = T((double)dl[r][d] * ih);
      }
    }
  }
}

// Refinement residual res = r - A_c (delta - delta0) for each cell (delta0 the
// iterate the solve started from, nullptr for none), with the per-cell
// matrix A_c = (cmass m + cvol w_v) I + clap ((w_s + w_a) L_tri + w_b L_bend)
// (fixed-width rows of the two Laplacians, shared by the class): the
// system matrix (cmass = 1/h^2, clap = cvol = 1; damped: cmass = (1 + alpha
// h)/h^2, clap = 1 + beta/h), or a damping term (cvol = 0). One workgroup handles CPB
// cells with one thread per row (up to 768 rows at a time): the row's table
// entries are fetched once and applied to all CPB cells, so the class tables
// are read from L2 once per CPB cells, and a thread has three round trips to
// memory in sequence (the cells' delta into LDS; the right-hand sides with
// the first table entries; the remaining entries). delta is staged as
// [cell][coordinate][N + 1] (the last value 0, for padding entries);
// products accumulate in FP64. colmax: per column max |res| (FP16 scaling):
// wave maxima, then LDS atomic max on the bit patterns of the non-negative
// floats.
//
// need (optional, with colmax): max |r| of each column of the right-hand side
// that the sweeps correct. A cell whose need_factor * max |r| (a bound on the
// error the previous solve left in its delta) is at most need_thr needs no
// further correction: its colmax entries are set to 0, which tells the
// correcting product to leave its columns alone. A workgroup whose cells all
// need none returns without reading anything else.
constexpr int kResidualBlock = 768;

template <typename T, int CPB>
__global__ void __launch_bounds__(kResidualBlock) residual_kernel(
    ClassSlice<T> cs, const T* __restrict__ rhs, const T* __restrict__ delta,
    const T* __restrict__ delta0, T* __restrict__ res,
    const T* __restrict__ weights, float* __restrict__ colmax, const float* __restrict__ need,
    double need_factor, double need_thr, double cmass, double clap, double cvol) {
  extern __shared__ double smem_res[];
  unsigned* cmx = reinterpret_cast<unsigned*>(smem_res);  // [3 CPB]
  T* sd = reinterpret_cast<T*>(smem_res + (3 * CPB + 1) / 2);  // [CPB][3][N + 1]
  const int N = cs.cv.N, Npad = cs.cv.Npad, DL = cs.cv.DL, N1 = N + 1;
  const int c0 = blockIdx.x * CPB, tid = threadIdx.x, nt = blockDim.x;
  const int ncell = min(CPB, cs.n_cells - c0);
  bool live[CPB];
  bool any_live = false;
#pragma unroll
  for (int c = 0; c < CPB; ++c) {
    live[c] = c < ncell;
    if (need && colmax && c < ncell) {
      const float* nc = need + cs.col0 + 3LL * (c0 + c);
      const double mx = fmax(fmax((double)nc[0], (double)nc[1]), (double)nc[2]);
      live[c] = !(need_factor * mx <= need_thr);  // NaN: live
    }
    any_live = any_live || live[c];
  }
  if (!any_live) {
    if (colmax && tid < 3 * ncell) colmax[cs.col0 + 3LL * c0 + tid] = 0.0f;
    return;
  }
  const T* __restrict__ dcell = delta + cs.elem0 + 3LL * c0 * Npad;
  const T* __restrict__ d0cell = delta0 ? delta0 + cs.elem0 + 3LL * c0 * Npad : nullptr;
  const T* __restrict__ rcell = rhs + cs.elem0 + 3LL * c0 * Npad;
  T* __restrict__ ocell = res + cs.elem0 + 3LL * c0 * Npad;
  const int* __restrict__ lcol = cs.cv.lap_col;
  const T* __restrict__ lt = cs.cv.lap_t;
  const T* __restrict__ lb = cs.cv.lap_b;
  for (int v0 = 0; v0 <= N; v0 += nt) {
    const int v = v0 + tid;
    if (v <= N) {
      const int vc = min(v, N - 1);
      T dv[CPB][3], d0[CPB][3];
#pragma unroll
      for (int c = 0; c < CPB; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const size_t e = (size_t)(3 * min(c, ncell - 1) + d) * Npad + vc;
          dv[c][d] = dcell[e];
          d0[c][d] = d0cell ? d0cell[e] : T(0);
        }
#pragma unroll
      for (int c = 0; c < CPB; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d)
          sd[(3 * c + d) * N1 + v] = (v < N && c < ncell) ? dv[c][d] - d0[c][d] : T(0);
    }
  }
  if (tid < 3 * CPB) cmx[tid] = 0u;
  __syncthreads();
  double diag[CPB], wt[CPB], wb[CPB];
#pragma unroll
  for (int c = 0; c < CPB; ++c) {
    const int cell = cs.cell0 + c0 + min(c, ncell - 1);
    double w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = weights ? (double)weights[4 * cell + k] : (double)cs.w_nom[k];
    diag[c] = cmass * (double)cs.mass + cvol * w[3];
    wt[c] = clap * (w[0] + w[1]);
    wb[c] = clap * w[2];
  }
  float cm[CPB][3];
#pragma unroll
  for (int c = 0; c < CPB; ++c) cm[c][0] = cm[c][1] = cm[c][2] = 0.f;
  for (int v = tid; v < Npad; v += nt) {
    double a[CPB][3];
    T r[CPB][3];
    const int vr = min(v, N - 1);
#pragma unroll
    for (int c = 0; c < CPB; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        r[c][d] = rcell[(size_t)(3 * min(c, ncell - 1) + d) * Npad + vr];
        a[c][d] = diag[c] * (double)sd[(3 * c + d) * N1 + vr];
      }
    // row entries fetched 8 at a time (the slots past the last clamped,
    // their weight zeroed)
    for (int k0 = 0; k0 < DL; k0 += 8) {
      int jj[8];
      T ct[8], cbv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = min(k0 + u, DL - 1) * N + vr;
        jj[u] = lcol[e];
        ct[u] = lt[e];
        cbv[u] = lb[e];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool on = k0 + u < DL;
        const int j = jj[u];
#pragma unroll
        for (int c = 0; c < CPB; ++c) {
          const double cf = on ? wt[c] * (double)ct[u] + wb[c] * (double)cbv[u] : 0.0;
#pragma unroll
          for (int d = 0; d < 3; ++d) a[c][d] += cf * (double)sd[(3 * c + d) * N1 + j];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CPB; ++c) {
      if (c < ncell) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double o = v < N ? (double)r[c][d] - a[c][d] : 0.0;
          ocell[(size_t)(3 * c + d) * Npad + v] = T(o);
          cm[c][d] = fmaxf(cm[c][d], fabsf((float)o));
        }
      }
    }
  }
  if (colmax) {
    // wave maxima first, then one LDS atomic per wave and column
#pragma unroll
    for (int c = 0; c < CPB; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float mx = wave_max(cm[c][d]);
        if ((tid & (kWave - 1)) == 0) atomicMax(&cmx[3 * c + d], __float_as_uint(mx));
      }
    __syncthreads();
    if (tid < 3 * ncell) {
      bool lv = false;
#pragma unroll
      for (int c = 0; c < CPB; ++c) lv = lv || (tid / 3 == c && live[c]);
      colmax[cs.col0 + 3LL * c0 + tid] = lv ? __uint_as_float(cmx[tid]) : 0.0f;
    }
  }
}

// FP64 enclosed volume (1/6) sum_t x_a . (x_b x x_c) of each cell.
template <typename T>
__global__ void __launch_bounds__(256) volume_kernel(ClassSlice<T> cs, const T* __restrict__ pos,
                                                     long long sumN, double* __restrict__ out) {
  __shared__ double red[4];
  const int lc = blockIdx.x;
  const int N = cs.cv.N;
  const long long vb = cs.vert0 + (long long)lc * N;
  double acc[1] = {0.0};
  for (int t = threadIdx.x; t < cs.cv.F; t += blockDim.x) {
    const int4 id = cs.cv.tri_v[t];
    double a[3], b[3], c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      a[d] = (double)pos[d * sumN + vb + id.x];
      b[d] = (double)pos[d * sumN + vb + id.y];
      c[d] = (double)pos[d * sumN + vb + id.z];
    }
    acc[0] += a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) +
              a[2] * (b[0] * c[1] - b[1] * c[0]);
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) out[cs.cell0 + lc] = acc[0] / 6.0;
}

template <typename T>
hipError_t launch_predict(const ClassSlice<T>& cs, const T* pos, const T* vel, const T* force,
                          long long sumN, T* delta, T* cterm, int* status, double h,
                          double alpha, hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  hipLaunchKernelGGL(predict_kernel<T>, dim3(cs.n_cells), dim3(256), 0, st, cs, pos, vel, force,
                     sumN, delta, cterm, status, h, alpha);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_update(const ClassSlice<T>& cs, T* pos, T* vel, long long sumN, const T* delta,
                         double h, hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  hipLaunchKernelGGL(update_kernel<T>, dim3(cs.n_cells), dim3(256), 0, st, cs, pos, vel, sumN,
                     delta, h);
  return hipGetLastError();
}

template <typename T, int CPB>
static size_t residual_smem(int N) {
  return sizeof(double) * ((3 * CPB + 1) / 2) + sizeof(T) * 3 * CPB * ((size_t)N + 1);
}

// Cells per workgroup: the most (up to 6 in FP32, 4 in FP64) whose delta fits
// 64 KB of LDS.
template <typename T>
hipError_t launch_residual(const ClassSlice<T>& cs, const T* rhs, const T* delta,
                           const T* delta0, T* res, const T* weights, float* colmax,
                           const float* need, double need_factor, double need_thr,
                           double cmass, double clap, double cvol, hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  const int N = cs.cv.N;
  const int block = std::min(kResidualBlock, (cs.cv.Npad + 63) / 64 * 64);
  const size_t cap = 64 * 1024;
  auto go = [&](auto kern, int cpb, size_t smem) {
    hipLaunchKernelGGL(kern, dim3((cs.n_cells + cpb - 1) / cpb), dim3(block), smem, st, cs, rhs,
                       delta, delta0, res, weights, colmax, need, need_factor, need_thr, cmass,
                       clap, cvol);
    return hipGetLastError();
  };
  if constexpr (sizeof(T) == 4) {  // (6 FP64 cells would not fit the registers)
    if (residual_smem<T, 6>(N) <= cap) return go(residual_kernel<T, 6>, 6, residual_smem<T, 6>(N));
  }
  if (residual_smem<T, 4>(N) <= cap) return go(residual_kernel<T, 4>, 4, residual_smem<T, 4>(N));
  if (residual_smem<T, 2>(N) <= cap) return go(residual_kernel<T, 2>, 2, residual_smem<T, 2>(N));
  if (residual_smem<T, 1>(N) <= cap) return go(residual_kernel<T, 1>, 1, residual_smem<T, 1>(N));
  return hipErrorInvalidValue;
}

// Staging buffer of npfem_get_volume_noalloc (one double per cell), for callers
// that cannot allocate device memory. Every device holds its own copy until
// the process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (volume_scratch below).
static __device__ __align__(256) double scratch[kVolumeScratchCells];

hipError_t volume_scratch(double** out) {
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(p);
  }
  *out = addr[dev];
  return hipSuccess;
}

template <typename T>
hipError_t launch_volume(const ClassSlice<T>& cs, const T* pos, long long sumN, double* out,
                         hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  hipLaunchKernelGGL(volume_kernel<T>, dim3(cs.n_cells), dim3(256), 0, st, cs, pos, sumN, out);
  return hipGetLastError();
}

#define NPFEM_INST(T)                                                                            \
  template hipError_t launch_predict<T>(const ClassSlice<T>&, const T*, const T*, const T*,      \
                                        long long, T*, T*, int*, double, double, hipStream_t);   \
  template hipError_t launch_update<T>(const ClassSlice<T>&, T*, T*, long long, const T*, double, \
                                       hipStream_t);                                             \
  template hipError_t launch_residual<T>(const ClassSlice<T>&, const T*, const T*, const T*, T*, \
                                         const T*, float*, const float*, double, double, double, \
                                         double, double, hipStream_t);                           \
  template hipError_t launch_volume<T>(const ClassSlice<T>&, const T*, long long, double*,       \
                                       hipStream_t);
NPFEM_INST(float)
NPFEM_INST(double)
#undef NPFEM_INST

// dst = s src (n values)
template <typename T>
__global__ void __launch_bounds__(256) scale_kernel(const T* __restrict__ src, T* __restrict__ dst,
                                                    long long n, double s) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = T(s * (double)src[i]);
}

template <typename T>
hipError_t launch_scale(const T* src, T* dst, long long n, double s, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(scale_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n, s);
  return hipGetLastError();
}
template hipError_t launch_scale<float>(const float*, float*, long long, double, hipStream_t);
template hipError_t launch_scale<double>(const double*, double*, long long, double, hipStream_t);

}  // namespace npfem
