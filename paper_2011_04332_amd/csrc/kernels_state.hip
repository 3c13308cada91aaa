// Streaming kernels around the PD iterations: predict, update, the
// refinement residual and per-cell volumes.
//
// Layouts: the caller's state is SoA [3][sumN]; the solver's column buffers
// hold one column per (cell, coordinate) of Npad entries (rows >= N are zero),
// so that the global step is a plain GEMM over 3 * cells columns.
#include <algorithm>

#include "device_utils.h"
#include "npfem_internal.h"

namespace npfem {

// Predict (start of a time step, delta form). With s = x + h v + (h^2/m) f:
//   cterm  = (m/h^2)(s - x) = (m/h) v + f   (constant over the PD iterations)
//   delta0 = s - x = (h^2/m) cterm          (q^0 = s)
template <typename T>
__global__ void __launch_bounds__(256) predict_kernel(ClassSlice<T> cs, const T* __restrict__ pos,
                                                      const T* __restrict__ vel,
                                                      const T* __restrict__ force, long long sumN,
                                                      T* __restrict__ delta, T* __restrict__ cterm,
                                                      int* status, double h) {
  const int lc = blockIdx.x;
  const int N = cs.cv.N, Npad = cs.cv.Npad;
  const long long vb = cs.vert0 + (long long)lc * N;
  const long long cb = cs.elem0 + 3LL * lc * Npad;
  const double m = (double)cs.mass;
  const double mh = m / h, hm = h * h / m;
  int bad = 0;
  for (int v = threadIdx.x; v < Npad; v += blockDim.x) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T c = T(0), dl = T(0);
      if (v < N) {
        const T x = pos[d * sumN + vb + v];
        const T u = vel[d * sumN + vb + v];
        const T f = force[d * sumN + vb + v];
        bad |= !(isfinite(x) && isfinite(u) && isfinite(f));
        const double cd = mh * (double)u + (double)f;
        c = T(cd);
        dl = T(h * (double)u + hm * (double)f);
      }
      cterm[cb + d * Npad + v] = c;
      delta[cb + d * Npad + v] = dl;
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
  for (int v = threadIdx.x; v < N; v += blockDim.x) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const T dl = delta[cb + d * Npad + v];
      pos[d * sumN + vb + v] += dl;
      vel[d * sumN + vb + v] = T((double)dl * ih);
    }
  }
}

// Refinement residual res = r - A_c delta for each cell, with the per-cell
// system A_c = (m/h^2 + w_v) I + (w_s + w_a) L_tri + w_b L_bend (fixed-width
// rows of the two Laplacians, shared by the class). One workgroup per cell
// with one thread per row (up to 1024 rows at a time), so that a wave has few
// memory round trips in sequence and many waves share each SIMD. The cell's
// delta is staged in LDS (N + 1 values per coordinate, the last one 0 for
// padding entries); products accumulate in FP64. colmax: per column max
// |res| (FP16 scaling): wave maxima, then LDS atomic max on the bit patterns
// of the non-negative floats.
template <typename T>
__global__ void __launch_bounds__(1024) residual_kernel(ClassSlice<T> cs, const T* __restrict__ rhs,
                                                        const T* __restrict__ delta,
                                                        T* __restrict__ res,
                                                        const T* __restrict__ weights,
                                                        float* __restrict__ colmax, double h) {
  extern __shared__ double smem_res[];
  unsigned* cmx = reinterpret_cast<unsigned*>(smem_res);  // [3]
  T* sd = reinterpret_cast<T*>(smem_res + 2);             // [3][N + 1]
  const int N = cs.cv.N, Npad = cs.cv.Npad, DL = cs.cv.DL;
  const int lc = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const long long cb = cs.elem0 + 3LL * lc * Npad;
  const int* __restrict__ lcol = cs.cv.lap_col;
  const T* __restrict__ lt = cs.cv.lap_t;
  const T* __restrict__ lb = cs.cv.lap_b;
  for (int v = tid; v <= N; v += nt) {
    const int vc = min(v, N - 1);
    const T dx = delta[cb + vc], dy = delta[cb + Npad + vc], dz = delta[cb + 2 * Npad + vc];
    sd[v] = v < N ? dx : T(0);
    sd[(N + 1) + v] = v < N ? dy : T(0);
    sd[2 * (N + 1) + v] = v < N ? dz : T(0);
  }
  if (tid < 3) cmx[tid] = 0u;
  __syncthreads();
  const int cell = cs.cell0 + lc;
  double w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = weights ? (double)weights[4 * cell + k] : (double)cs.w_nom[k];
  const double diag = (double)cs.mass / (h * h) + w[3];
  const double wt = w[0] + w[1], wb = w[2];
  float cm[3] = {0.f, 0.f, 0.f};
  for (int v = tid; v < Npad; v += nt) {
    double a0 = 0, a1 = 0, a2 = 0;
    if (v < N) {
      const T r0 = rhs[cb + v], r1 = rhs[cb + Npad + v], r2 = rhs[cb + 2 * Npad + v];
      a0 = diag * (double)sd[v];
      a1 = diag * (double)sd[(N + 1) + v];
      a2 = diag * (double)sd[2 * (N + 1) + v];
      // row entries fetched 8 at a time (the slots past the last clamped,
      // their weight zeroed)
      for (int k0 = 0; k0 < DL; k0 += 8) {
        int jj[8];
        T ct[8], cbv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = min(k0 + u, DL - 1) * N + v;
          jj[u] = lcol[e];
          ct[u] = lt[e];
          cbv[u] = lb[e];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double c = k0 + u < DL ? wt * (double)ct[u] + wb * (double)cbv[u] : 0.0;
          const int j = jj[u];
          a0 += c * (double)sd[j];
          a1 += c * (double)sd[(N + 1) + j];
          a2 += c * (double)sd[2 * (N + 1) + j];
        }
      }
      a0 = (double)r0 - a0;
      a1 = (double)r1 - a1;
      a2 = (double)r2 - a2;
    }
    res[cb + v] = T(a0);
    res[cb + Npad + v] = T(a1);
    res[cb + 2 * Npad + v] = T(a2);
    cm[0] = fmaxf(cm[0], fabsf((float)a0));
    cm[1] = fmaxf(cm[1], fabsf((float)a1));
    cm[2] = fmaxf(cm[2], fabsf((float)a2));
  }
  if (colmax) {
    // wave maxima first, then one LDS atomic per wave and coordinate
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float mx = wave_max(cm[d]);
      if ((tid & (kWave - 1)) == 0) atomicMax(&cmx[d], __float_as_uint(mx));
    }
    __syncthreads();
    if (tid < 3) colmax[cs.col0 + 3LL * lc + tid] = __uint_as_float(cmx[tid]);
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
                          hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  hipLaunchKernelGGL(predict_kernel<T>, dim3(cs.n_cells), dim3(256), 0, st, cs, pos, vel, force,
                     sumN, delta, cterm, status, h);
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

template <typename T>
hipError_t launch_residual(const ClassSlice<T>& cs, const T* rhs, const T* delta, T* res,
                           const T* weights, float* colmax, double h, hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  const int N = cs.cv.N;
  const size_t smem = 2 * sizeof(double) + sizeof(T) * 3 * ((size_t)N + 1);
  if (smem > 64 * 1024) return hipErrorInvalidValue;
  const int block = std::min(1024, (cs.cv.Npad + 63) / 64 * 64);
  hipLaunchKernelGGL(residual_kernel<T>, dim3(cs.n_cells), dim3(block), smem, st, cs, rhs, delta,
                     res, weights, colmax, h);
  return hipGetLastError();
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
                                        long long, T*, T*, int*, double, hipStream_t);           \
  template hipError_t launch_update<T>(const ClassSlice<T>&, T*, T*, long long, const T*, double, \
                                       hipStream_t);                                             \
  template hipError_t launch_residual<T>(const ClassSlice<T>&, const T*, const T*, T*, const T*, \
                                         float*, double, hipStream_t);                           \
  template hipError_t launch_volume<T>(const ClassSlice<T>&, const T*, long long, double*,       \
                                       hipStream_t);
NPFEM_INST(float)
NPFEM_INST(double)
#undef NPFEM_INST

}  // namespace npfem
