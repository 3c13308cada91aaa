// Quasi-Newton implicit step (L-BFGS on the step's objective with the PD
// matrix as initial Hessian; the redesigned projective dynamics the solver
// follows, Implementation and architecture), the per-cell parts. One
// workgroup per cell; vectors are the batch's column sets (3 columns of Npad
// rows per cell, rows >= N zero); reductions in FP64 with a fixed order.
//
// With g = grad of the objective = -r (r the local step's increment
// right-hand side at the iterate) and the history pairs (s_i, y_i, rho_i)
// in a ring of `hist` slots, newest at head - 1:
//   qn_loop1:   v = g; for newest..oldest: a_i = rho_i s_i.v, v -= a_i y_i
//   (product)   z = A^-1 v
//   qn_loop2:   for oldest..newest: z += (a_i - rho_i y_i.z) s_i; d = -z;
//               gd = g.d; alpha = 1; trial = delta + d
//   (local step at the trial: its r and objective)
//   qn_accept:  Armijo E_trial <= E + c alpha gd + e_tol |E| (or the last
//               round; e_tol covers the rounding of an FP32 state's objective,
//               0 for FP64): store
//               s = trial - delta, y = r - r_trial, rho = 1/(s.y) (0 when
//               s.y <= 0: the pair is inert), take the trial; else halve
//               alpha and form the next trial.
#include "device_utils.h"
#include "npfem_internal.h"

namespace npfem {

constexpr int kQnBlock = 256;
constexpr double kArmijo = 1e-4;

template <typename T>
struct QnCell {
  long long cb;  // first element of the cell's column set
  int Npad;
  int cell;
};

template <typename T>
__device__ __forceinline__ QnCell<T> qn_cell(const ClassSlice<T>& cs) {
  QnCell<T> c;
  c.Npad = cs.cv.Npad;
  c.cb = cs.elem0 + 3LL * blockIdx.x * c.Npad;
  c.cell = cs.cell0 + blockIdx.x;
  return c;
}

// rows handled by a thread: r = tid + j * kQnBlock over the 3 Npad entries
constexpr int kQnRows = (3 * 2576 + kQnBlock - 1) / kQnBlock;  // up to Npad 2576

template <typename T, int R>
__device__ __forceinline__ double qn_dot(const T* __restrict__ a, const T (&x)[R], int n3,
                                         double* red) {
  double s[1] = {0.0};
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int e = threadIdx.x + j * kQnBlock;
    if (e < n3) s[0] += (double)a[e] * (double)x[j];
  }
  block_sum<1>(s, red);
  return s[0];
}

template <typename T, int R>
__global__ void __launch_bounds__(kQnBlock) qn_loop1_kernel(ClassSlice<T> cs, QnArgs<T> q,
                                                             int count, int head) {
  __shared__ double red[kQnBlock / kWave];
  const QnCell<T> c = qn_cell(cs);
  const int n3 = 3 * c.Npad;
  T v[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int e = threadIdx.x + j * kQnBlock;
    v[j] = e < n3 ? -q.r_cur[c.cb + e] : T(0);
  }
  for (int u = 0; u < count; ++u) {
    const int i = (head - 1 - u + q.hist) % q.hist;
    const T* __restrict__ si = q.s[i] + c.cb;
    const T* __restrict__ yi = q.y[i] + c.cb;
    const double a = q.scal[c.cell * q.stride + kQnRho + i] * qn_dot<T, R>(si, v, n3, red);
    if (threadIdx.x == 0) q.scal[c.cell * q.stride + kQnA + i] = a;
    const T at = T(a);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int e = threadIdx.x + j * kQnBlock;
      if (e < n3) v[j] -= at * yi[e];
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int e = threadIdx.x + j * kQnBlock;
    if (e < n3) q.v[c.cb + e] = v[j];
  }
}

template <typename T, int R>
__global__ void __launch_bounds__(kQnBlock) qn_loop2_kernel(ClassSlice<T> cs, QnArgs<T> q,
                                                             int count, int head) {
  __shared__ double red[kQnBlock / kWave];
  const QnCell<T> c = qn_cell(cs);
  const int n3 = 3 * c.Npad;
  double* sc = q.scal + c.cell * q.stride;
  T z[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int e = threadIdx.x + j * kQnBlock;
    z[j] = e < n3 ? q.z[c.cb + e] : T(0);
  }
  for (int u = count - 1; u >= 0; --u) {
    const int i = (head - 1 - u + q.hist) % q.hist;
    const T* __restrict__ si = q.s[i] + c.cb;
    const T* __restrict__ yi = q.y[i] + c.cb;
    const double beta = sc[kQnRho + i] * qn_dot<T, R>(yi, z, n3, red);
    const T k = T(sc[kQnA + i] - beta);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int e = threadIdx.x + j * kQnBlock;
      if (e < n3) z[j] += k * si[e];
    }
  }
  // d = -z; gd = g.d = r.z; trial = delta + d
  double gd[1] = {0.0};
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int e = threadIdx.x + j * kQnBlock;
    if (e < n3) {
      const long long o = c.cb + e;
      gd[0] += (double)q.r_cur[o] * (double)z[j];
      q.d[o] = -z[j];
      q.delta_trial[o] = q.delta[o] - z[j];
    }
  }
  block_sum<1>(gd, red);
  if (threadIdx.x == 0) {
    sc[kQnGd] = gd[0];
    sc[kQnAlpha] = 1.0;
    q.done[c.cell] = 0;
  }
}

template <typename T, int R>
__global__ void __launch_bounds__(kQnBlock) qn_accept_kernel(ClassSlice<T> cs, QnArgs<T> q,
                                                              int head, int last, int it) {
  __shared__ double red[kQnBlock / kWave];
  const QnCell<T> c = qn_cell(cs);
  const int n3 = 3 * c.Npad;
  if (q.done[c.cell]) return;  // (uniform)
  double* sc = q.scal + c.cell * q.stride;
  const double E = q.e_cur[c.cell], Et = q.e_trial[c.cell];
  const double alpha = sc[kQnAlpha];
  const bool take = last || Et <= E + kArmijo * alpha * sc[kQnGd] + q.e_tol * fabs(E);
  if (take) {
    T* __restrict__ si = q.hist > 0 ? q.s[head] + c.cb : nullptr;
    T* __restrict__ yi = q.hist > 0 ? q.y[head] + c.cb : nullptr;
    double sy[1] = {0.0};
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int e = threadIdx.x + j * kQnBlock;
      if (e < n3) {
        const long long o = c.cb + e;
        const T dt = q.delta_trial[o], rt = q.r_trial[o];
        const T s = dt - q.delta[o];
        const T y = q.r_cur[o] - rt;
        sy[0] += (double)s * (double)y;
        if (si) {
          si[e] = s;
          yi[e] = y;
        }
        q.delta[o] = dt;
        q.r_cur[o] = rt;
      }
    }
    block_sum<1>(sy, red);
    if (threadIdx.x == 0) {
      if (q.hist > 0) sc[kQnRho + head] = sy[0] > 0.0 ? 1.0 / sy[0] : 0.0;
      q.e_cur[c.cell] = Et;
      if (q.energy && it + 1 < q.energy_iters) q.energy[(size_t)(it + 1) * q.n_cells + c.cell] = Et;
      q.done[c.cell] = 1;
    }
  } else {
    const double a2 = 0.5 * alpha;
    const T at = T(a2);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int e = threadIdx.x + j * kQnBlock;
      if (e < n3) {
        const long long o = c.cb + e;
        q.delta_trial[o] = q.delta[o] + at * q.d[o];
      }
    }
    if (threadIdx.x == 0) sc[kQnAlpha] = a2;
  }
}

// rows per thread for a class (3 Npad entries over kQnBlock threads)
template <typename T>
static int qn_rows(int Npad) {
  return (3 * Npad + kQnBlock - 1) / kQnBlock;
}

#define QN_DISPATCH(KERNEL, ...)                                                              \
  do {                                                                                        \
    const int rows = qn_rows<T>(cs.cv.Npad);                                                  \
    if (rows <= 3)                                                                            \
      hipLaunchKernelGGL((KERNEL<T, 3>), dim3(cs.n_cells), dim3(kQnBlock), 0, st, __VA_ARGS__); \
    else if (rows <= 8)                                                                       \
      hipLaunchKernelGGL((KERNEL<T, 8>), dim3(cs.n_cells), dim3(kQnBlock), 0, st, __VA_ARGS__); \
    else if (rows <= kQnRows)                                                                 \
      hipLaunchKernelGGL((KERNEL<T, kQnRows>), dim3(cs.n_cells), dim3(kQnBlock), 0, st,       \
                         __VA_ARGS__);                                                        \
    else                                                                                      \
      return hipErrorInvalidValue;                                                            \
  } while (0)

template <typename T>
hipError_t launch_qn_loop1(const ClassSlice<T>& cs, const QnArgs<T>& q, int count, int head,
                           hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  QN_DISPATCH(qn_loop1_kernel, cs, q, count, head);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_qn_loop2(const ClassSlice<T>& cs, const QnArgs<T>& q, int count, int head,
                           hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  QN_DISPATCH(qn_loop2_kernel, cs, q, count, head);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_qn_accept(const ClassSlice<T>& cs, const QnArgs<T>& q, int head, int last,
                            int it, hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  QN_DISPATCH(qn_accept_kernel, cs, q, head, last, it);
  return hipGetLastError();
}

#define NPFEM_INST(T)                                                                         \
  template hipError_t launch_qn_loop1<T>(const ClassSlice<T>&, const QnArgs<T>&, int, int,    \
                                         hipStream_t);                                        \
  template hipError_t launch_qn_loop2<T>(const ClassSlice<T>&, const QnArgs<T>&, int, int,    \
                                         hipStream_t);                                        \
  template hipError_t launch_qn_accept<T>(const ClassSlice<T>&, const QnArgs<T>&, int, int, int, \
                                          hipStream_t);
NPFEM_INST(float)
NPFEM_INST(double)
#undef NPFEM_INST

}  // namespace npfem
