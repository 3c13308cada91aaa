// Pieces shared by the local-step kernel and its adjoint: LDS vertex
// records and the volume projection (closest point of q on V(p) = V_rest).
#pragma once

#include "device_utils.h"
#include "npfem_internal.h"

namespace npfem {

template <typename T>
struct alignas(4 * sizeof(T)) V4 {
  T x, y, z, w;
};

template <typename T>
struct alignas(2 * sizeof(T)) V2 {
  T x, y;
};

template <typename T>
__device__ __forceinline__ T comp(const V4<T>& v, int d) {
  return d == 0 ? v.x : (d == 1 ? v.y : v.z);
}

// grad_v V(p) = (1/6) sum over the fan of v of p_b x p_c, (v, b, c)
// counter-clockwise; padding fan entries point at the zero record ps[N].
template <typename T>
__device__ __forceinline__ void volume_gradient(const ClassView<T>& cv, const V4<T>* ps, int v,
                                                T& gx, T& gy, T& gz) {
  const int N = cv.N;
  gx = gy = gz = T(0);
  const int* __restrict__ fix = cv.vt_fan + v;
#pragma unroll 6
  for (int k = 0; k < cv.DT; ++k) {
    const int bc = fix[k * N];
    const V4<T> pb = ps[bc & 0xffff];
    const V4<T> pc = ps[bc >> 16];
    gx += pb.y * pc.z - pb.z * pc.y;
    gy += pb.z * pc.x - pb.x * pc.z;
    gz += pb.x * pc.y - pb.y * pc.x;
  }
  gx *= T(1.0 / 6.0);
  gy *= T(1.0 / 6.0);
  gz *= T(1.0 / 6.0);
}

// Volume projection by the fixed-point map
//   p <- q + lam grad V(p),  lam = (V_rest - V(p) - grad V(p).(q - p)) / |grad V(p)|^2,
// with V(p) = (1/3) sum_v p_v . grad_v V(p) (Euler: V is cubic); per-vertex
// dot products in T, sums over the cell in FP64. Stops when the last change
// of lam moves the cell by less than vol_tol of the correction itself or
// than vol_abs absolutely (|dp|_2 = |d lam| |grad V|_2). On return ps[0..N)
// holds p, ps[N] = 0, g the gradient at the last iterate that produced p, and
// the value is lam. Call from uniform control flow (contains barriers).
template <typename T, int BLOCK, int VPT>
__device__ double volume_project(const ClassView<T>& cv, const V4<T>* qs, V4<T>* ps, double* red,
                                 T (&g)[VPT][3], int max_it, double vol_tol, double vol_abs,
                                 int& bad) {
  const int N = cv.N, tid = threadIdx.x;
  for (int v = tid; v < N; v += BLOCK) ps[v] = qs[v];
  if (tid == 0) ps[N] = V4<T>{T(0), T(0), T(0), T(0)};
  __syncthreads();
  double lam = 0.0;
  for (int it = 0; it < max_it; ++it) {
    double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      g[j][0] = g[j][1] = g[j][2] = T(0);
      if (v < N) {
        T gx, gy, gz;
        volume_gradient(cv, ps, v, gx, gy, gz);
        g[j][0] = gx;
        g[j][1] = gy;
        g[j][2] = gz;
        const V4<T> p = ps[v];
        const V4<T> q = qs[v];
        s[0] += (double)(p.x * gx + p.y * gy + p.z * gz);
        s[1] += (double)(gx * gx + gy * gy + gz * gz);
        s[2] += (double)(gx * (q.x - p.x) + gy * (q.y - p.y) + gz * (q.z - p.z));
      }
    }
    block_sum<3>(s, red);  // barrier: all reads of ps are done
    double lam_new = (cv.vol_rest - s[0] / 3.0 - s[2]) / s[1];
    if (!isfinite(lam_new)) {
      bad = 1;
      lam_new = 0.0;
    }
    const T lt = T(lam_new);
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      if (v < N) {
        const V4<T> q = qs[v];
        V4<T> p;
        p.x = q.x + lt * g[j][0];
        p.y = q.y + lt * g[j][1];
        p.z = q.z + lt * g[j][2];
        p.w = T(0);
        ps[v] = p;
      }
    }
    __syncthreads();
    const double gn = sqrt(s[1]);
    const bool conv = fabs(lam_new - lam) * gn <= fmax(vol_tol * fabs(lam_new) * gn, vol_abs);
    lam = lam_new;
    if (conv) break;
  }
  return lam;
}

}  // namespace npfem
