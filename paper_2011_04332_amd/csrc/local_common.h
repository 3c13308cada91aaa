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

// Three-component record (12 bytes in FP32): the local step's LDS vertex
// records, so that a 642-vertex cell's step fits four workgroups per CU.
template <typename T>
struct alignas(sizeof(T)) V3 {
  T x, y, z;
};

template <typename T>
__device__ __forceinline__ T comp(const V4<T>& v, int d) {
  return d == 0 ? v.x : (d == 1 ? v.y : v.z);
}
template <typename T>
__device__ __forceinline__ T comp(const V3<T>& v, int d) {
  return d == 0 ? v.x : (d == 1 ? v.y : v.z);
}

// Record of the local step's LDS vertex arrays: 12 bytes in FP32, a
// 32-byte vector record in FP64.
template <typename T>
struct LocalRec {
  typedef V4<T> type;
};
template <>
struct LocalRec<float> {
  typedef V3<float> type;
};

template <typename R>
__device__ __forceinline__ R make_rec(decltype(R::x) x, decltype(R::x) y, decltype(R::x) z) {
  R r{};
  r.x = x;
  r.y = y;
  r.z = z;
  return r;
}

// grad_v V(p) = (1/6) sum over the fan of v of p_b x p_c, (v, b, c)
// counter-clockwise; padding fan entries point at record N (b = c gives an
// exact zero cross product whatever the record holds). KT > 0 fixes the fan
// width at compile time (it must equal cv.DT): all indices are fetched in
// one round trip before any is used. KT = 0 reads cv.DT, 8 entries a time.
template <typename T, int KT, typename R>
__device__ __forceinline__ void volume_gradient(const ClassView<T>& cv, const R* ps, int v,
                                                T& gx, T& gy, T& gz) {
  const int N = cv.N;
  gx = gy = gz = T(0);
  const int* __restrict__ fix = cv.vt_fan + v * (KT > 0 ? KT : cv.DT);
  auto add = [&](int bc) {
    const R pb = ps[bc & 0xffff];
    const R pc = ps[bc >> 16];
    gx += pb.y * pc.z - pb.z * pc.y;
    gy += pb.z * pc.x - pb.x * pc.z;
    gz += pb.x * pc.y - pb.y * pc.x;
  };
  if constexpr (KT > 0) {
    int bc[KT];
#pragma unroll
    for (int u = 0; u < KT; ++u) bc[u] = fix[u];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < KT; ++u) add(bc[u]);
  } else {
    const int DT = cv.DT;
    for (int k0 = 0; k0 < DT; k0 += 8) {
      int bc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) bc[u] = k0 + u < DT ? fix[k0 + u] : (N | (N << 16));
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k0 + u < DT) add(bc[u]);
    }
  }
  gx *= T(1.0 / 6.0);
  gy *= T(1.0 / 6.0);
  gz *= T(1.0 / 6.0);
}

// The same sum from the one-ring n_0 .. n_{KT-1} (indices in registers; a
// ring shorter than KT is padded with n_0, whose terms n_0 x n_0 vanish):
// (1/6) sum_k n_k x n_{k+1 mod KT}, one LDS record per neighbour.
template <typename T, int KT, typename R>
__device__ __forceinline__ void volume_gradient_ring(const R* ps, const int (&r)[KT], T& gx,
                                                     T& gy, T& gz) {
  R p[KT];
#pragma unroll
  for (int u = 0; u < KT; ++u) p[u] = ps[r[u]];
  gx = gy = gz = T(0);
#pragma unroll
  for (int u = 0; u < KT; ++u) {
    const R& pb = p[u];
    const R& pc = p[(u + 1) % KT];
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
// starting from p = q, with V(p) = (1/3) sum_v p_v . grad_v V(p) (Euler: V is
// cubic); per-vertex dot products in T, sums over the cell in FP64.
//
// Stopping. After an iteration that is not the first, stop when the change
// of lam moved the cell by less than vol_tol of the correction itself or than
// vol_abs absolutely (|dp|_2 = |d lam| |grad V|_2). After the first, the next
// change is predicted instead: to first order in lam the second iterate
// moves by (3/2) lam^2 |g^T H g| / |g| along g plus lam^2 |H g| (H the
// Hessian of V, g its gradient at q), at most (5/2) lam^2 |H| |g|, and
// |g^T H g| <= |H| |g|^2 with |H| <= (DT / 3) max_v |q_v| (each block H_vw is
// a sum of two cross-product matrices (1/6)[q_u]x, and g^T H g does not
// change under translation). The test takes twice that bound.
//
// On return g holds the gradient that produced p (p = q + lam g) for this
// thread's vertices and the value is lam. With STORE_P, pv holds p and
// ps[0..N) too, with ps[N] = 0, behind a barrier. Without it, pv is left
// unset (the caller takes p - q = lam g, which is also exact where the
// rounded p - q is not), ps is scratch (written only when a second iteration
// runs) and no thread reads it any more. red: 8 * (BLOCK / 64) doubles. KT:
// fan width (0 = runtime; > 0 needs cv.vt_ring, whose rings the caller
// fetches into ring with ring_indices, before it needs them). Call from
// uniform control flow.
template <typename T, int BLOCK, int VPT, int KT>
__device__ __forceinline__ void ring_indices(const ClassView<T>& cv, int (&ring)[VPT][KT]) {
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const int v = min((int)threadIdx.x + j * BLOCK, cv.N - 1);
#pragma unroll
    for (int u = 0; u < KT; ++u) ring[j][u] = cv.vt_ring[v * KT + u];
  }
}

// One pass's per-thread part: the gradient g at src (q itself on the first
// pass) for this thread's vertices and its partial sums s[0] = p.g,
// s[1] = |g|^2, s[2] = g.(q - p) (later passes) and mq = max |q|^2 (first).
template <typename T, int BLOCK, int VPT, int KT, typename R>
__device__ __forceinline__ void volume_pass_local(const ClassView<T>& cv, const R* qs,
                                                  const R* src, bool first,
                                                  T (&g)[VPT][3], double (&s)[3], double& mq,
                                                  const int (&fan)[VPT][KT > 0 ? KT : 1]) {
  const int N = cv.N, tid = threadIdx.x;
  s[0] = s[1] = s[2] = 0.0;
  mq = 0.0;
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const int v = tid + j * BLOCK;
    g[j][0] = g[j][1] = g[j][2] = T(0);
    if (v < N) {
      T gx, gy, gz;
      if constexpr (KT > 0) {
        volume_gradient_ring<T, KT>(src, fan[j], gx, gy, gz);
      } else {
        volume_gradient<T, 0, R>(cv, src, v, gx, gy, gz);
      }
      g[j][0] = gx;
      g[j][1] = gy;
      g[j][2] = gz;
      const R q = qs[v];
      const R p = first ? q : src[v];
      s[0] += (double)(p.x * gx + p.y * gy + p.z * gz);
      s[1] += (double)(gx * gx + gy * gy + gz * gz);
      if (!first) s[2] += (double)(gx * (q.x - p.x) + gy * (q.y - p.y) + gz * (q.z - p.z));
      else mq = fmax(mq, (double)(q.x * q.x + q.y * q.y + q.z * q.z));
    }
  }
}

// The multiplier of pass it from the cell totals, and the stopping test
// (see volume_project).
template <typename T>
__device__ __forceinline__ double volume_lambda(const ClassView<T>& cv, const double (&s)[3],
                                                double mq, int it, double lam_prev,
                                                double vol_tol, double vol_abs, int& bad,
                                                bool& conv) {
  double lam_new = (cv.vol_rest - s[0] / 3.0 - s[2]) / s[1];
  if (!isfinite(lam_new)) {
    bad = 1;
    lam_new = 0.0;
  }
  const double gn = sqrt(s[1]);
  const double allow = fmax(vol_tol * fabs(lam_new) * gn, vol_abs);
  if (it == 0) {
    const double hb = (double)cv.DT / 3.0 * sqrt(mq);
    conv = 5.0 * lam_new * lam_new * hb * gn <= allow;
  } else {
    conv = fabs(lam_new - lam_prev) * gn <= allow;
  }
  return lam_new;
}

// Passes after the first `done` ones, whose last gave (lam, g, conv): publish
// p = q + lam g, take the gradient there, and so on (see volume_project).
// Uses red halves (pass & 1); ps needs N + 1 records. Call from uniform
// control flow.
template <typename T, int BLOCK, int VPT, bool STORE_P, int KT, typename R>
__device__ double volume_continue(const ClassView<T>& cv, const R* qs, R* ps,
                                  double* red, T (&g)[VPT][3], T (&pv)[VPT][3], double lam,
                                  bool conv, int done, int max_it, double vol_tol,
                                  double vol_abs, int& bad,
                                  const int (&fan)[VPT][KT > 0 ? KT : 1]) {
  const int N = cv.N, tid = threadIdx.x;
  bool stored = false;
  for (int it = done;; ++it) {
    const bool last = conv || it >= max_it;
    if (last && !STORE_P) break;
    // publish p for the next pass's gradient (or for the caller)
    const T lt = T(lam);
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      const R q = v < N ? qs[v] : make_rec<R>(T(0), T(0), T(0));
      pv[j][0] = q.x + lt * g[j][0];
      pv[j][1] = q.y + lt * g[j][1];
      pv[j][2] = q.z + lt * g[j][2];
      if (v < N) ps[v] = make_rec<R>(pv[j][0], pv[j][1], pv[j][2]);
    }
    if (!stored && tid == 0) ps[N] = make_rec<R>(T(0), T(0), T(0));
    stored = true;
    __syncthreads();
    if (last) break;
    double s[3], mq;
    volume_pass_local<T, BLOCK, VPT, KT, R>(cv, qs, ps, false, g, s, mq, fan);
    // one barrier; afterwards every read of ps in this pass is done
    block_sum_max<3, false>(s, mq, red, it & 1);
    lam = volume_lambda<T>(cv, s, mq, it, lam, vol_tol, vol_abs, bad, conv);
  }
  return lam;
}

template <typename T, int BLOCK, int VPT, bool STORE_P, int KT = 0, typename R = V4<T>>
__device__ double volume_project(const ClassView<T>& cv, const R* qs, R* ps, double* red,
                                 T (&g)[VPT][3], T (&pv)[VPT][3], int max_it, double vol_tol,
                                 double vol_abs, int& bad,
                                 const int (&fan)[VPT][KT > 0 ? KT : 1]) {
  double s[3], mq;
  volume_pass_local<T, BLOCK, VPT, KT, R>(cv, qs, qs, true, g, s, mq, fan);
  block_sum_max<3, true>(s, mq, red, 0);
  bool conv;
  const double lam = volume_lambda<T>(cv, s, mq, 0, 0.0, vol_tol, vol_abs, bad, conv);
  return volume_continue<T, BLOCK, VPT, STORE_P, KT, R>(cv, qs, ps, red, g, pv, lam, conv, 1, max_it,
                                                     vol_tol, vol_abs, bad, fan);
}

}  // namespace npfem
