// Device-side element projections of the local step and their
// vector-Jacobian products (used by the forward and the adjoint kernels).
//
// Triangle projections are written through the invariants of the right
// Cauchy-Green tensor S = F^T F (F the 3x2 deformation gradient):
//   I1 = tr S = s1^2 + s2^2,  J = sqrt(det S) = s1 s2,  tau = s1 + s2 = sqrt(I1 + 2J).
// Strain (nearest matrix with orthonormal columns, the polar factor):
//   Ps = F W,  W = S^{-1/2} = ((I1 + J) I - S) / (J tau).
// Area (nearest matrix with s1 s2 = 1): stationarity of |d - s|^2 / 2 -
// mu (d1 d2 - 1) gives d1 = (s1 + mu s2)/(1 - mu^2), d2 = (s2 + mu s1)/(1 - mu^2),
// so with the same singular vectors
//   Pa = F M,  M = (I + (mu/J) adj S) / (1 - mu^2),
// where mu is a root of g(mu) = (1 - mu^2)^2 - J (1 + mu^2) - mu I1 (the
// constraint d1 d2 = 1). Neither form needs the singular vectors, and both are
// smooth where s1 = s2.
// Which root: with s1 >= s2, the nearest point is d = (t, 1/t) with t the
// largest positive root of t^4 - s1 t^3 + s2 t - 1 (its multiplier is
// mu = t (t - s1)), and that mu is the only root of g in (-1, 1): g(-1) =
// (s1 - s2)^2 >= 0, g(1) = -(I1 + 2J) < 0, and on (-1, -s2/s1] the product
// (s1 + mu s2)(s2 + mu s1) is <= 0, so g > 0 there; the other roots of g lie
// outside [-1, 1] and give a farther stationary point (or a negative d).
#pragma once

#include <hip/hip_runtime.h>

namespace npfem {

// FP32 uses the hardware square root and reciprocal (about 1 ulp); FP64 keeps
// the correctly rounded forms.
__device__ __forceinline__ float f_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double f_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float f_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double f_rcp(double x) { return 1.0 / x; }
// 1 / sqrt(x): FP32 the hardware reciprocal square root (about 1 ulp), FP64
// the correctly rounded square root and division.
__device__ __forceinline__ float f_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double f_rsq(double x) { return 1.0 / sqrt(x); }

// g(mu) and g'(mu) of the area multiplier's equation.
template <typename T>
__device__ __forceinline__ void area_g(T mu, T J, T I1, T& g, T& dg) {
  const T u = T(1) - mu * mu;
  g = u * u - J * (T(1) + mu * mu) - mu * I1;
  dg = T(-4) * mu * u - T(2) * J * mu - I1;
}

// The area multiplier: the root of g in (-1, 1) (see the header).
// Fast path: NEWTON unconditional steps from the linearisation (1 - J)/I1,
// exact to first order in the strain (errors go ~e^2 -> e^4 -> e^8), accepted
// when the last step is below the tolerance and the iterate lies in (-1, 1),
// which then makes it the wanted root. Otherwise (strong compression or
// stretch): Newton safeguarded by bisection on the bracket [-1, 1], where g
// changes sign once. The tolerance is relative (2^-12 FP32, 2^-26 FP64: the
// error after such a step is of the order of its square) plus an absolute
// floor at the rounding noise of g near rest (J ~ 1 cancels 1 - mu^2).
// Sets bad when the safeguarded iteration does not settle.
template <typename T, int NEWTON>
__device__ __forceinline__ T area_multiplier(T J, T I1, int& bad) {
  constexpr T rtol = sizeof(T) == 4 ? T(1.0 / 4096.0) : T(1.0 / 67108864.0);
  constexpr T atol = sizeof(T) == 4 ? T(4.76837158203125e-7) : T(8.881784197001252e-16);
  T mu = (T(1) - J) * f_rcp(I1);
  T g, dg, step = T(0);
#pragma unroll
  for (int it = 0; it < NEWTON; ++it) {
    area_g(mu, J, I1, g, dg);
    step = g * f_rcp(dg);
    mu -= step;
  }
  if (fabs(step) <= rtol * fabs(mu) + atol && fabs(mu) < T(1)) return mu;
  T lo = T(-1), hi = T(1);
  mu = T(0);
  for (int it = 0; it < 96; ++it) {
    area_g(mu, J, I1, g, dg);
    if (g > T(0)) {
      lo = mu;
    } else if (g < T(0)) {
      hi = mu;
    } else {
      return mu;  // exact root (or NaN input, flagged by the caller's tests)
    }
    step = g * f_rcp(dg);
    T next = mu - step;
    const T tol = rtol * fabs(mu) + atol;
    if (fabs(step) <= tol) return (next >= lo && next <= hi) ? next : mu;
    if (!(next > lo && next < hi)) next = T(0.5) * (lo + hi);
    mu = next;
    if (hi - lo <= tol) return mu;
  }
  bad = 1;
  return mu;
}

template <typename T>
struct TriProj;
template <typename T>
__device__ __forceinline__ void triangle_targets(const T (&f)[3][2], TriProj<T>& P);

template <typename T>
struct TriProj {
  T a, b, c;        // S = [[a, b], [b, c]]
  T I1, J, tau;     // invariants
  T iJ;             // 1 / J
  T w00, w01, w11;  // W = S^{-1/2}
  T mu, om;         // area multiplier, 1 / (1 - mu^2)
  T m00, m01, m11;  // M
  T ps[3][2];       // strain projection F W
  T pa[3][2];       // area projection F M
};

// TARGETS: also form P.ps and P.pa (the forward step applies W and M through
// triangle_force instead). FP32 takes J and 1/J from one reciprocal square
// root of |f0 x f1|^2, and 1/tau likewise; FP64 keeps square roots and
// divisions.
template <typename T, int NEWTON, bool TARGETS = true>
__device__ __forceinline__ void project_triangle(const T (&f)[3][2], TriProj<T>& P, int& bad) {
  P.a = f[0][0] * f[0][0] + f[1][0] * f[1][0] + f[2][0] * f[2][0];
  P.b = f[0][0] * f[0][1] + f[1][0] * f[1][1] + f[2][0] * f[2][1];
  P.c = f[0][1] * f[0][1] + f[1][1] * f[1][1] + f[2][1] * f[2][1];
  const T nx = f[1][0] * f[2][1] - f[2][0] * f[1][1];
  const T ny = f[2][0] * f[0][1] - f[0][0] * f[2][1];
  const T nz = f[0][0] * f[1][1] - f[1][0] * f[0][1];
  P.I1 = P.a + P.c;
  const T n2 = nx * nx + ny * ny + nz * nz;  // |f0 x f1|^2 = det S
  T iJ, iw;
  if constexpr (sizeof(T) == 4) {
    iJ = f_rsq(n2);
    P.J = n2 * iJ;
    // (the test on n2 also catches a zero or denormal area, where
    // the reciprocal square root is infinite)
    if (!(n2 > T(1e-24) * P.I1 * P.I1) || !isfinite(P.I1)) bad = 1;
    const T t2 = P.I1 + T(2) * P.J;
    const T itau = f_rsq(t2);
    P.tau = t2 * itau;
    iw = iJ * itau;
  } else {
    P.J = f_sqrt(n2);
    if (!(P.J > T(1e-12) * P.I1) || !isfinite(P.I1)) bad = 1;
    P.tau = f_sqrt(P.I1 + T(2) * P.J);
    iw = f_rcp(P.J * P.tau);
    iJ = f_rcp(P.J);
  }
  P.iJ = iJ;
  P.w00 = (P.I1 + P.J - P.a) * iw;  // ((I1 + J) I - S) / (J tau)
  P.w01 = -P.b * iw;
  P.w11 = (P.I1 + P.J - P.c) * iw;
  const T mu = area_multiplier<T, NEWTON>(P.J, P.I1, bad);
  P.mu = mu;
  P.om = f_rcp(T(1) - mu * mu);
  if (!isfinite(P.om)) bad = 1;
  const T k = mu * iJ;  // M = (I + (mu/J) adj S)/(1 - mu^2), adj S = [[c, -b], [-b, a]]
  P.m00 = (T(1) + k * P.c) * P.om;
  P.m01 = -k * P.b * P.om;
  P.m11 = (T(1) + k * P.a) * P.om;
  if constexpr (TARGETS) triangle_targets(f, P);
}

template <typename T>
__device__ __forceinline__ void triangle_targets(const T (&f)[3][2], TriProj<T>& P) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    P.ps[d][0] = f[d][0] * P.w00 + f[d][1] * P.w01;
    P.ps[d][1] = f[d][0] * P.w01 + f[d][1] * P.w11;
    P.pa[d][0] = f[d][0] * P.m00 + f[d][1] * P.m01;
    P.pa[d][1] = f[d][0] * P.m01 + f[d][1] * P.m11;
  }
}

// The triangle's term of the local step, area (w_s (Ps - F) + w_a (Pa - F)),
// as F Z with the symmetric 2x2 Z = area (w_s (W - I) + w_a (M - I)); M - I
// in the cancellation-free form (mu^2 I + (mu/J) adj S) / (1 - mu^2).
template <typename T>
__device__ __forceinline__ void triangle_force(const T (&f)[3][2], const TriProj<T>& P, T area,
                                               T ws, T wa, T (&w)[3][2]) {
  const T k = P.mu * P.iJ * P.om, u = P.mu * P.mu * P.om;
  const T z00 = area * (ws * (P.w00 - T(1)) + wa * fma(k, P.c, u));
  const T z01 = area * (ws * P.w01 - wa * k * P.b);
  const T z11 = area * (ws * (P.w11 - T(1)) + wa * fma(k, P.a, u));
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    w[d][0] = f[d][0] * z00 + f[d][1] * z01;
    w[d][1] = f[d][0] * z01 + f[d][1] * z11;
  }
}

// VJP of the strain projection. With R = F W, U = W^{-1}, dR = R Omega +
// (I - R R^T) dF W where Omega = om J2 (J2 = [[0,-1],[1,0]]) solves
// Omega U + U Omega = R^T dF - dF^T R, i.e. om = <dF, R J2> / tau. Hence
//   F_bar = (I - R R^T) G W + (mu'/tau) R J2,   mu' = (R^T G)_10 - (R^T G)_01.
template <typename T>
__device__ __forceinline__ void vjp_strain(const TriProj<T>& P, const T (&g)[3][2],
                                           T (&out)[3][2]) {
  T rg[2][2];  // R^T G
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      rg[i][j] = P.ps[0][i] * g[0][j] + P.ps[1][i] * g[1][j] + P.ps[2][i] * g[2][j];
  const T sk = (rg[1][0] - rg[0][1]) * f_rcp(P.tau);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    // (I - R R^T) G = G - R (R^T G)
    const T h0 = g[d][0] - (P.ps[d][0] * rg[0][0] + P.ps[d][1] * rg[1][0]);
    const T h1 = g[d][1] - (P.ps[d][0] * rg[0][1] + P.ps[d][1] * rg[1][1]);
    out[d][0] += h0 * P.w00 + h1 * P.w01 + sk * P.ps[d][1];
    out[d][1] += h0 * P.w01 + h1 * P.w11 - sk * P.ps[d][0];
  }
}

// VJP of the area projection Pa = F M(S). With Q = sym(F^T G):
//   <Q, dM> = c_mu dmu + c_J dJ + (mu / (J (1 - mu^2))) <adj Q, dS>,
//   dmu = (mu dI1 + (1 + mu^2) dJ) / g_mu   (implicit function of g = 0),
//   dI1 = <I, dS>,  dJ = <adj S, dS> / (2 J),
// so <Q, dM> = <Z, dS> and F_bar = G M + 2 F Z.
template <typename T>
__device__ __forceinline__ void vjp_area(const T (&f)[3][2], const TriProj<T>& P,
                                         const T (&g)[3][2], T (&out)[3][2]) {
  T q00 = T(0), q01 = T(0), q10 = T(0), q11 = T(0);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    q00 += f[d][0] * g[d][0];
    q01 += f[d][0] * g[d][1];
    q10 += f[d][1] * g[d][0];
    q11 += f[d][1] * g[d][1];
  }
  const T qs01 = T(0.5) * (q01 + q10);
  const T mu = P.mu, J = P.J, iJ = f_rcp(J), om = P.om;
  const T q_adjS = q00 * P.c - T(2) * qs01 * P.b + q11 * P.a;  // <Q, adj S>
  const T q_I = q00 + q11;
  const T c_mu = q_adjS * iJ * om + T(2) * mu * (q_I + mu * iJ * q_adjS) * om * om;
  const T c_J = -mu * q_adjS * iJ * iJ * om;
  const T g_mu = T(-4) * mu * (T(1) - mu * mu) - T(2) * J * mu - P.I1;
  const T ig = f_rcp(g_mu);
  const T k1 = c_mu * mu * ig;
  const T kJ = (c_J + c_mu * (T(1) + mu * mu) * ig) * T(0.5) * iJ;
  const T kq = mu * iJ * om;
  // Z = k1 I + kJ adj S + kq adj Q_s
  const T z00 = k1 + kJ * P.c + kq * q11;
  const T z01 = -kJ * P.b - kq * qs01;
  const T z11 = k1 + kJ * P.a + kq * q00;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    out[d][0] += g[d][0] * P.m00 + g[d][1] * P.m01 + T(2) * (f[d][0] * z00 + f[d][1] * z01);
    out[d][1] += g[d][0] * P.m01 + g[d][1] * P.m11 + T(2) * (f[d][0] * z01 + f[d][1] * z11);
  }
}

}  // namespace npfem
