// Reverse of one projective-dynamics iteration, one workgroup per cell.
//
// Forward iteration: q' = A^-1 b(P(q), s; w) with A = (m/h^2 + w_v) I +
// (w_s + w_a) L_tri + w_b L_bend. Given g' = dL/dq' the host first solves
// lam = A^-1 g' (A is symmetric: the same GEMM as the forward). This kernel
// then forms, from q = q^k, q' = q^{k+1} and lam:
//   dL/dw_s += sum_t A_t <F_t(lam), Ps_t(q) - F_t(q')>        (and w_a with Pa)
//   dL/dw_b += sum_e c_e <y_e(lam), Pb_e(q) - y_e(q')>
//   dL/dw_v += <lam, Pv(q) - q'>
//   dL/ds   += (m/h^2) lam
//   dL/dq    = sum_i (dP_i/dq)^T (w_i S_i lam)     (projection VJPs)
// The volume VJP uses the implicit function theorem on the projection's
// optimality conditions p - q - mu grad V(p) = 0, V(p) = V_rest: with
// H = hess V(p), g = grad V(p),
//   u = (I - mu H)^-1 pbar,  w = (I - mu H)^-1 g,  qbar = u - (g.u / g.w) w,
// where (I - mu H)^-1 is applied to first order (I + mu H): |mu H| is the
// volume correction per unit length, 1e-7..1e-4 at the solver's operating
// points. Element VJPs go through LDS and are gathered per vertex in a fixed
// order, as in the forward kernel.
//
// The element arithmetic runs in FP64 also for FP32 state (see the kernel).
// The weight-gradient residuals P_i(q) - S_i q' are formed in displacement
// form, (P_i(q) - S_i q) + S_i (q - q'), and the volume's P(q) - q = lam grad V
// is taken from the projection itself: near rest the residual is far smaller
// than the positions. q is the point the forward local step projected, the
// rounded sum x + delta^k, while the forward's next iterate is x + delta^{k+1}
// held as its increment; so q - q' = (q - x) - delta^{k+1}, formed in FP64
// from the stored values (q - x is exact there), which keeps the rounding of
// q itself (an ulp of the coordinates, for FP32 state as large as the
// residual's own scale near rest) and of positions rebuilt from q' out of it.
#include <algorithm>

#include "device_utils.h"
#include "local_common.h"
#include "npfem_internal.h"
#include "projections.h"

namespace npfem {

template <typename T>
struct AdjLaunch {
  AdjArgs<T> a;
  int tch;
  int hch;
};

template <typename T>
__device__ __forceinline__ void cross_acc(const V4<T>& a, const V4<T>& b, T (&o)[3]) {
  o[0] += a.y * b.z - a.z * b.y;
  o[1] += a.z * b.x - a.x * b.z;
  o[2] += a.x * b.y - a.y * b.x;
}

// Register budget: a 642-vertex cell's FP32 adjoint step (512 threads, two
// vertices per thread, 62 KB of LDS) leaves LDS for two workgroups per CU,
// which needs at most 128 registers (four waves per SIMD); uncapped it took
// 150 and ran one workgroup per CU. At the cap a few values spill (80 bytes
// per thread), and the backward pass is still 10 % faster.
template <typename T, int BLOCK, int VPT>
constexpr int adjoint_waves_per_eu() {
  return sizeof(T) == 4 && BLOCK == 512 && VPT <= 2 ? 4 : 1;
}

template <typename T, int BLOCK, int VPT>
__global__ void __launch_bounds__(BLOCK, (adjoint_waves_per_eu<T, BLOCK, VPT>()))
    adjoint_local_kernel(AdjLaunch<T> L) {
  extern __shared__ double smem_adj[];
  constexpr int NW = BLOCK / kWave;
  // Element arithmetic (projections, their VJPs and the weight-gradient
  // residuals) in FP64 for both state types, from FP64 element records (G,
  // area, K, c, r): near rest the residuals P_i(q) - S_i q are ~1e-3 of the
  // O(1) terms they are formed from, and the weight gradients sum them
  // against lam with heavy cancellation, so an FP32 rounding of G or K alone
  // moves them by ~1e-3 (a rest shape perturbed at 1e-7).
  using A = double;
  const AdjArgs<T>& a = L.a;
  const ClassView<T>& cv = a.cs.cv;
  const int N = cv.N, Npad = cv.Npad, F = cv.F, E = cv.E, DT = cv.DT, DH = cv.DH;
  const int tid = threadIdx.x;
  const int lc = blockIdx.x;
  const int cell = a.cs.cell0 + lc;
  const long long vb = a.cs.vert0 + (long long)lc * N;
  const long long cb = a.cs.elem0 + 3LL * lc * Npad;
  const T* __restrict__ px = a.xn + vb;
  const T* __restrict__ py = px + a.sumN;
  const T* __restrict__ pz = py + a.sumN;
  const T* __restrict__ d0 = a.delta_k + cb;
  const T* __restrict__ d1 = a.delta_k1 + cb;
  const T* __restrict__ lcol = a.lam + cb;
  T* __restrict__ gout = a.gbar + cb;
  T* __restrict__ sb = a.sbar + cb;

  double* red = smem_adj;  // 8 * NW doubles
  V4<T>* qs = reinterpret_cast<V4<T>*>(smem_adj + 8 * NW);  // q^k
  V4<T>* dds = qs + N;                                        // q^k - q^{k+1}
  V4<T>* ls = dds + N;                                        // lam, N + 1 records
  T* work = reinterpret_cast<T*>(ls + N + 1);

  T ws, wa, wb, wv;
  if (a.weights) {
    ws = a.weights[4 * cell + 0];
    wa = a.weights[4 * cell + 1];
    wb = a.weights[4 * cell + 2];
    wv = a.weights[4 * cell + 3];
  } else {
    ws = a.cs.w_nom[0];
    wa = a.cs.w_nom[1];
    wb = a.cs.w_nom[2];
    wv = a.cs.w_nom[3];
  }
  int bad = 0;
  double wacc[4] = {0.0, 0.0, 0.0, 0.0};

  // the records of vertex v: q = x + delta_0 (rounded as the forward staged
  // it), q - q' = (q - x) - delta_1, lambda
  auto fetch = [&](int v, V4<T>& q, V4<T>& dd, V4<T>& l) {
    const T x0 = px[v], x1 = py[v], x2 = pz[v];
    q = V4<T>{x0 + d0[v], x1 + d0[Npad + v], x2 + d0[2 * Npad + v], T(0)};
    dd = V4<T>{T(((A)q.x - (A)x0) - (A)d1[v]), T(((A)q.y - (A)x1) - (A)d1[Npad + v]),
               T(((A)q.z - (A)x2) - (A)d1[2 * Npad + v]), T(0)};
    l = V4<T>{lcol[v], lcol[Npad + v], lcol[2 * Npad + v], T(0)};
  };
  if constexpr (VPT <= 4) {
    // every vertex set's loads in flight at once (VPT * BLOCK >= N, clamped
    // reads)
    V4<T> fq[VPT], fd[VPT], fl[VPT];
#pragma unroll
    for (int j = 0; j < VPT; ++j) fetch(min(tid + j * BLOCK, N - 1), fq[j], fd[j], fl[j]);
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      if (v < N) {
        qs[v] = fq[j];
        dds[v] = fd[j];
        ls[v] = fl[j];
      }
    }
  } else {
    for (int v = tid; v < N; v += BLOCK) fetch(v, qs[v], dds[v], ls[v]);
  }
  if (tid == 0) ls[N] = V4<T>{T(0), T(0), T(0), T(0)};
  __syncthreads();

  T acc[VPT][3];
#pragma unroll
  for (int j = 0; j < VPT; ++j) acc[j][0] = acc[j][1] = acc[j][2] = T(0);

  // ---- volume ----
  {
    V4<T>* ps = reinterpret_cast<V4<T>*>(work);  // N + 1 records
    V4<T>* gs = ps + N + 1;                      // N + 1 records
    // The projection p = q + mu grad V(p), V(p) = V_rest (the fixed point of
    // the forward's volume step) in FP64 arithmetic for both state types:
    // the iterate is kept as its displacement from q, which is small, so T
    // records (in gs while iterating) hold it far below the rounding of q.
    // Near rest mu grad V is the volume weight's residual itself, and an
    // FP32 evaluation of V(q) would carry ~1e-3 of it.
    T g[VPT][3];
    A gd[VPT][3];
    A mu = A(0);
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      if (v < N) gs[v] = V4<T>{T(0), T(0), T(0), T(0)};
    }
    if (tid == 0) gs[N] = V4<T>{T(0), T(0), T(0), T(0)};
    __syncthreads();
    const int passes = max(2, a.max_vol_iter);
    for (int it = 0; it < passes; ++it) {
      double sv[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int j = 0; j < VPT; ++j) {
        const int v = tid + j * BLOCK;
        gd[j][0] = gd[j][1] = gd[j][2] = A(0);
        if (v < N) {
          // grad_v V(p) = (1/6) sum over the fan of p_b x p_c, p = q + d
          const int* __restrict__ fix = cv.vt_fan + v * DT;
          for (int k = 0; k < DT; ++k) {
            const int bc = fix[k], ib = bc & 0xffff, ic = bc >> 16;
            const V4<T> qb = qs[ib], db = gs[ib], qc = qs[ic], dc = gs[ic];
            const A bx = (A)qb.x + (A)db.x, by = (A)qb.y + (A)db.y, bz = (A)qb.z + (A)db.z;
            const A cx = (A)qc.x + (A)dc.x, cy = (A)qc.y + (A)dc.y, cz = (A)qc.z + (A)dc.z;
            gd[j][0] += by * cz - bz * cy;
            gd[j][1] += bz * cx - bx * cz;
            gd[j][2] += bx * cy - by * cx;
          }
          const V4<T> qv = qs[v], dv = gs[v];
          const A dd3[3] = {(A)dv.x, (A)dv.y, (A)dv.z};
          const A pp[3] = {(A)qv.x + dd3[0], (A)qv.y + dd3[1], (A)qv.z + dd3[2]};
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            gd[j][d] *= A(1.0 / 6.0);
            sv[0] += pp[d] * gd[j][d];
            sv[1] += gd[j][d] * gd[j][d];
            sv[2] -= gd[j][d] * dd3[d];  // grad V . (q - p)
          }
        }
      }
      block_sum<3>(sv, red);
      const A mu_new = (cv.vol_rest - sv[0] / 3.0 - sv[2]) / sv[1];
      if (!isfinite(mu_new)) bad = 1;
      const bool conv = it > 0 && fabs(mu_new - mu) <= 1e-14 * fabs(mu_new);  // (uniform)
      mu = isfinite(mu_new) ? mu_new : A(0);
      __syncthreads();  // every read of the displacement records is done
#pragma unroll
      for (int j = 0; j < VPT; ++j) {
        const int v = tid + j * BLOCK;
        if (v < N) gs[v] = V4<T>{T(mu * gd[j][0]), T(mu * gd[j][1]), T(mu * gd[j][2]), T(0)};
      }
      __syncthreads();
      if (conv) break;
    }
    // p and grad V(p) as records for the Hessian products below
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      g[j][0] = T(gd[j][0]);
      g[j][1] = T(gd[j][1]);
      g[j][2] = T(gd[j][2]);
      if (v < N) {
        const V4<T> qv = qs[v], dv = gs[v];
        ps[v] = V4<T>{T((A)qv.x + (A)dv.x), T((A)qv.y + (A)dv.y), T((A)qv.z + (A)dv.z), T(0)};
      }
    }
    __syncthreads();  // every displacement record is read
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      if (v < N) gs[v] = V4<T>{g[j][0], g[j][1], g[j][2], T(0)};
    }
    if (tid == 0) {
      ps[N] = V4<T>{T(0), T(0), T(0), T(0)};
      gs[N] = V4<T>{T(0), T(0), T(0), T(0)};
    }
    __syncthreads();
    const T mt = T(mu);
    T u[VPT][3], w[VPT][3];
    double r[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      u[j][0] = u[j][1] = u[j][2] = T(0);
      w[j][0] = w[j][1] = w[j][2] = T(0);
      if (v < N) {
        // (H z)_v = (1/6) sum over the fan of (z_b x p_c + p_b x z_c)
        T hl[3] = {T(0), T(0), T(0)}, hg[3] = {T(0), T(0), T(0)};
        const int* __restrict__ fix = cv.vt_fan + v * DT;
        for (int k0 = 0; k0 < DT; k0 += 8) {
          int bcs[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) bcs[e] = fix[min(k0 + e, DT - 1)];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            if (k0 + e >= DT) break;
            const int ib = bcs[e] & 0xffff, ic = bcs[e] >> 16;
            const V4<T> pb = ps[ib], pc = ps[ic];
            cross_acc(ls[ib], pc, hl);
            cross_acc(pb, ls[ic], hl);
            cross_acc(gs[ib], pc, hg);
            cross_acc(pb, gs[ic], hg);
          }
        }
        const V4<T> l = ls[v];
        const T lv[3] = {l.x, l.y, l.z};
        const T c6 = mt * T(1.0 / 6.0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          u[j][d] = wv * (lv[d] + c6 * hl[d]);  // pbar = w_v lam
          w[j][d] = g[j][d] + c6 * hg[d];
        }
        r[0] += (double)(g[j][0] * u[j][0] + g[j][1] * u[j][1] + g[j][2] * u[j][2]);
        r[1] += (double)(g[j][0] * w[j][0] + g[j][1] * w[j][1] + g[j][2] * w[j][2]);
        // P_v(q) - q' = mu grad V + (q - q')
        const V4<T> dq = dds[v];
        wacc[3] += (A)l.x * (mu * gd[j][0] + (A)dq.x) + (A)l.y * (mu * gd[j][1] + (A)dq.y) +
                   (A)l.z * (mu * gd[j][2] + (A)dq.z);
      }
    }
    block_sum<2>(r, red);
    const T beta = T(r[0] / r[1]);
    if (!isfinite(r[0] / r[1])) bad = 1;
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
#pragma unroll
      for (int d = 0; d < 3; ++d) acc[j][d] += u[j][d] - beta * w[j][d];
    }
    __syncthreads();
  }

  // ---- triangles: strain + area ----
  for (int base = 0; base < F; base += L.tch) {
    const int nt = min(L.tch, F - base);
    int4 idn = tid < nt ? cv.tri_v[base + tid] : int4{0, 0, 0, 0};
    for (int t = base + tid; t < base + nt; t += BLOCK) {
      const int4 id = idn;
      if (t + BLOCK < base + nt) idn = cv.tri_v[t + BLOCK];
      // the element records in FP64 for both state types
      const V4<A> r0 = reinterpret_cast<const V4<A>*>(cv.tri_rec64)[2 * t];
      const V4<A> r1 = reinterpret_cast<const V4<A>*>(cv.tri_rec64)[2 * t + 1];
      const A g00 = r0.x, g01 = r0.y, g10 = r0.z, g11 = r0.w, g20 = r1.x, g21 = r1.y;
      const A area = r1.z;
      A fq[3][2], fd[3][2], fl[3][2];  // F(q), F(q - q'), F(lam)
      {
        const V4<T> qa = qs[id.x], qb = qs[id.y], qc = qs[id.z];
        const V4<T> ua = dds[id.x], ub = dds[id.y], uc = dds[id.z];
        const V4<T> la = ls[id.x], lb = ls[id.y], lcc = ls[id.z];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          // F(q) from the edge vectors, as in the forward step
          const A e1 = (A)comp(qb, d) - (A)comp(qa, d), e2 = (A)comp(qc, d) - (A)comp(qa, d);
          fq[d][0] = e1 * g10 + e2 * g20;
          fq[d][1] = e1 * g11 + e2 * g21;
          fd[d][0] = (A)comp(ua, d) * g00 + (A)comp(ub, d) * g10 + (A)comp(uc, d) * g20;
          fd[d][1] = (A)comp(ua, d) * g01 + (A)comp(ub, d) * g11 + (A)comp(uc, d) * g21;
          fl[d][0] = (A)comp(la, d) * g00 + (A)comp(lb, d) * g10 + (A)comp(lcc, d) * g20;
          fl[d][1] = (A)comp(la, d) * g01 + (A)comp(lb, d) * g11 + (A)comp(lcc, d) * g21;
        }
      }
      TriProj<A> P;
      project_triangle<A, 4>(fq, P, bad);
      A es = A(0), ea = A(0);
      A gs2[3][2], ga2[3][2], fb[3][2];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          es += fl[d][k] * ((P.ps[d][k] - fq[d][k]) + fd[d][k]);
          ea += fl[d][k] * ((P.pa[d][k] - fq[d][k]) + fd[d][k]);
          gs2[d][k] = (A)ws * area * fl[d][k];
          ga2[d][k] = (A)wa * area * fl[d][k];
          fb[d][k] = A(0);
        }
      }
      wacc[0] += (double)(area * es);
      wacc[1] += (double)(area * ea);
      vjp_strain(P, gs2, fb);
      vjp_area(fq, P, ga2, fb);
      T* wsl = work + 6 * (t - base);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        wsl[2 * d] = T(fb[d][0]);
        wsl[2 * d + 1] = T(fb[d][1]);
      }
    }
    __syncthreads();
    const bool whole = (nt == F);
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      if (v < N) {
        const int* __restrict__ tix = cv.vt_tri + v * DT;
        const V2<T>* __restrict__ gix = reinterpret_cast<const V2<T>*>(cv.vt_g) + v * DT;
        for (int k0 = 0; k0 < DT; k0 += 8) {
          int ts[8];
          V2<T> gs2[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            ts[e] = tix[min(k0 + e, DT - 1)];
            gs2[e] = gix[min(k0 + e, DT - 1)];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            if (k0 + e >= DT) break;
            const int t = ts[e] - base;
            if (!whole && (t < 0 || t >= nt)) continue;
            const T* w6 = work + 6 * t;
            acc[j][0] += gs2[e].x * w6[0] + gs2[e].y * w6[1];
            acc[j][1] += gs2[e].x * w6[2] + gs2[e].y * w6[3];
            acc[j][2] += gs2[e].x * w6[4] + gs2[e].y * w6[5];
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- hinges: bending ----
  for (int base = 0; base < E; base += L.hch) {
    const int ne = min(L.hch, E - base);
    V4<T>* ys = reinterpret_cast<V4<T>*>(work);
    int4 idn = tid < ne ? cv.hin_v[base + tid] : int4{0, 0, 0, 0};
    for (int e = base + tid; e < base + ne; e += BLOCK) {
      const int4 id = idn;
      if (e + BLOCK < base + ne) idn = cv.hin_v[e + BLOCK];
      const V4<A> r0 = reinterpret_cast<const V4<A>*>(cv.hin_rec64)[2 * e];
      const V4<A> r1 = reinterpret_cast<const V4<A>*>(cv.hin_rec64)[2 * e + 1];
      const A k0 = r0.x, k1 = r0.y, k2 = r0.z, k3 = r0.w, ce = r1.x, rr = r1.y;
      A yq[3], yd[3], yl[3];  // y(q), y(q - q'), y(lam)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        // y(q) from the differences to q_i, as in the forward step
        const A qi_d = (A)comp(qs[id.x], d);
        yq[d] = k1 * ((A)comp(qs[id.y], d) - qi_d) + k2 * ((A)comp(qs[id.z], d) - qi_d) +
                k3 * ((A)comp(qs[id.w], d) - qi_d);
        yd[d] = k0 * (A)comp(dds[id.x], d) + k1 * (A)comp(dds[id.y], d) +
                k2 * (A)comp(dds[id.z], d) + k3 * (A)comp(dds[id.w], d);
        yl[d] = k0 * (A)comp(ls[id.x], d) + k1 * (A)comp(ls[id.y], d) +
                k2 * (A)comp(ls[id.z], d) + k3 * (A)comp(ls[id.w], d);
      }
      const A n2 = yq[0] * yq[0] + yq[1] * yq[1] + yq[2] * yq[2];
      const A in = n2 > A(0) ? f_rsq(n2) : A(0);
      const A sc = n2 > A(0) ? rr * in : A(1);
      A eb = A(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) eb += yl[d] * ((sc - A(1)) * yq[d] + yd[d]);
      wacc[2] += (double)(ce * eb);
      // Pb = r y/|y|: Jacobian (r/|y|)(I - yh yh^T), symmetric
      const A wc = (A)wb * ce;
      A pb[3] = {wc * yl[0], wc * yl[1], wc * yl[2]};
      V4<T> yb;
      if (n2 > A(0)) {
        const A yh0 = yq[0] * in, yh1 = yq[1] * in, yh2 = yq[2] * in;
        const A dp = yh0 * pb[0] + yh1 * pb[1] + yh2 * pb[2];
        yb = V4<T>{T(sc * (pb[0] - yh0 * dp)), T(sc * (pb[1] - yh1 * dp)),
                   T(sc * (pb[2] - yh2 * dp)), T(0)};
      } else {
        yb = V4<T>{T(pb[0]), T(pb[1]), T(pb[2]), T(0)};
      }
      ys[e - base] = yb;
    }
    __syncthreads();
    const bool whole = (ne == E);
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      if (v < N) {
        const int* __restrict__ hix = cv.vh_hin + v * DH;
        const T* __restrict__ kix = cv.vh_k + v * DH;
        for (int k0 = 0; k0 < DH; k0 += 8) {
          int hs[8];
          T ks[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            hs[e] = hix[min(k0 + e, DH - 1)];
            ks[e] = kix[min(k0 + e, DH - 1)];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            if (k0 + e >= DH) break;
            const int hh = hs[e] - base;
            if (!whole && (hh < 0 || hh >= ne)) continue;
            const V4<T> y = ys[hh];
            acc[j][0] += ks[e] * y.x;
            acc[j][1] += ks[e] * y.y;
            acc[j][2] += ks[e] * y.z;
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- outputs ----
  const T ms = T(a.m / (a.h * a.h));
#pragma unroll
  for (int j = 0; j <= VPT; ++j) {
    const int v = tid + j * BLOCK;
    if (v < Npad) {
      if (v < N) {
        const V4<T> l = ls[v];
        const T lv[3] = {l.x, l.y, l.z};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          gout[d * Npad + v] = acc[j < VPT ? j : VPT - 1][d];
          sb[d * Npad + v] += ms * lv[d];
        }
      } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) gout[d * Npad + v] = T(0);
      }
    }
  }
  block_sum<4>(wacc, red);
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) a.wbar[4 * cell + i] += wacc[i];
    if (!isfinite(wacc[0] + wacc[1] + wacc[2] + wacc[3])) bad = 1;
  }
  if (__syncthreads_or(bad) && tid == 0) atomicOr(a.status, ST_NONFINITE);
}

// Start of a reversed step: g = dL/dq^K = xbar + vbar / h (x' = q^K,
// v' = (q^K - x)/h), sbar = 0.
template <typename T>
__global__ void __launch_bounds__(256) adj_begin_kernel(ClassSlice<T> cs, const T* __restrict__ xbar,
                                                        const T* __restrict__ vbar, long long sumN,
                                                        T* __restrict__ gbar, T* __restrict__ sbar,
                                                        double h) {
  const int lc = blockIdx.x;
  const int N = cs.cv.N, Npad = cs.cv.Npad;
  const long long vb = cs.vert0 + (long long)lc * N;
  const long long cb = cs.elem0 + 3LL * lc * Npad;
  const T ih = T(1.0 / h);
  for (int v = threadIdx.x; v < Npad; v += blockDim.x) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T gv = T(0);
      if (v < N) gv = xbar[d * sumN + vb + v] + vbar[d * sumN + vb + v] * ih;
      gbar[cb + d * Npad + v] = gv;
      sbar[cb + d * Npad + v] = T(0);
    }
  }
}

// End of a reversed step: with S = sbar + dL/dq^0 (q^0 = s),
//   xbar <- -vbar/h + S,  vbar <- h S,  fbar += (h^2/m) S
// (s = x + h v + (h^2/m) f).
template <typename T>
__global__ void __launch_bounds__(256) adj_end_kernel(ClassSlice<T> cs, T* __restrict__ xbar,
                                                      T* __restrict__ vbar, long long sumN,
                                                      const T* __restrict__ gbar,
                                                      const T* __restrict__ sbar,
                                                      T* __restrict__ fbar, double h) {
  const int lc = blockIdx.x;
  const int N = cs.cv.N, Npad = cs.cv.Npad;
  const long long vb = cs.vert0 + (long long)lc * N;
  const long long cb = cs.elem0 + 3LL * lc * Npad;
  const T ih = T(1.0 / h), hh = T(h), hm = T(h * h / (double)cs.mass);
  for (int v = threadIdx.x; v < N; v += blockDim.x) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const long long i = d * sumN + vb + v;
      const T S = sbar[cb + d * Npad + v] + gbar[cb + d * Npad + v];
      const T vb_old = vbar[i];
      xbar[i] = S - vb_old * ih;
      vbar[i] = hh * S;
      if (fbar) fbar[i] += hm * S;
    }
  }
}

// LDS: reductions, q, q', lam (N + 1 records) and a work region holding the
// volume iterate and gradient (2 (N + 1) records) or an element chunk.
template <typename T>
size_t adjoint_smem_bytes_chunks(const ClassView<T>& cv, int block, int* tch, int* hch) {
  const size_t fixed =
      8 * sizeof(double) * (block / kWave) + sizeof(T) * 4 * (3 * (size_t)cv.N + 1);
  const size_t max_total = 160 * 1024;
  const size_t work_min = 8 * ((size_t)cv.N + 1);
  const size_t want = std::max<size_t>(6 * (size_t)cv.F, 4 * (size_t)cv.E);
  const size_t avail = max_total > fixed ? (max_total - fixed) / sizeof(T) : 0;
  size_t budget = std::min(want, std::max(work_min, std::min(avail, (size_t)16384)));
  if (budget < work_min) budget = work_min;
  const int t = (int)std::min<size_t>(cv.F, budget / 6);
  const int h = (int)std::min<size_t>(cv.E, budget / 4);
  if (tch) *tch = std::max(t, 1);
  if (hch) *hch = std::max(h, 1);
  return fixed + sizeof(T) * budget;
}

template <typename T>
using AdjFn = void (*)(AdjLaunch<T>);

template <typename T, int BLOCK>
static AdjFn<T> pick_adj_vpt(int N) {
  const int vpt = (N + BLOCK - 1) / BLOCK;
  if (vpt <= 1) return adjoint_local_kernel<T, BLOCK, 1>;
  if (vpt <= 2) return adjoint_local_kernel<T, BLOCK, 2>;
  if (vpt <= 3) return adjoint_local_kernel<T, BLOCK, 3>;
  if (vpt <= 6) return adjoint_local_kernel<T, BLOCK, 6>;
  return nullptr;
}

template <typename T>
static int adjoint_block(int N) {
  return N <= 256 ? 256 : 512;
}

template <typename T>
hipError_t adjoint_prepare(const ClassView<T>& cv) {
  const int block = adjoint_block<T>(cv.N);
  AdjFn<T> fn = block == 256 ? pick_adj_vpt<T, 256>(cv.N) : pick_adj_vpt<T, 512>(cv.N);
  if (!fn) return hipErrorInvalidValue;
  const size_t smem = adjoint_smem_bytes_chunks(cv, block, nullptr, nullptr);
  if (smem > 160 * 1024) return hipErrorInvalidValue;
  if (smem > 64 * 1024)
    return hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)smem);
  return hipSuccess;
}

template <typename T>
hipError_t launch_adjoint_local(const AdjArgs<T>& a, hipStream_t st) {
  if (a.cs.n_cells == 0) return hipSuccess;
  const int block = adjoint_block<T>(a.cs.cv.N);
  AdjFn<T> fn = block == 256 ? pick_adj_vpt<T, 256>(a.cs.cv.N) : pick_adj_vpt<T, 512>(a.cs.cv.N);
  if (!fn) return hipErrorInvalidValue;
  AdjLaunch<T> L;
  L.a = a;
  const size_t smem = adjoint_smem_bytes_chunks(a.cs.cv, block, &L.tch, &L.hch);
  if (smem > 160 * 1024) return hipErrorInvalidValue;
  void* args[] = {&L};
  return hipLaunchKernel((const void*)fn, dim3(a.cs.n_cells), dim3(block), args, smem, st);
}

template <typename T>
hipError_t launch_adj_begin(const ClassSlice<T>& cs, const T* xbar, const T* vbar, long long sumN,
                            T* gbar, T* sbar, double h, hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  hipLaunchKernelGGL(adj_begin_kernel<T>, dim3(cs.n_cells), dim3(256), 0, st, cs, xbar, vbar, sumN,
                     gbar, sbar, h);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_end(const ClassSlice<T>& cs, T* xbar, T* vbar, long long sumN,
                          const T* gbar, const T* sbar, T* fbar, double h, hipStream_t st) {
  if (cs.n_cells == 0) return hipSuccess;
  hipLaunchKernelGGL(adj_end_kernel<T>, dim3(cs.n_cells), dim3(256), 0, st, cs, xbar, vbar, sumN,
                     gbar, sbar, fbar, h);
  return hipGetLastError();
}

#define NPFEM_INST(T)                                                                             \
  template hipError_t adjoint_prepare<T>(const ClassView<T>&);                                   \
  template hipError_t launch_adjoint_local<T>(const AdjArgs<T>&, hipStream_t);                   \
  template hipError_t launch_adj_begin<T>(const ClassSlice<T>&, const T*, const T*, long long,   \
                                          T*, T*, double, hipStream_t);                          \
  template hipError_t launch_adj_end<T>(const ClassSlice<T>&, T*, T*, long long, const T*,       \
                                        const T*, T*, double, hipStream_t);
NPFEM_INST(float)
NPFEM_INST(double)
#undef NPFEM_INST

}  // namespace npfem
