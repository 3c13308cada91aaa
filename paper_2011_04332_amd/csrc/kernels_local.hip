// Local step of projective dynamics plus the right-hand-side gather, one
// workgroup per cell.
//
// For the current iterate q = x + delta (delta form: the global step solves
// A delta = b - A x, with x the positions at the start of the step and
// A = (m/h^2) I + S, S the constraint stiffness), the kernel computes per cell
// the increment right-hand side
//   r = (m/h)v + f - (m/h^2) delta                 (inertia term, precomputed)
//     + sum_t A_t G_t (w_s (Ps_t - F_t(q)) + w_a (Pa_t - F_t(q)))^T
//     + sum_e w_b c_e K_e (x) (Pb_e - y_e(q))
//     + w_v (Pv - q)
// where Ps/Pa are the strain/area projections of F_t(q), Pb the bending
// projection of y_e(q) = sum_r K_e[r] q_r and Pv the closest point of q on the
// rest-volume surface. This is b - A x - A delta (the projections' terms
// against q instead of x differ by S delta), so the global step's solve
// returns the next iterate as delta + A^-1 r; the same iteration as
// delta_next = A^-1 (b - A x), but r no longer needs x at all: only q is
// staged, the element phases read half as much LDS, and r is small (it
// vanishes at the fixed point), which also shrinks the absolute error of a
// 16-bit product.
//
// LDS holds the cell's vertices as 12-byte (FP32) or 32-byte (FP64) records,
// and the per-element contributions, which each vertex then gathers
// through fixed-width incidence lists in a fixed order (no atomics): results
// are bitwise reproducible. Triangles and hinges go through LDS in chunks
// sized to the budget (a vertex adds its entries chunk by chunk, each chunk's
// in list order).
#include <algorithm>

#include "device_utils.h"
#include "local_common.h"
#include "npfem_internal.h"
#include "projections.h"

namespace npfem {

template <typename T>
struct LocalLaunch {
  LocalArgs<T> a;
  int tch;  // triangles per LDS chunk
  int hch;  // hinges per LDS chunk
};

// KT, KH > 0: compile-time incidence widths (triangles and hinges per
// vertex; they must equal cv.DT and cv.DH, and the class must have its
// one-rings, cv.vt_ring), so that every incidence entry of a vertex is
// fetched in one memory round trip before the gathers use them.
// 0: widths read at run time.
// Occupancy target (waves per SIMD) for FP32, which sets the register
// budget (at most 128 registers at four): with 12-byte vertex records the
// LDS of a 642-vertex cell (38.7 KB at 256 threads) lets four workgroups
// share a CU, four waves per SIMD (16-byte records allowed three). The
// extra wave hides more of the gathers' latency than the second LDS
// instruction per 12-byte record read costs. Four vertices per thread
// (meshes of up to 1024 vertices) take three: their LDS leaves room for
// fewer workgroups, and at 128 registers they would spill. Six or more
// vertices per thread means a large mesh whose LDS allows one workgroup per
// CU: no register cap.
template <typename T, int BLOCK, int VPT>
constexpr int local_waves_per_eu() {
  return VPT >= 6 ? 1 : sizeof(T) == 4 ? (VPT <= 3 ? 4 : 3) : 2;
}

// LDS taken by the q records (N + 1) in doubles, rounded up to 16 bytes so
// that the work region's vector records stay aligned.
template <typename T>
__host__ __device__ constexpr int local_q_doubles(int N) {
  return ((int)sizeof(typename LocalRec<T>::type) * (N + 1) + 15) / 16 * 2;
}

template <typename T, int BLOCK, int VPT, int KT, int KH>
__global__ void __launch_bounds__(BLOCK, (local_waves_per_eu<T, BLOCK, VPT>()))
    local_kernel(LocalLaunch<T> L) {
  extern __shared__ double smem_local[];
  constexpr int NW = BLOCK / kWave;
  constexpr int NEWTON = sizeof(T) == 8 ? 4 : 3;  // area multiplier (projections.h)
  const LocalArgs<T>& a = L.a;
  const ClassView<T>& cv = a.cs.cv;
  const int N = cv.N, Npad = cv.Npad, F = cv.F, E = cv.E;
  const int DT = KT > 0 ? KT : cv.DT, DH = KH > 0 ? KH : cv.DH;
  const int tid = threadIdx.x;
  const int lc = blockIdx.x;
  const int cell = a.cs.cell0 + lc;
  if (a.skip && a.skip[cell]) return;  // (uniform)
  const long long vb = a.cs.vert0 + (long long)lc * N;
  const long long cb = a.cs.elem0 + 3LL * lc * Npad;
  // per-cell base pointers: everything below indexes with 32-bit offsets
  const T* __restrict__ px = a.pos + vb;
  const T* __restrict__ py = px + a.sumN;
  const T* __restrict__ pz = py + a.sumN;
  const T* __restrict__ dcol = a.delta + cb;
  const T* __restrict__ ccol = a.cterm + cb;
  T* __restrict__ rcol = a.rhs + cb;

  typedef typename LocalRec<T>::type Q;
  double* red = smem_local;  // 8 * NW doubles
  // q: N records and a zero record N, which the padding entries of the volume
  // fan lists point at (their cross product is 0 only for finite records);
  // the work region starts at the next 16-byte boundary
  Q* qs = reinterpret_cast<Q*>(smem_local + 8 * NW);
  T* work = reinterpret_cast<T*>(smem_local + 8 * NW + local_q_doubles<T>(N));

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
  const bool want_energy = a.energy != nullptr;
  double e_acc = 0.0;
  int bad = 0;

  // the volume gradient's ring indices, requested while q is staged
  int ring[VPT][KT > 0 ? KT : 1];
  if constexpr (KT > 0) ring_indices<T, BLOCK, VPT, KT>(cv, ring);

  // ---- stage q = x + delta (up to six vertex sets per thread: every set's
  // loads in flight at once, VPT * BLOCK >= N, clamped reads) ----
  if constexpr (VPT <= 6) {
    Q sq[VPT];
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = min(tid + j * BLOCK, N - 1);
      sq[j] = make_rec<Q>(px[v] + dcol[v], py[v] + dcol[Npad + v], pz[v] + dcol[2 * Npad + v]);
    }
#pragma unroll
    for (int j = 0; j < VPT; ++j)
      if (tid + j * BLOCK < N) qs[tid + j * BLOCK] = sq[j];
  } else {
    for (int v = tid; v < N; v += BLOCK)
      qs[v] = make_rec<Q>(px[v] + dcol[v], py[v] + dcol[Npad + v], pz[v] + dcol[2 * Npad + v]);
  }
  if (tid == 0) qs[N] = make_rec<Q>(T(0), T(0), T(0));
  __syncthreads();

  T acc[VPT][3];
#pragma unroll
  for (int j = 0; j < VPT; ++j) acc[j][0] = acc[j][1] = acc[j][2] = T(0);

  // ---- volume, first pass: closest point of q on {V(p) = V_rest}
  // (local_common.h). The gradient at q and the waves' partial sums are
  // formed here; the cell totals are read after the triangle phase's first
  // barrier, which so serves the volume reduction too, and any further
  // passes run after the triangle phase (they need the work region). ----
  T g[VPT][3];
  double vs[3], vmq;
  volume_pass_local<T, BLOCK, VPT, KT, Q>(cv, qs, qs, true, g, vs, vmq, ring);
  block_sum_max_write<3, true>(vs, vmq, red, 0);
  bool vol_pending = true, vol_conv = false;
  double lam = 0.0;

  // ---- triangles: strain + area ----
  for (int base = 0; base < F; base += L.tch) {
    const int nt = min(L.tch, F - base);
    // the next element's vertex ids and record are fetched one iteration
    // ahead, so that their round trip overlaps the current element's work
    const V4<T>* __restrict__ trec = reinterpret_cast<const V4<T>*>(cv.tri_rec);
    const int t0 = base + min(tid, nt - 1);
    int4 idn = cv.tri_v[t0];
    V4<T> r0n = trec[2 * t0], r1n = trec[2 * t0 + 1];
    for (int t = base + tid; t < base + nt; t += BLOCK) {
      const int4 id = idn;
      const V4<T> r0 = r0n, r1 = r1n;
      if (t + BLOCK < base + nt) {
        idn = cv.tri_v[t + BLOCK];
        r0n = trec[2 * (t + BLOCK)];
        r1n = trec[2 * (t + BLOCK) + 1];
      }
      const T g00 = r0.x, g01 = r0.y, g10 = r0.z, g11 = r0.w, g20 = r1.x, g21 = r1.y;
      const T area = r1.z;
      const Q qa = qs[id.x], qb = qs[id.y], qc = qs[id.z];
      // F from the edge vectors (the rows of G sum to zero): exactly
      // translation-invariant with the rounded G, and the differences of
      // nearby coordinates are exact, so F carries the rounding of O(1)
      // products instead of the cancellation of O(R/edge) terms
      (void)g00;
      (void)g01;
      T fq[3][2];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T e1 = comp(qb, d) - comp(qa, d), e2 = comp(qc, d) - comp(qa, d);
        fq[d][0] = e1 * g10 + e2 * g20;
        fq[d][1] = e1 * g11 + e2 * g21;
      }
      TriProj<T> P;
      project_triangle<T, NEWTON, false>(fq, P, bad);
      T wt[3][2];
      triangle_force(fq, P, area, ws, wa, wt);
      T* w = work + 6 * (t - base);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        w[2 * d] = wt[d][0];
        w[2 * d + 1] = wt[d][1];
      }
      if (want_energy) {
        triangle_targets(fq, P);
        const T(&ps)[3][2] = P.ps;
        const T(&pa)[3][2] = P.pa;
        double es = 0.0, ea = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const double u = (double)fq[d][k] - (double)ps[d][k];
            const double z = (double)fq[d][k] - (double)pa[d][k];
            es += u * u;
            ea += z * z;
          }
        }
        e_acc += 0.5 * (double)area * ((double)ws * es + (double)wa * ea);
      }
    }
    __syncthreads();
    if (vol_pending) {  // (uniform)
      block_sum_max_read<3, true>(vs, vmq, red, 0);
      lam = volume_lambda<T>(cv, vs, vmq, 0, 0.0, a.vol_tol, a.vol_abs, bad, vol_conv);
      vol_pending = false;
    }
    const bool whole = (nt == F);  // one chunk: every entry is in range
    // two fused multiply-adds per component
    auto tri_add = [&](int j, int t, V2<T> g2) {
      const T* w = work + 6 * t;
      acc[j][0] = fma(g2.y, w[1], fma(g2.x, w[0], acc[j][0]));
      acc[j][1] = fma(g2.y, w[3], fma(g2.x, w[2], acc[j][1]));
      acc[j][2] = fma(g2.y, w[5], fma(g2.x, w[4], acc[j][2]));
    };
    if constexpr (KT > 0) {
      if (whole) {
        // the entries of vertex j + 1 are fetched before vertex j is summed
        // (two register sets), so one round trip overlaps the previous work
        int tt[2][KT];
        V2<T> gg[2][KT];
        auto fetch = [&](int j, int set) {
          const int v = min(tid + j * BLOCK, N - 1);  // clamped: always a valid row
          const int* __restrict__ tp = cv.vt_tri + v * KT;
          const V2<T>* __restrict__ gp = reinterpret_cast<const V2<T>*>(cv.vt_g) + v * KT;
#pragma unroll
          for (int u = 0; u < KT; ++u) {
            tt[set][u] = tp[u];
            gg[set][u] = gp[u];
          }
        };
        fetch(0, 0);
#pragma unroll
        for (int j = 0; j < VPT; ++j) {
          if (j + 1 < VPT) fetch(j + 1, (j + 1) & 1);
          __builtin_amdgcn_sched_barrier(0);
          if (tid + j * BLOCK < N) {
#pragma unroll
            for (int u = 0; u < KT; ++u) tri_add(j, tt[j & 1][u], gg[j & 1][u]);
          }
        }
      }
    }
    if (KT == 0 || !whole) {
#pragma unroll
      for (int j = 0; j < VPT; ++j) {
        const int v = tid + j * BLOCK;
        if (v < N) {
          const int* __restrict__ tix = cv.vt_tri + v * DT;
          const V2<T>* __restrict__ gix = reinterpret_cast<const V2<T>*>(cv.vt_g) + v * DT;
          if (whole) {
#pragma unroll 6
            for (int k = 0; k < DT; ++k) tri_add(j, tix[k], gix[k]);
          } else {
            for (int k = 0; k < DT; ++k) {
              const int t = tix[k] - base;
              if (t < 0 || t >= nt) continue;
              tri_add(j, t, gix[k]);
            }
          }
        }
      }
    }
    __syncthreads();
  }

  if (vol_pending) {  // (a mesh without triangles: no chunk barrier ran)
    __syncthreads();
    block_sum_max_read<3, true>(vs, vmq, red, 0);
    lam = volume_lambda<T>(cv, vs, vmq, 0, 0.0, a.vol_tol, a.vol_abs, bad, vol_conv);
  }
  // ---- volume, further passes (the triangle chunks are done with the work
  // region), then w_v (Pv - q) with Pv - q = lam g ----
  if (!vol_conv && a.max_vol_iter > 1) {  // (uniform)
    int ring2[VPT][KT > 0 ? KT : 1];
    if constexpr (KT > 0) ring_indices<T, BLOCK, VPT, KT>(cv, ring2);
    T p[VPT][3];
    lam = volume_continue<T, BLOCK, VPT, false, KT, Q>(cv, qs, reinterpret_cast<Q*>(work), red,
                                                    g, p, lam, vol_conv, 1, a.max_vol_iter,
                                                    a.vol_tol, a.vol_abs, bad, ring2);
  }
  {
    const T wl = wv * T(lam);
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      if (v < N) {
        acc[j][0] += wl * g[j][0];
        acc[j][1] += wl * g[j][1];
        acc[j][2] += wl * g[j][2];
        if (want_energy) {
          const double g2 = (double)g[j][0] * g[j][0] + (double)g[j][1] * g[j][1] +
                            (double)g[j][2] * g[j][2];
          e_acc += 0.5 * (double)wv * lam * lam * g2;
        }
      }
    }
  }

  // ---- contacts: w_c (Pc - q) with Pc the closest point of q in the
  // half-space of its nearest contact point (first minimum on ties) ----
  if (a.contact_w != 0.0) {  // (uniform)
    const int k0 = a.contact_off[cell], k1 = a.contact_off[cell + 1];
    const T* __restrict__ cpx = a.contact_p;
    const T* __restrict__ cpy = cpx + a.contact_np;
    const T* __restrict__ cpz = cpy + a.contact_np;
    const T* __restrict__ cnx = a.contact_n;
    const T* __restrict__ cny = cnx + a.contact_np;
    const T* __restrict__ cnz = cny + a.contact_np;
    const T wc = T(a.contact_w);
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      if (v < N && k1 > k0) {
        const Q q = qs[v];
        T best = T(0);
        int kb = k0;
        for (int k = k0; k < k1; ++k) {
          const T dx = q.x - cpx[k], dy = q.y - cpy[k], dz = q.z - cpz[k];
          const T d2 = dx * dx + dy * dy + dz * dz;
          if (k == k0 || d2 < best) {
            best = d2;
            kb = k;
          }
        }
        const T nx = cnx[kb], ny = cny[kb], nz = cnz[kb];
        const T sd = (q.x - cpx[kb]) * nx + (q.y - cpy[kb]) * ny + (q.z - cpz[kb]) * nz;
        if (sd < T(0)) {
          const T f = -wc * sd;
          acc[j][0] += f * nx;
          acc[j][1] += f * ny;
          acc[j][2] += f * nz;
          if (want_energy) e_acc += 0.5 * (double)wc * (double)sd * (double)sd;
        }
      }
    }
  }

  // inertia term of the own vertices, cterm - (m/h^2) delta, loaded here so
  // that the loads are in flight during the hinge phase (barriers wait for
  // LDS only)
  const T mh2 = T(a.mdelta);
  T ct[VPT][3];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    int v = min(tid + j * BLOCK, N - 1);  // (rows past N are not stored)
    // an opaque copy of the index: the addresses are formed here again
    // instead of the staging's 64-bit addresses staying live through the
    // triangle phase (at the four-wave register budget they were spilled)
    asm volatile("" : "+v"(v));
#pragma unroll
    for (int d = 0; d < 3; ++d) ct[j][d] = ccol[d * Npad + v] - mh2 * dcol[d * Npad + v];
  }

  // ---- hinges: bending ----
  for (int base = 0; base < E; base += L.hch) {
    const int ne = min(L.hch, E - base);
    V4<T>* ys = reinterpret_cast<V4<T>*>(work);
    const V4<T>* __restrict__ hrec = reinterpret_cast<const V4<T>*>(cv.hin_rec);
    const int e0 = base + min(tid, ne - 1);
    int4 idn = cv.hin_v[e0];
    V4<T> r0n = hrec[2 * e0], r1n = hrec[2 * e0 + 1];
    for (int e = base + tid; e < base + ne; e += BLOCK) {
      const int4 id = idn;
      const V4<T> r0 = r0n, r1 = r1n;
      if (e + BLOCK < base + ne) {
        idn = cv.hin_v[e + BLOCK];
        r0n = hrec[2 * (e + BLOCK)];
        r1n = hrec[2 * (e + BLOCK) + 1];
      }
      const T k0 = r0.x, k1 = r0.y, k2 = r0.z, k3 = r0.w, ce = r1.x, rr = r1.y;
      const Q qi = qs[id.x], qj = qs[id.y], qk = qs[id.z], ql = qs[id.w];
      // y from the differences to q_i (the stencil weights sum to zero), as F
      (void)k0;
      T yq[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T qi_d = comp(qi, d);
        yq[d] = k1 * (comp(qj, d) - qi_d) + k2 * (comp(qk, d) - qi_d) + k3 * (comp(ql, d) - qi_d);
      }
      const T n2 = yq[0] * yq[0] + yq[1] * yq[1] + yq[2] * yq[2];
      const T sc = n2 > T(0) ? rr * f_rsq(n2) : T(1);
      const T wc = wb * ce;
      // w_b c_e (Pb - y(q)), Pb = sc y(q)
      const T ws1 = wc * (sc - T(1));
      V4<T> y;
      y.x = ws1 * yq[0];
      y.y = ws1 * yq[1];
      y.z = ws1 * yq[2];
      y.w = T(0);
      ys[e - base] = y;
      if (want_energy) {
        double eb = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double u = (double)yq[d] - (double)(sc * yq[d]);
          eb += u * u;
        }
        e_acc += 0.5 * (double)wc * eb;
      }
    }
    __syncthreads();
    const bool whole = (ne == E);
    auto hin_add = [&](int j, int hh, T kk) {
      const V4<T> y = ys[hh];
      acc[j][0] += kk * y.x;
      acc[j][1] += kk * y.y;
      acc[j][2] += kk * y.z;
    };
    if constexpr (KH > 0) {
      if (whole) {
        int hh[2][KH];
        T kk[2][KH];
        auto fetch = [&](int j, int set) {
          const int v = min(tid + j * BLOCK, N - 1);
          const int* __restrict__ hp = cv.vh_hin + v * KH;
          const T* __restrict__ kp = cv.vh_k + v * KH;
#pragma unroll
          for (int u = 0; u < KH; ++u) {
            hh[set][u] = hp[u];
            kk[set][u] = kp[u];
          }
        };
        fetch(0, 0);
#pragma unroll
        for (int j = 0; j < VPT; ++j) {
          if (j + 1 < VPT) fetch(j + 1, (j + 1) & 1);
          __builtin_amdgcn_sched_barrier(0);
          if (tid + j * BLOCK < N) {
#pragma unroll
            for (int u = 0; u < KH; ++u) hin_add(j, hh[j & 1][u], kk[j & 1][u]);
          }
        }
      }
    }
    if (KH == 0 || !whole) {
#pragma unroll
      for (int j = 0; j < VPT; ++j) {
        const int v = tid + j * BLOCK;
        if (v < N) {
          const int* __restrict__ hix = cv.vh_hin + v * DH;
          const T* __restrict__ kix = cv.vh_k + v * DH;
          if (whole) {
#pragma unroll 4
            for (int k = 0; k < DH; ++k) hin_add(j, hix[k], kix[k]);
          } else {
            for (int k = 0; k < DH; ++k) {
              const int hh = hix[k] - base;
              if (hh < 0 || hh >= ne) continue;
              hin_add(j, hh, kix[k]);
            }
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- r = inertia - (m/h^2) delta + elastic contributions; zero padding rows ----
  float cmax[3] = {0.f, 0.f, 0.f};
  const double hm = a.h * a.h / a.m;
  const bool want_max = a.colmax != nullptr;
#pragma unroll
  for (int j = 0; j <= VPT; ++j) {
    const int v = tid + j * BLOCK;
    if (v < Npad) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        T r = T(0);
        if (v < N) {
          const int jj = j < VPT ? j : VPT - 1;
          r = ct[jj][d] + acc[jj][d];
          if (want_energy) {
            // (m/2h^2) |q - s|^2 with q - s = delta - (h^2/m) cterm
            const double dd = (double)dcol[d * Npad + v] - hm * (double)ccol[d * Npad + v];
            e_acc += 0.5 * (a.m / (a.h * a.h)) * dd * dd;
          }
        }
        if (want_max) cmax[d] = fmaxf(cmax[d], fabsf((float)r));
        rcol[d * Npad + v] = r;
      }
    }
  }
  if (a.colmax) {
    // (red was last read in the volume projection, many barriers ago)
    block_max_n<3>(cmax, reinterpret_cast<float*>(red));
    if (tid < 3) a.colmax[a.cs.col0 + 3LL * lc + tid] = tid == 0 ? cmax[0] : tid == 1 ? cmax[1] : cmax[2];
  }
  if (want_energy) {
    double ev[1] = {e_acc};
    block_sum<1>(ev, red);
    if (tid == 0) {
      a.energy[cell] = ev[0];
      if (!isfinite(ev[0])) bad = 1;
    }
  }
  if (__syncthreads_or(bad) && tid == 0) atomicOr(a.status, ST_NONFINITE);
}

// LDS: reductions, q as vertex records (plus a zero record; 12 or 32 bytes,
// the region rounded up to 16 bytes), and a work region that holds the
// volume iterate p (N records plus a zero record) or one chunk of triangle
// (6 values) or hinge (4 values) contributions.
template <typename T>
size_t local_smem_bytes_chunks(const ClassView<T>& cv, int block, int* tch, int* hch) {
  const size_t fixed = 8 * sizeof(double) * (block / kWave) + sizeof(double) * local_q_doubles<T>(cv.N);
  const size_t max_total = 160 * 1024;
  // the volume iterate's N + 1 records, in elements of T
  const size_t work_min = sizeof(typename LocalRec<T>::type) / sizeof(T) * ((size_t)cv.N + 1);
  const size_t want = std::max<size_t>(6 * (size_t)cv.F, 4 * (size_t)cv.E);
  const size_t avail = max_total > fixed ? (max_total - fixed) / sizeof(T) : 0;
  // cap the chunk budget so that small meshes leave room for several
  // workgroups per CU
  size_t budget = std::min(want, std::max(work_min, std::min(avail, (size_t)16384)));
  if (budget < work_min) budget = work_min;
  const int t = (int)std::min<size_t>(cv.F, budget / 6);
  const int h = (int)std::min<size_t>(cv.E, budget / 4);
  if (tch) *tch = std::max(t, 1);
  if (hch) *hch = std::max(h, 1);
  return fixed + sizeof(T) * budget;
}

template <typename T>
size_t local_smem_bytes(const ClassView<T>& cv, int block) {
  return local_smem_bytes_chunks(cv, block, nullptr, nullptr);
}

template <typename T>
using LocalFn = void (*)(LocalLaunch<T>);

// Incidence widths with a compile-time instance: 6 triangles and 12 hinges
// per vertex (every vertex of valence <= 6, e.g. subdivided icosahedra).
constexpr int kFixedDT = 6, kFixedDH = 12;

template <typename T, int BLOCK, int VPT>
static LocalFn<T> pick_widths(int DT, int DH, bool ring) {
  if (DT == kFixedDT && DH == kFixedDH && ring)
    return local_kernel<T, BLOCK, VPT, kFixedDT, kFixedDH>;
  return local_kernel<T, BLOCK, VPT, 0, 0>;
}

template <typename T, int BLOCK>
static LocalFn<T> pick_vpt(int N, int DT, int DH, bool ring) {
  const int vpt = (N + BLOCK - 1) / BLOCK;
  if (vpt <= 1) return pick_widths<T, BLOCK, 1>(DT, DH, ring);
  if (vpt <= 2) return pick_widths<T, BLOCK, 2>(DT, DH, ring);
  if (vpt <= 3) return pick_widths<T, BLOCK, 3>(DT, DH, ring);
  if (vpt <= 4) return pick_widths<T, BLOCK, 4>(DT, DH, ring);
  if (vpt <= 6) return pick_widths<T, BLOCK, 6>(DT, DH, ring);
  if (vpt <= 8) return local_kernel<T, BLOCK, 8, 0, 0>;
  if (vpt <= kLocalMaxVertsPerThread) return local_kernel<T, BLOCK, kLocalMaxVertsPerThread, 0, 0>;
  return nullptr;
}

// 1024 threads (FP32, up to three vertices per thread): a large mesh whose
// LDS allows one workgroup per CU gets four waves per SIMD instead of two.
template <typename T>
static LocalFn<T> pick_1024(int N, int DT, int DH, bool ring) {
  if constexpr (sizeof(T) == 4) {
    const int vpt = (N + 1023) / 1024;
    if (vpt <= 2) return pick_widths<T, 1024, 2>(DT, DH, ring);
    if (vpt <= 3) return pick_widths<T, 1024, 3>(DT, DH, ring);
  }
  return nullptr;
}

template <typename T>
static LocalFn<T> pick_local(const ClassView<T>& cv, int block) {
  switch (block) {
    case 128: return pick_vpt<T, 128>(cv.N, cv.DT, cv.DH, cv.vt_ring != nullptr);
    case 256: return pick_vpt<T, 256>(cv.N, cv.DT, cv.DH, cv.vt_ring != nullptr);
    case 512: return pick_vpt<T, 512>(cv.N, cv.DT, cv.DH, cv.vt_ring != nullptr);
    case 1024: return pick_1024<T>(cv.N, cv.DT, cv.DH, cv.vt_ring != nullptr);
    default: return nullptr;
  }
}

// Raises the dynamic-LDS limit of the kernel instance a class will use (not
// a stream operation: call before graph capture).
template <typename T>
hipError_t local_prepare(const ClassView<T>& cv, int block) {
  LocalFn<T> fn = pick_local<T>(cv, block);
  if (!fn) return hipErrorInvalidValue;
  const size_t smem = local_smem_bytes_chunks(cv, block, nullptr, nullptr);
  if (smem > 160 * 1024) return hipErrorInvalidValue;
  if (smem > 64 * 1024)
    return hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)smem);
  return hipSuccess;
}

template <typename T>
hipError_t launch_local(const LocalArgs<T>& a, int block, hipStream_t st) {
  if (a.cs.n_cells == 0) return hipSuccess;
  LocalFn<T> fn = pick_local<T>(a.cs.cv, block);
  if (!fn) return hipErrorInvalidValue;
  LocalLaunch<T> L;
  L.a = a;
  const size_t smem = local_smem_bytes_chunks(a.cs.cv, block, &L.tch, &L.hch);
  if (smem > 160 * 1024) return hipErrorInvalidValue;
  void* args[] = {&L};
  return hipLaunchKernel((const void*)fn, dim3(a.cs.n_cells), dim3(block), args, smem, st);
}

template hipError_t launch_local<float>(const LocalArgs<float>&, int, hipStream_t);
template hipError_t launch_local<double>(const LocalArgs<double>&, int, hipStream_t);
template hipError_t local_prepare<float>(const ClassView<float>&, int);
template hipError_t local_prepare<double>(const ClassView<double>&, int);
template size_t local_smem_bytes<float>(const ClassView<float>&, int);
template size_t local_smem_bytes<double>(const ClassView<double>&, int);

}  // namespace npfem
