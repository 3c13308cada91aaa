// Local step of projective dynamics plus the right-hand-side gather, one
// workgroup per cell.
//
// For the current iterate q = x + delta (delta form: the global step solves
// A delta = b - A x), the kernel computes per cell
//   r = (m/h)v + f                                     (inertia, precomputed)
//     + sum_t A_t G_t (w_s (Ps_t - F_t(x)) + w_a (Pa_t - F_t(x)))^T
//     + sum_e w_b c_e K_e (x) (Pb_e - y_e(x))
//     + w_v (Pv - x)
// where Ps/Pa are the strain/area projections of F_t(q), Pb the bending
// projection of y_e(q) = sum_r K_e[r] q_r and Pv the closest point of q on the
// rest-volume surface. Element contributions are staged in LDS and gathered
// per vertex through CSR incidence lists in a fixed order (no atomics), so
// results are bitwise reproducible. Triangles and hinges are processed in
// chunks sized to the LDS budget; chunking does not change the summation
// order.
#include <algorithm>

#include "device_utils.h"
#include "npfem_internal.h"

namespace npfem {

template <typename T>
struct LocalLaunch {
  LocalArgs<T> a;
  int tch;   // triangles per LDS chunk
  int hch;   // hinges per LDS chunk
};

template <typename T>
__device__ __forceinline__ T rsqrt_t(T x) {
  return T(1) / sqrt(x);
}

// Strain (polar factor) and area projections of a 3x2 deformation gradient.
// S = F^T F = [[a, b], [b, c]], sigma1^2 sigma2^2 = |f0 x f1|^2.
//   polar:  F S^{-1/2},  S^{-1/2} = [[c + s, -b], [-b, a + s]] / (s (sigma1 + sigma2)),
//           s = sigma1 sigma2 (closed-form square root of a 2x2 SPD matrix);
//   area:   F V diag(t/sigma1, (1/t)/sigma2) V^T with t the positive root of
//           t^4 - sigma1 t^3 + sigma2 t - 1 (Newton from sqrt(sigma1/sigma2))
//           and V the eigenvectors of S (half-angle formulas).
template <typename T, int NEWTON>
__device__ __forceinline__ void project_triangle(const T (&f)[3][2], T (&ps)[3][2], T (&pa)[3][2],
                                                 int& bad) {
  const T a = f[0][0] * f[0][0] + f[1][0] * f[1][0] + f[2][0] * f[2][0];
  const T b = f[0][0] * f[0][1] + f[1][0] * f[1][1] + f[2][0] * f[2][1];
  const T c = f[0][1] * f[0][1] + f[1][1] * f[1][1] + f[2][1] * f[2][1];
  const T nx = f[1][0] * f[2][1] - f[2][0] * f[1][1];
  const T ny = f[2][0] * f[0][1] - f[0][0] * f[2][1];
  const T nz = f[0][0] * f[1][1] - f[1][0] * f[0][1];
  const T det = nx * nx + ny * ny + nz * nz;
  const T hd = (a - c) * T(0.5);
  const T rr = sqrt(hd * hd + b * b);
  const T l1 = (a + c) * T(0.5) + rr;
  const T s1 = sqrt(l1);
  const T s12 = sqrt(det);
  const T s2 = s12 / s1;
  if (!(s2 > T(1e-12) * s1) || !isfinite(l1)) bad = 1;
  // polar factor
  const T inv = T(1) / (s12 * (s1 + s2));
  const T m00 = (c + s12) * inv, m01 = -b * inv, m11 = (a + s12) * inv;
  // area root
  T t = sqrt(s1 / s2);
#pragma unroll
  for (int it = 0; it < NEWTON; ++it) {
    const T t2 = t * t;
    const T p = t2 * t * (t - s1) + s2 * t - T(1);
    const T dp = t2 * (T(4) * t - T(3) * s1) + s2;
    t -= p / dp;
  }
  if (!(t > T(0)) || !isfinite(t)) bad = 1;
  const T al1 = t / s1;
  const T al2 = T(1) / (t * s2);
  T cs = T(1), sn = T(0);
  if (rr > T(0)) {
    const T c2 = hd / rr, s2a = b / rr;
    if (c2 >= T(0)) {
      cs = sqrt((T(1) + c2) * T(0.5));
      sn = s2a / (T(2) * cs);
    } else {
      sn = copysign(sqrt((T(1) - c2) * T(0.5)), s2a);
      cs = s2a / (T(2) * sn);
    }
  }
  const T da = al1 - al2;
  const T n00 = al2 + da * cs * cs, n01 = da * cs * sn, n11 = al2 + da * sn * sn;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    ps[d][0] = f[d][0] * m00 + f[d][1] * m01;
    ps[d][1] = f[d][0] * m01 + f[d][1] * m11;
    pa[d][0] = f[d][0] * n00 + f[d][1] * n01;
    pa[d][1] = f[d][0] * n01 + f[d][1] * n11;
  }
}

template <typename T, int BLOCK, int VPT>
__global__ void __launch_bounds__(BLOCK) local_kernel(LocalLaunch<T> L) {
  extern __shared__ double smem_local[];
  constexpr int NW = BLOCK / kWave;
  constexpr int NEWTON = sizeof(T) == 8 ? 5 : 4;
  const LocalArgs<T>& a = L.a;
  const ClassView<T>& cv = a.cs.cv;
  const int N = cv.N, Npad = cv.Npad, F = cv.F, E = cv.E;
  const int tid = threadIdx.x;
  const int lc = blockIdx.x;
  const int cell = a.cs.cell0 + lc;
  const long long vb = a.cs.vert0 + (long long)lc * N;
  const long long cb = a.cs.elem0 + 3LL * lc * Npad;
  const long long sumN = a.sumN;

  double* red = smem_local;  // 8 * NW doubles
  T* qs = reinterpret_cast<T*>(smem_local + 8 * NW);
  T* xs = qs + 3 * N;
  T* work = xs + 3 * N;

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

  // ---- stage x and q = x + delta in LDS ----
  for (int v = tid; v < N; v += BLOCK) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const T x = a.pos[d * sumN + vb + v];
      xs[d * N + v] = x;
      qs[d * N + v] = x + a.delta[cb + d * Npad + v];
    }
  }
  __syncthreads();

  T acc[VPT][3];
#pragma unroll
  for (int j = 0; j < VPT; ++j) acc[j][0] = acc[j][1] = acc[j][2] = T(0);

  // ---- volume: closest point of q on {V(p) = V_rest} ----
  // p <- q + lam grad V(p), lam = (V_rest - V(p) - grad V(p).(q - p)) / |grad V(p)|^2,
  // V(p) = (1/3) sum_v p_v . grad_v V(p) (Euler, V is cubic); sums in FP64.
  {
    T* ps = work;
    for (int v = tid; v < N; v += BLOCK) {
      ps[v] = qs[v];
      ps[N + v] = qs[N + v];
      ps[2 * N + v] = qs[2 * N + v];
    }
    __syncthreads();
    T g[VPT][3];
    double lam = 0.0;
    for (int it = 0; it < a.max_vol_iter; ++it) {
      double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int j = 0; j < VPT; ++j) {
        const int v = tid + j * BLOCK;
        g[j][0] = g[j][1] = g[j][2] = T(0);
        if (v < N) {
          T gx = T(0), gy = T(0), gz = T(0);
          const int e1 = cv.vt_ptr[v + 1];
          for (int e = cv.vt_ptr[v]; e < e1; ++e) {
            const int bc = cv.vt_fan[e];
            const int vb2 = bc & 0xffff, vc = bc >> 16;
            const T bx = ps[vb2], by = ps[N + vb2], bz = ps[2 * N + vb2];
            const T cx = ps[vc], cy = ps[N + vc], cz = ps[2 * N + vc];
            gx += by * cz - bz * cy;
            gy += bz * cx - bx * cz;
            gz += bx * cy - by * cx;
          }
          gx *= T(1.0 / 6.0);
          gy *= T(1.0 / 6.0);
          gz *= T(1.0 / 6.0);
          g[j][0] = gx;
          g[j][1] = gy;
          g[j][2] = gz;
          const T px = ps[v], py = ps[N + v], pz = ps[2 * N + v];
          s[0] += (double)px * gx + (double)py * gy + (double)pz * gz;
          s[1] += (double)gx * gx + (double)gy * gy + (double)gz * gz;
          s[2] += (double)gx * (double)(qs[v] - px) + (double)gy * (double)(qs[N + v] - py) +
                  (double)gz * (double)(qs[2 * N + v] - pz);
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
          ps[v] = qs[v] + lt * g[j][0];
          ps[N + v] = qs[N + v] + lt * g[j][1];
          ps[2 * N + v] = qs[2 * N + v] + lt * g[j][2];
        }
      }
      __syncthreads();
      const bool conv = fabs(lam_new - lam) <= a.vol_tol * fabs(lam_new);
      lam = lam_new;
      if (conv) break;
    }
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      if (v < N) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const T p = ps[d * N + v];
          acc[j][d] += wv * (p - xs[d * N + v]);
          if (want_energy) {
            const double dq = (double)qs[d * N + v] - (double)p;
            e_acc += 0.5 * (double)wv * dq * dq;
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- triangles: strain + area ----
  for (int base = 0; base < F; base += L.tch) {
    const int nt = min(L.tch, F - base);
    for (int t = base + tid; t < base + nt; t += BLOCK) {
      const int4 id = cv.tri_v[t];
      const T* rec = cv.tri_rec + 8 * t;
      const T g00 = rec[0], g01 = rec[1], g10 = rec[2], g11 = rec[3], g20 = rec[4], g21 = rec[5];
      const T area = rec[6];
      T fq[3][2], fx[3][2];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T qa = qs[d * N + id.x], qb = qs[d * N + id.y], qc = qs[d * N + id.z];
        const T xa = xs[d * N + id.x], xb = xs[d * N + id.y], xc = xs[d * N + id.z];
        fq[d][0] = qa * g00 + qb * g10 + qc * g20;
        fq[d][1] = qa * g01 + qb * g11 + qc * g21;
        fx[d][0] = xa * g00 + xb * g10 + xc * g20;
        fx[d][1] = xa * g01 + xb * g11 + xc * g21;
      }
      T ps[3][2], pa[3][2];
      project_triangle<T, NEWTON>(fq, ps, pa, bad);
      T* w = work + 6 * (t - base);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          w[2 * d + k] = area * (ws * (ps[d][k] - fx[d][k]) + wa * (pa[d][k] - fx[d][k]));
        }
      }
      if (want_energy) {
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
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      if (v < N) {
        const int e1 = cv.vt_ptr[v + 1];
        for (int e = cv.vt_ptr[v]; e < e1; ++e) {
          const int t = cv.vt_tri[e] - base;
          if (t < 0 || t >= nt) continue;
          const T ga = cv.vt_g[2 * e], gb = cv.vt_g[2 * e + 1];
          const T* w = work + 6 * t;
          acc[j][0] += ga * w[0] + gb * w[1];
          acc[j][1] += ga * w[2] + gb * w[3];
          acc[j][2] += ga * w[4] + gb * w[5];
        }
      }
    }
    __syncthreads();
  }

  // ---- hinges: bending ----
  for (int base = 0; base < E; base += L.hch) {
    const int ne = min(L.hch, E - base);
    for (int e = base + tid; e < base + ne; e += BLOCK) {
      const int4 id = cv.hin_v[e];
      const T* rec = cv.hin_rec + 8 * e;
      const T k0 = rec[0], k1 = rec[1], k2 = rec[2], k3 = rec[3], ce = rec[4], rr = rec[5];
      T yq[3], yx[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        yq[d] = k0 * qs[d * N + id.x] + k1 * qs[d * N + id.y] + k2 * qs[d * N + id.z] +
                k3 * qs[d * N + id.w];
        yx[d] = k0 * xs[d * N + id.x] + k1 * xs[d * N + id.y] + k2 * xs[d * N + id.z] +
                k3 * xs[d * N + id.w];
      }
      const T n2 = yq[0] * yq[0] + yq[1] * yq[1] + yq[2] * yq[2];
      const T sc = n2 > T(0) ? rr / sqrt(n2) : T(1);
      const T wc = wb * ce;
      T* w = work + 3 * (e - base);
      double eb = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T pb = sc * yq[d];
        w[d] = wc * (pb - yx[d]);
        const double u = (double)yq[d] - (double)pb;
        eb += u * u;
      }
      if (want_energy) e_acc += 0.5 * (double)wc * eb;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = tid + j * BLOCK;
      if (v < N) {
        const int e1 = cv.vh_ptr[v + 1];
        for (int e = cv.vh_ptr[v]; e < e1; ++e) {
          const int hh = cv.vh_hin[e] - base;
          if (hh < 0 || hh >= ne) continue;
          const T kk = cv.vh_k[e];
          const T* w = work + 3 * hh;
          acc[j][0] += kk * w[0];
          acc[j][1] += kk * w[1];
          acc[j][2] += kk * w[2];
        }
      }
    }
    __syncthreads();
  }

  // ---- r = inertia + elastic contributions; zero padding rows ----
  float cmax[3] = {0.f, 0.f, 0.f};
  const double hm = a.h * a.h / a.m;
#pragma unroll
  for (int j = 0; j <= VPT; ++j) {
    const int v = tid + j * BLOCK;
    if (v < Npad) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        T r = T(0);
        if (v < N) {
          const T ct = a.cterm[cb + d * Npad + v];
          r = ct + acc[j < VPT ? j : VPT - 1][d];
          if (want_energy) {
            // (m/2h^2) |q - s|^2 with q - s = delta - (h^2/m) cterm
            const double dd = (double)a.delta[cb + d * Npad + v] - hm * (double)ct;
            e_acc += 0.5 * (a.m / (a.h * a.h)) * dd * dd;
          }
        }
        cmax[d] = fmaxf(cmax[d], fabsf((float)r));
        a.rhs[cb + d * Npad + v] = r;
      }
    }
  }
  if (a.colmax) {
    float* redf = reinterpret_cast<float*>(red);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float mx = block_max(cmax[d], redf);
      if (tid == 0) a.colmax[a.cs.col0 + 3LL * lc + d] = mx;
    }
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

template <typename T>
size_t local_smem_bytes_chunks(const ClassView<T>& cv, int block, int* tch, int* hch) {
  const size_t fixed = 8 * sizeof(double) * (block / kWave) + sizeof(T) * 6 * (size_t)cv.N;
  // element chunk budget: the larger of 3N (volume iterate) and what fits in
  // the remaining LDS, capped by the element counts
  const size_t max_total = 160 * 1024;
  size_t work_elems = 3 * (size_t)cv.N;
  size_t want = std::max<size_t>(6 * (size_t)cv.F, 3 * (size_t)cv.E);
  size_t avail = max_total > fixed ? (max_total - fixed) / sizeof(T) : 0;
  // keep a margin so two workgroups can share a CU when the mesh is small
  size_t budget = std::min(want, std::max(work_elems, std::min(avail, (size_t)16384)));
  if (budget < work_elems) budget = work_elems;
  int t = (int)std::min<size_t>(cv.F, budget / 6);
  int h = (int)std::min<size_t>(cv.E, budget / 3);
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

template <typename T, int BLOCK>
static LocalFn<T> pick_vpt(int N) {
  const int vpt = (N + BLOCK - 1) / BLOCK;
  if (vpt <= 1) return local_kernel<T, BLOCK, 1>;
  if (vpt <= 2) return local_kernel<T, BLOCK, 2>;
  if (vpt <= 3) return local_kernel<T, BLOCK, 3>;
  if (vpt <= 4) return local_kernel<T, BLOCK, 4>;
  if (vpt <= 6) return local_kernel<T, BLOCK, 6>;
  if (vpt <= 8) return local_kernel<T, BLOCK, 8>;
  if (vpt <= 11) return local_kernel<T, BLOCK, 11>;
  return nullptr;
}

template <typename T>
static LocalFn<T> pick_local(int N, int block) {
  switch (block) {
    case 128: return pick_vpt<T, 128>(N);
    case 256: return pick_vpt<T, 256>(N);
    case 512: return pick_vpt<T, 512>(N);
    default: return nullptr;
  }
}

// Raises the dynamic-LDS limit of the kernel instance a class will use (not
// a stream operation: call before graph capture).
template <typename T>
hipError_t local_prepare(const ClassView<T>& cv, int block) {
  LocalFn<T> fn = pick_local<T>(cv.N, block);
  if (!fn) return hipErrorInvalidValue;
  const size_t smem = local_smem_bytes_chunks(cv, block, nullptr, nullptr);
  if (smem > 64 * 1024)
    return hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)smem);
  return hipSuccess;
}

template <typename T>
hipError_t launch_local(const LocalArgs<T>& a, int block, hipStream_t st) {
  if (a.cs.n_cells == 0) return hipSuccess;
  LocalFn<T> fn = pick_local<T>(a.cs.cv.N, block);
  if (!fn) return hipErrorInvalidValue;
  LocalLaunch<T> L;
  L.a = a;
  const size_t smem = local_smem_bytes_chunks(a.cs.cv, block, &L.tch, &L.hch);
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
