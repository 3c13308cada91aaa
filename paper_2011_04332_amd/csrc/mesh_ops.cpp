// Host-side FP64 rest operators of a mesh class.
//
// Per triangle t = (a, b, c): e1 = X_b - X_a, e2 = X_c - X_a, area |e1 x e2|/2,
// an orthonormal in-plane frame (u along e1, w = n_hat x u), D = [[u.e1, u.e2],
// [w.e1, w.e2]] and G_t = [[-1,-1],[1,0],[0,1]] D^-1, so that the deformation
// gradient of a configuration q is F_t(q) = sum_r q_{t_r} (x) G_t[r, :] and the
// rest configuration maps to orthonormal columns (mass-lumped linear membrane
// element).
// Per hinge (edge i-j shared by (i, j, k), where the edge runs i -> j, and
// (j, i, l)): cotangent stencil K = [c03 + c04, c01 + c02, -(c01 + c03),
// -(c02 + c04)] with c01 = cot angle_i(ijk), c02 = cot angle_i(ijl),
// c03 = cot angle_j(ijk), c04 = cot angle_j(ijl); weight 3 / (A_ijk + A_ijl);
// rest magnitude |sum_r K_r X_r|.
#include "mesh_ops.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <unordered_map>

#include "npfem.h"

namespace npfem {

namespace {

inline void sub3(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}
inline void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline double norm3(const double* a) { return std::sqrt(dot3(a, a)); }

// cot of the angle at p between p->a and p->b
double cot_at(const double* p, const double* a, const double* b) {
  double u[3], v[3], c[3];
  sub3(a, p, u);
  sub3(b, p, v);
  cross3(u, v, c);
  return dot3(u, v) / norm3(c);
}

inline uint64_t ekey(int u, int v) { return ((uint64_t)(uint32_t)u << 32) | (uint32_t)v; }

double power_norm(const MeshOps& m, const std::vector<double>& val) {
  std::vector<double> x(m.N), y(m.N);
  for (int i = 0; i < m.N; ++i) x[i] = 1.0 + 0.37 * std::sin(1.0 + i);  // not in the null space
  double lam = 0.0;
  for (int it = 0; it < 200; ++it) {
    double nx = 0.0;
    for (double v : x) nx += v * v;
    nx = std::sqrt(nx);
    for (double& v : x) v /= nx;
    for (int i = 0; i < m.N; ++i) {
      double s = 0.0;
      for (int e = m.lap_ptr[i]; e < m.lap_ptr[i + 1]; ++e) s += val[e] * x[m.lap_col[e]];
      y[i] = s;
    }
    double ny = 0.0;
    for (double v : y) ny += v * v;
    lam = std::sqrt(ny);
    x.swap(y);
  }
  return lam;
}

}  // namespace

int build_mesh_ops(const double* xyz, int n, const int32_t* tris, int nt, MeshOps& M,
                   std::string& err) {
  char buf[256];
  if (n < 4 || nt < 4) {
    err = "mesh needs at least 4 vertices and 4 triangles";
    return NPFEM_ERR_INVALID_ARG;
  }
  if (n > 65535) {
    err = "mesh has more than 65535 vertices";
    return NPFEM_ERR_INVALID_ARG;
  }
  for (int i = 0; i < 3 * n; ++i) {
    if (!std::isfinite(xyz[i])) {
      err = "non-finite rest coordinate";
      return NPFEM_ERR_INVALID_ARG;
    }
  }
  M = MeshOps();
  M.N = n;
  M.F = nt;
  M.X.assign(xyz, xyz + 3 * (size_t)n);
  M.tris.assign(tris, tris + 3 * (size_t)nt);
  std::unordered_map<uint64_t, int> third;  // directed edge -> opposite vertex
  third.reserve(3 * (size_t)nt * 2);
  std::vector<int> used(n, 0);
  for (int t = 0; t < nt; ++t) {
    const int a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    if (a < 0 || b < 0 || c < 0 || a >= n || b >= n || c >= n) {
      std::snprintf(buf, sizeof buf, "triangle %d has a vertex index out of range", t);
      err = buf;
      return NPFEM_ERR_INVALID_ARG;
    }
    if (a == b || b == c || a == c) {
      std::snprintf(buf, sizeof buf, "triangle %d repeats a vertex", t);
      err = buf;
      return NPFEM_ERR_DEGENERATE_TRI;
    }
    used[a] = used[b] = used[c] = 1;
    const int ring[3] = {a, b, c};
    for (int r = 0; r < 3; ++r) {
      const int u = ring[r], v = ring[(r + 1) % 3], w = ring[(r + 2) % 3];
      if (!third.emplace(ekey(u, v), w).second) {
        std::snprintf(buf, sizeof buf, "directed edge %d->%d used twice (non-manifold or flipped)", u, v);
        err = buf;
        return NPFEM_ERR_MESH_NONMANIFOLD;
      }
    }
  }
  for (auto& kv : third) {
    const int u = (int)(kv.first >> 32), v = (int)(kv.first & 0xffffffffu);
    if (!third.count(ekey(v, u))) {
      std::snprintf(buf, sizeof buf, "edge %d-%d has a single triangle (open mesh)", u, v);
      err = buf;
      return NPFEM_ERR_MESH_OPEN;
    }
  }
  for (int i = 0; i < n; ++i) {
    if (!used[i]) {
      std::snprintf(buf, sizeof buf, "vertex %d is not used by any triangle", i);
      err = buf;
      return NPFEM_ERR_INVALID_ARG;
    }
  }
  const int n_edges = (int)(third.size() / 2);
  if (n - n_edges + nt != 2) {
    err = "Euler characteristic V - E + F is not 2 (not a closed genus-0 surface)";
    return NPFEM_ERR_MESH_NONMANIFOLD;
  }

  // triangle operators
  M.G.resize(6 * (size_t)nt);
  M.area.resize(nt);
  double vol6 = 0.0;
  for (int t = 0; t < nt; ++t) {
    const double* A = &xyz[3 * tris[3 * t]];
    const double* B = &xyz[3 * tris[3 * t + 1]];
    const double* C = &xyz[3 * tris[3 * t + 2]];
    double e1[3], e2[3], nn[3], bc[3];
    sub3(B, A, e1);
    sub3(C, A, e2);
    cross3(e1, e2, nn);
    const double nl = norm3(nn);
    if (!(nl > 1e-14 * norm3(e1) * norm3(e2))) {
      std::snprintf(buf, sizeof buf, "rest triangle %d has zero area", t);
      err = buf;
      return NPFEM_ERR_DEGENERATE_TRI;
    }
    M.area[t] = 0.5 * nl;
    const double l1 = norm3(e1);
    double u[3] = {e1[0] / l1, e1[1] / l1, e1[2] / l1};
    double nh[3] = {nn[0] / nl, nn[1] / nl, nn[2] / nl};
    double w[3];
    cross3(nh, u, w);
    const double d00 = dot3(u, e1), d01 = dot3(u, e2), d10 = dot3(w, e1), d11 = dot3(w, e2);
    const double det = d00 * d11 - d01 * d10;
    const double i00 = d11 / det, i01 = -d01 / det, i10 = -d10 / det, i11 = d00 / det;
    double* g = &M.G[6 * (size_t)t];
    // rows of [[-1,-1],[1,0],[0,1]] times D^-1
    g[0] = -i00 - i10;
    g[1] = -i01 - i11;
    g[2] = i00;
    g[3] = i01;
    g[4] = i10;
    g[5] = i11;
    cross3(B, C, bc);
    vol6 += dot3(A, bc);
  }
  M.vol_rest = vol6 / 6.0;
  {
    double cen[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i)
      for (int d = 0; d < 3; ++d) cen[d] += xyz[3 * i + d] / n;
    for (int i = 0; i < n; ++i) {
      double r[3];
      sub3(&xyz[3 * i], cen, r);
      M.radius = std::max(M.radius, norm3(r));
    }
  }
  if (!(M.vol_rest > 0.0)) {
    err = "enclosed volume is not positive (triangles must be counter-clockwise seen from outside)";
    return NPFEM_ERR_INVALID_ARG;
  }

  // hinges, one per undirected edge (i < j), sorted by (i, j)
  std::vector<std::pair<uint64_t, int>> dir;
  dir.reserve(third.size());
  for (auto& kv : third) {
    const int u = (int)(kv.first >> 32), v = (int)(kv.first & 0xffffffffu);
    if (u < v) dir.push_back(kv);
  }
  std::sort(dir.begin(), dir.end());
  M.E = (int)dir.size();
  M.hin.resize(4 * (size_t)M.E);
  M.K.resize(4 * (size_t)M.E);
  M.cw.resize(M.E);
  M.rr.resize(M.E);
  for (int e = 0; e < M.E; ++e) {
    const int i = (int)(dir[e].first >> 32), j = (int)(dir[e].first & 0xffffffffu);
    const int k = dir[e].second, l = third[ekey(j, i)];
    int* hv = &M.hin[4 * (size_t)e];
    hv[0] = i;
    hv[1] = j;
    hv[2] = k;
    hv[3] = l;
    const double *xi = &xyz[3 * i], *xj = &xyz[3 * j], *xk = &xyz[3 * k], *xl = &xyz[3 * l];
    const double c01 = cot_at(xi, xj, xk), c02 = cot_at(xi, xj, xl);
    const double c03 = cot_at(xj, xi, xk), c04 = cot_at(xj, xi, xl);
    double* K = &M.K[4 * (size_t)e];
    K[0] = c03 + c04;
    K[1] = c01 + c02;
    K[2] = -(c01 + c03);
    K[3] = -(c02 + c04);
    double ji[3], ki[3], li[3], c1[3], c2[3];
    sub3(xj, xi, ji);
    sub3(xk, xi, ki);
    sub3(xl, xi, li);
    cross3(ji, ki, c1);
    cross3(ji, li, c2);
    M.cw[e] = 3.0 / (0.5 * norm3(c1) + 0.5 * norm3(c2));
    double y[3] = {0, 0, 0};
    const double* xs[4] = {xi, xj, xk, xl};
    for (int r = 0; r < 4; ++r)
      for (int d = 0; d < 3; ++d) y[d] += K[r] * xs[r][d];
    M.rr[e] = norm3(y);
  }

  // vertex -> triangle incidence (ascending triangle index)
  M.vt_ptr.assign(n + 1, 0);
  for (int t = 0; t < nt; ++t)
    for (int r = 0; r < 3; ++r) M.vt_ptr[tris[3 * t + r] + 1]++;
  for (int i = 0; i < n; ++i) M.vt_ptr[i + 1] += M.vt_ptr[i];
  const int nvt = M.vt_ptr[n];
  M.vt_tri.resize(nvt);
  M.vt_fan.resize(nvt);
  M.vt_g.resize(2 * (size_t)nvt);
  {
    std::vector<int> fill(M.vt_ptr.begin(), M.vt_ptr.end() - 1);
    for (int t = 0; t < nt; ++t) {
      for (int r = 0; r < 3; ++r) {
        const int v = tris[3 * t + r];
        const int b = tris[3 * t + (r + 1) % 3], c = tris[3 * t + (r + 2) % 3];
        const int p = fill[v]++;
        M.vt_tri[p] = t;
        M.vt_fan[p] = b | (c << 16);
        M.vt_g[2 * (size_t)p] = M.G[6 * (size_t)t + 2 * r];
        M.vt_g[2 * (size_t)p + 1] = M.G[6 * (size_t)t + 2 * r + 1];
      }
    }
  }
  // vertex -> hinge incidence (ascending hinge index)
  M.vh_ptr.assign(n + 1, 0);
  for (int e = 0; e < M.E; ++e)
    for (int r = 0; r < 4; ++r) M.vh_ptr[M.hin[4 * (size_t)e + r] + 1]++;
  for (int i = 0; i < n; ++i) M.vh_ptr[i + 1] += M.vh_ptr[i];
  const int nvh = M.vh_ptr[n];
  M.vh_hin.resize(nvh);
  M.vh_k.resize(nvh);
  {
    std::vector<int> fill(M.vh_ptr.begin(), M.vh_ptr.end() - 1);
    for (int e = 0; e < M.E; ++e) {
      for (int r = 0; r < 4; ++r) {
        const int v = M.hin[4 * (size_t)e + r];
        const int p = fill[v]++;
        M.vh_hin[p] = e;
        M.vh_k[p] = M.K[4 * (size_t)e + r];
      }
    }
  }
  // Laplacians: rows as sorted maps col -> (lt, lb)
  {
    std::vector<std::vector<std::pair<int, std::pair<double, double>>>> rows(n);
    auto add = [&](int i, int j, double lt, double lb) {
      auto& R = rows[i];
      for (auto& p : R) {
        if (p.first == j) {
          p.second.first += lt;
          p.second.second += lb;
          return;
        }
      }
      R.push_back({j, {lt, lb}});
    };
    for (int t = 0; t < nt; ++t) {
      const double* g = &M.G[6 * (size_t)t];
      for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s)
          add(tris[3 * t + r], tris[3 * t + s],
              M.area[t] * (g[2 * r] * g[2 * s] + g[2 * r + 1] * g[2 * s + 1]), 0.0);
    }
    for (int e = 0; e < M.E; ++e) {
      const double* K = &M.K[4 * (size_t)e];
      for (int r = 0; r < 4; ++r)
        for (int s = 0; s < 4; ++s)
          add(M.hin[4 * (size_t)e + r], M.hin[4 * (size_t)e + s], 0.0, M.cw[e] * K[r] * K[s]);
    }
    M.lap_ptr.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
      std::sort(rows[i].begin(), rows[i].end(),
                [](const auto& a, const auto& b) { return a.first < b.first; });
      M.lap_ptr[i + 1] = M.lap_ptr[i] + (int)rows[i].size();
    }
    M.lap_col.resize(M.lap_ptr[n]);
    M.lap_t.resize(M.lap_ptr[n]);
    M.lap_b.resize(M.lap_ptr[n]);
    for (int i = 0; i < n; ++i) {
      int p = M.lap_ptr[i];
      for (auto& q : rows[i]) {
        M.lap_col[p] = q.first;
        M.lap_t[p] = q.second.first;
        M.lap_b[p] = q.second.second;
        ++p;
      }
    }
  }
  M.norm_t = power_norm(M, M.lap_t);
  M.norm_b = power_norm(M, M.lap_b);
  return NPFEM_OK;
}

void dense_system_matrix(const MeshOps& m, const double w[4], double mass, double dt, double* A,
                         int ld) {
  const double diag = mass / (dt * dt) + w[3];
  const double wt = w[0] + w[1], wb = w[2];
  for (int i = 0; i < m.N; ++i) {
    for (int j = 0; j < m.N; ++j) A[(size_t)i * ld + j] = 0.0;
    A[(size_t)i * ld + i] = diag;
    for (int e = m.lap_ptr[i]; e < m.lap_ptr[i + 1]; ++e)
      A[(size_t)i * ld + m.lap_col[e]] += wt * m.lap_t[e] + wb * m.lap_b[e];
  }
}

}  // namespace npfem
