// Host-side FP64 rest operators of a mesh class (no HIP calls).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace npfem {

struct MeshOps {
  int N = 0, F = 0, E = 0;
  std::vector<double> X;     // [N][3]
  std::vector<int> tris;     // [F][3]
  std::vector<double> G;     // [F][3][2]
  std::vector<double> area;  // [F]
  std::vector<int> hin;      // [E][4] (i, j, k, l)
  std::vector<double> K;     // [E][4]
  std::vector<double> cw;    // [E] 3 / (A1 + A2)
  std::vector<double> rr;    // [E] rest |y|
  double vol_rest = 0.0;
  double radius = 0.0;       // max distance of a rest vertex from the rest centroid
  // vertex incidence (CSR, entries in ascending element order)
  std::vector<int> vt_ptr, vt_tri, vt_fan;
  std::vector<double> vt_g;  // [entries][2]
  std::vector<int> vh_ptr, vh_hin;
  std::vector<double> vh_k;
  // Laplacian pattern (diagonal included) and the two operators
  std::vector<int> lap_ptr, lap_col;
  std::vector<double> lap_t, lap_b;
  double norm_t = 0.0, norm_b = 0.0;  // spectral norms (power iteration)
};

// Validates a closed, consistently oriented 2-manifold and builds all
// operators. Returns 0 or an NPFEM_ERR_* code with a message in err.
int build_mesh_ops(const double* xyz, int n_verts, const int32_t* tris, int n_tris, MeshOps& out,
                   std::string& err);

// Dense system matrix (m/h^2 + w_v) I + (w_s + w_a) L_tri + w_b L_bend into
// A[i * ld + j] (entries outside n x n untouched).
void dense_system_matrix(const MeshOps& m, const double w[4], double mass, double dt, double* A,
                         int ld);

}  // namespace npfem
