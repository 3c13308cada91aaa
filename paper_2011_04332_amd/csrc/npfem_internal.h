// Internal types shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace npfem {

// Device-resident, read-only description of one mesh class. Element records
// are padded to 16/32-byte multiples so that a thread fetches one record with
// vector loads; incidence lists are CSR over vertices.
template <typename T>
struct ClassView {
  int N;      // vertices
  int Npad;   // rows of the padded column layout (multiple of 16)
  int F;      // triangles
  int E;      // hinges
  const int4* tri_v;   // [F] (a, b, c, 0)
  const T* tri_rec;    // [F][8]: G (3x2 row-major), area, 0
  const int4* hin_v;   // [E] (i, j, k, l)
  const T* hin_rec;    // [E][8]: K[4], c, r_rest, 0, 0
  // the same records in FP64 (the adjoint's element arithmetic: near rest
  // the weight gradients move with the rounding of G, area and K)
  const double* tri_rec64;
  const double* hin_rec64;
  // Vertex incidence padded to a fixed width, vertex-major ([N][slot]: a
  // thread reads its vertex's entries as one contiguous run, and a wave's
  // runs are contiguous too); entries of a vertex are in ascending element
  // order, padding entries contribute zero.
  int DT;              // max triangles per vertex
  int DH;              // max hinges per vertex
  const int* vt_tri;   // [N][DT] triangle index (0 in padding)
  const T* vt_g;       // [N][DT][2] G row of the vertex in that triangle (0 in padding)
  const int* vt_fan;   // [N][DT] other two vertices b | c << 16, (v, b, c) counter-clockwise;
                       // padding N | N << 16 (a zero record in the kernel's LDS)
  const int* vt_ring;  // [N][DT] the one-ring n_0 .. n_{d-1} in fan order (the fan
                       // triangles are (v, n_k, n_k+1 mod d)), padded with n_0; nullptr
                       // unless every vertex's fan closes into one cycle
  const int* vh_hin;   // [N][DH] hinge index (0 in padding)
  const T* vh_k;       // [N][DH] stencil coefficient of the vertex (0 in padding)
  // Rows of the two Laplacians on their joint pattern (diagonal included),
  // padded to a fixed width DL, slot-major [DL][N]; padding entries have
  // column N and coefficient 0.
  int DL;
  const int* lap_col;  // [DL][N]
  const T* lap_t;      // [DL][N] sum_t A_t G_t G_t^T entries
  const T* lap_b;      // [DL][N] sum_e c_e K_e K_e^T entries
  double vol_rest;
};

// Per-class slice of the batch.
template <typename T>
struct ClassSlice {
  ClassView<T> cv;
  int n_cells;       // cells of this class
  int cell0;         // global index of its first cell
  long long col0;    // first column (3 per cell) of the class in the column buffers
  long long elem0;   // element offset of that column (classes differ in Npad)
  long long vert0;   // first vertex of its first cell in the SoA state
  T mass;
  T w_nom[4];        // nominal weights
};

// The local step's widest instance: 512 threads with at most 11 vertices
// each, so a class may have at most 5632 vertices.
constexpr int kLocalMaxBlock = 512;
constexpr int kLocalMaxVertsPerThread = 11;

// Kernel launch helpers (defined in the .hip files). All take the stream last.
struct StepScalars {
  double h;       // time step
  double m;       // vertex mass of the class
};

template <typename T>
struct LocalArgs {
  ClassSlice<T> cs;
  const T* pos;        // state SoA [3][sumN]
  long long sumN;
  const T* delta;      // column buffers [cols][Npad] (batch base; class at cs.elem0)
  const T* cterm;      // inertial term (m/h) v + f, same layout
  T* rhs;              // output r = b - A x, same layout
  const T* weights;    // [n_cells_total][4] or nullptr
  double* energy;      // [n_cells_total] slot for this iteration, or nullptr
  float* colmax;       // [cols] max |r| per column (low-precision global step), or nullptr
  int* status;         // device flags
  double h, m;
  double mdelta;       // coefficient of delta in r: m (1 + alpha h)/h^2 (m/h^2 undamped)
  // contact potentials (0 weight: none): points and outward normals SoA
  // [3][n_points] in cell-local coordinates, cell c's at [off[c], off[c + 1])
  double contact_w = 0.0;
  const T* contact_p = nullptr;
  const T* contact_n = nullptr;
  const int* contact_off = nullptr;
  long long contact_np = 0;
  const int* skip = nullptr;  // per cell: nonzero = leave the cell alone (quasi-Newton rounds)
  int max_vol_iter;
  double vol_tol;      // relative settling test of the volume multiplier
  double vol_abs;      // absolute test: |d lam| |grad V|_2 below this (length units)
};

// Reverse of one PD iteration (kernels_adjoint.hip).
template <typename T>
struct AdjArgs {
  ClassSlice<T> cs;
  const T* xn;         // positions x_n of the step, SoA [3][sumN]
  long long sumN;
  const T* delta_k;    // q^k = x_n + delta_k (columns)
  const T* delta_k1;   // q^{k+1}
  const T* lam;        // A^-1 gbar(q^{k+1}) (columns)
  T* gbar;             // out: dL/dq^k (columns)
  T* sbar;             // accumulates (m/h^2) lam (columns)
  double* wbar;        // [n_cells_total][4] accumulates dL/dw
  const T* weights;    // [n_cells_total][4] or nullptr
  int* status;
  double h, m;
  int max_vol_iter;
  double vol_tol, vol_abs;
};

enum EpilogueMode : int { EPI_SET = 0, EPI_ADD = 1, EPI_SPLIT_SET = 2, EPI_SPLIT_ADD = 3 };

struct GemmArgs {
  const void* A;       // [Npad][Npad] symmetric operator (element type per kernel)
  // 16-bit operator in fragment order for the column-stationary kernel
  // (launch_convert_fragments), required by it, ignored by the others
  const void* A_frag = nullptr;
  const void* B;       // input columns [ncols][Npad] (float or double)
  void* C;             // output columns [ncols][Npad]
  const void* D = nullptr;  // SET modes: columns added to the product (may be C), or nullptr
  const float* colscale;  // per-column scale of B for low-precision operands, or nullptr
  int Npad;
  int ncols;
  int mode;            // EpilogueMode
  double hm;           // h^2/m (split epilogue)
  double beta;         // scale of the stored low-precision operator (split epilogue)
};

enum StatusBits : int { ST_NONFINITE = 1 };

// ---- launchers ----
// alpha: mass-proportional damping coefficient (the first increment is
// divided by 1 + alpha h); 0 without damping.
template <typename T>
hipError_t launch_predict(const ClassSlice<T>& cs, const T* pos, const T* vel, const T* force,
                          long long sumN, T* delta, T* cterm, int* status, double h,
                          double alpha, hipStream_t st);
template <typename T>
hipError_t launch_update(const ClassSlice<T>& cs, T* pos, T* vel, long long sumN, const T* delta,
                         double h, hipStream_t st);
template <typename T>
hipError_t launch_local(const LocalArgs<T>& a, int block, hipStream_t st);
template <typename T>
size_t local_smem_bytes(const ClassView<T>& cv, int block);
template <typename T>
hipError_t local_prepare(const ClassView<T>& cv, int block);
// res = rhs - M (delta - delta0) with M = (cm m + cv w_v) I + cl ((w_s + w_a)
// L_tri + w_b L_bend) per cell (w the cell's weights, m the class mass).
// The system matrix: cm = 1/h^2, cl = cv = 1; with damping cm = (1 + alpha
// h)/h^2, cl = 1 + beta/h.
template <typename T>
hipError_t launch_residual(const ClassSlice<T>& cs, const T* rhs, const T* delta,
                           const T* delta0, T* res, const T* weights, float* colmax,
                           const float* need, double need_factor, double need_thr, double cm,
                           double cl, double cv, hipStream_t st);
// Cells the static staging buffer of npfem_get_volume_noalloc holds, and the
// devices whose addresses of it are kept.
constexpr int kVolumeScratchCells = 1 << 16;
constexpr int kMaxDevices = 64;
// Device address of that buffer on the current device (looked up once per
// device with hipGetSymbolAddress).
hipError_t volume_scratch(double** out);

template <typename T>
hipError_t launch_volume(const ClassSlice<T>& cs, const T* pos, long long sumN, double* out,
                         hipStream_t st);

// Quasi-Newton step (kernels_qn.hip). Per-cell scalars, stride kQnStride:
// [gd, alpha, rho[kQnMaxHist], a[kQnMaxHist]].
constexpr int kQnMaxHist = 16;
constexpr int kQnGd = 0, kQnAlpha = 1, kQnRho = 2, kQnA = 2 + kQnMaxHist;
constexpr int kQnStride = 2 + 2 * kQnMaxHist;
template <typename T>
struct QnArgs {
  T* s[kQnMaxHist];  // history column sets s_i (batch bases)
  T* y[kQnMaxHist];  // history column sets y_i
  int hist;          // ring slots (0: no history)
  T* r_cur;          // r at the current iterate (columns)
  T* r_trial;        // r at the trial iterate
  T* v;              // first-loop result (the product's input)
  T* z;              // the product's output
  T* d;              // search direction
  T* delta;          // current iterate (increment form)
  T* delta_trial;    // trial iterate
  double* scal;      // [n_cells][stride]
  int stride;
  double* e_cur;     // [n_cells] objective at the current iterate
  double* e_trial;   // [n_cells] objective at the trial iterate
  int* done;         // [n_cells] 1 once this iteration's step is taken
  double e_tol;      // Armijo allowance relative to |E| (state rounding)
  double* energy;    // optional record [energy_iters][n_cells]
  int energy_iters;
  int n_cells;
};
template <typename T>
hipError_t launch_qn_loop1(const ClassSlice<T>& cs, const QnArgs<T>& q, int count, int head,
                           hipStream_t st);
template <typename T>
hipError_t launch_qn_loop2(const ClassSlice<T>& cs, const QnArgs<T>& q, int count, int head,
                           hipStream_t st);
template <typename T>
hipError_t launch_qn_accept(const ClassSlice<T>& cs, const QnArgs<T>& q, int head, int last,
                            int it, hipStream_t st);

// Periodic Cartesian fluid grid of the immersed-boundary transfer
// (kernels_ibm.hip): node (i, j, k) at (ox, oy, oz) + dx (i, j, k), fields
// SoA [3][nx ny nz] with flat index i + nx (j + ny k).
struct IbmGrid {
  int nx, ny, nz;
  double dx, ox, oy, oz;
};
template <typename T>
hipError_t launch_ibm_interpolate(const ClassSlice<T>& cs, const T* pos, long long sumN,
                                  const double* origins, const T* u, const IbmGrid& g, T* out,
                                  hipStream_t st);
template <typename T>
hipError_t launch_ibm_maxabs(const ClassSlice<T>& cs, const T* f, long long sumN,
                             unsigned long long* mx, int* status, hipStream_t st);
template <typename T>
hipError_t launch_ibm_spread(const ClassSlice<T>& cs, const T* pos, long long sumN,
                             const double* origins, const T* f, const IbmGrid& g,
                             const unsigned long long* mx, double n_total,
                             unsigned long long* acc, hipStream_t st);
template <typename T>
hipError_t launch_ibm_convert(const unsigned long long* acc, long long count,
                              const unsigned long long* mx, double n_total, double dx, T* out,
                              hipStream_t st);
hipError_t launch_ibm_zero(unsigned long long* p, long long count, hipStream_t st);
template <typename T>
hipError_t adjoint_prepare(const ClassView<T>& cv);
template <typename T>
hipError_t launch_adjoint_local(const AdjArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_adj_begin(const ClassSlice<T>& cs, const T* xbar, const T* vbar, long long sumN,
                            T* gbar, T* sbar, double h, hipStream_t st);
template <typename T>
hipError_t launch_adj_end(const ClassSlice<T>& cs, T* xbar, T* vbar, long long sumN,
                          const T* gbar, const T* sbar, T* fbar, double h, hipStream_t st);

// Global-step GEMM variants. kind: 0 = FP32, 1 = FP64, 2 = BF16, 3 = FP16.
hipError_t launch_gemm(int kind, int tile, const GemmArgs& g, hipStream_t st);
hipError_t gemm_prepare(int kind, int tile, int npad);
int gemm_num_tiles(int kind);
void gemm_tile_shape(int tile, int* bm, int* bn);

// FP64 Gauss-Jordan inverse of an SPD matrix in place (device, n x n,
// leading dimension ld); *pivot_fail set non-zero if a pivot is <= 0.
hipError_t launch_spd_inverse(double* A, int n, int ld, double* scratch, int* pivot_fail,
                              hipStream_t st);
// Convert an FP64 padded inverse to the stored operator.
// Copies the FP32 operator (kind 0) into fragment order: for row block rb
// and 16-k group kg, lane l's 4 values of row 16 rb + l%16 at
// k = 16 kg + 4 (l/16) .. + 3 at ((rb * (Npad/16) + kg) * 64 + l) * 4
// ((Npad/16)^2 * 256 values). Copies the 16-bit operator (kind 2: BF16,
// 3: FP16) likewise: for row block rb (16 rows), k-step ks (32 k) and lane l,
// the 8 values of row 16 rb + l%16 at k = 32 ks + 8 (l/16) .. + 7 (zero past
// Npad) are contiguous at ((rb * nks + ks) * 64 + l) * 8, so that a wave's
// load of one k-step of a row block reads 1 KB of consecutive memory. out
// holds (Npad / 16) * nks * 512 values, nks = gemm_rs_nks(Npad) (0 where
// the column-stationary kernel does not take the class: then no copy).
hipError_t launch_convert_fragments(int kind, const void* op, int Npad, void* out, hipStream_t st);
int gemm_rs_nks(int Npad);
hipError_t launch_convert_offdiag(const double* Ainv, int Npad, double s, float* out,
                                  hipStream_t st);
template <typename T>
hipError_t launch_scale(const T* src, T* dst, long long n, double s, hipStream_t st);
hipError_t launch_convert_operator(int kind, const double* Ainv, int Npad, double hm, double beta,
                                   void* out, hipStream_t st);
hipError_t launch_max_abs_split(const double* Ainv, int n, int Npad, double hm, double* out,
                                hipStream_t st);

}  // namespace npfem
