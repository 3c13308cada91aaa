// C ABI of the batched projective-dynamics solver: argument checks, batch
// layout, one-time FP64 factorisation on the GPU, per-step kernel sequence
// and its hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "mesh_ops.h"
#include "npfem.h"
#include "npfem_internal.h"

using namespace npfem;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory)
    return fail(NPFEM_ERR_OOM, "%s: out of device memory", what);
  return fail(NPFEM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                 \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

constexpr uint32_t kMeshTag = 0x6e704d31u;   // "npM1"
constexpr uint32_t kBatchTag = 0x6e704231u;  // "npB1"

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
  }
};

}  // namespace

struct npfem_mesh_s {
  uint32_t tag = kMeshTag;
  npfem_material mat{};
  MeshOps ops;
};

namespace {

struct ClassState {
  MeshOps ops;                 // copy of the class operators
  npfem_material mat{};
  int N = 0, Npad = 0, F = 0, E = 0;
  int n_cells = 0, cell0 = 0;
  long long col0 = 0, elem0 = 0, vert0 = 0;
  std::vector<void*> dev;      // device arrays of the class view
  void* view_ptrs[19] = {};    // device pointers (see upload_class)
  void* op = nullptr;          // stored global-step operator [Npad][Npad]
  void* op_frag = nullptr;     // 16-bit operator in fragment order (column-stationary kernel)
  void* op_adj = nullptr;      // non-FP64 batches: FP32 A^-1 - adj_s I (the adjoint's solve)
  double adj_s = 0.0;
  double beta = 0.0;           // split scale (low precision)
  double kappa = 0.0;          // max row sum of |Ainv - (h^2/m) I| / (h^2/m) (low precision)
  double r_rest = 0.0;         // max distance of a rest vertex from the rest centroid
  int local_block = 256;
  int gemm_tile = 3;
  int DT = 0, DH = 0, DL = 0;  // padded incidence and Laplacian widths
  // viscous damping C = alpha m I + beta ((w_s + w_a) L_tri + w_b L_bend)
  // (npfem_set_damping); 0, 0 = none
  double alpha = 0.0, beta_d = 0.0;
  // contact weight of the batch (npfem_set_contacts): w_c I in the system
  double wc = 0.0;
  // the damped system A + C/h is the undamped one with the mass and the
  // stretch/area/bend weights scaled: these are the scales at time step h;
  // the contact potentials add w_c to the diagonal, which the operator sees
  // as the mass diag_mass(h) = m (1 + alpha h) + w_c h^2
  double mass_scale(double h) const { return 1.0 + alpha * h; }
  double lap_scale(double h) const { return 1.0 + beta_d / h; }
  double diag_mass(double h) const { return mat.vertex_mass * mass_scale(h) + wc * h * h; }
  double hm_eff(double h) const { return h * h / diag_mass(h); }
};

}  // namespace

struct npfem_batch_s {
  uint32_t tag = kBatchTag;
  int device = 0;
  int precision = NPFEM_FP32;
  bool fp64 = false;
  int gemm_kind = 0;  // 0 FP32, 1 FP64, 2 BF16, 3 FP16
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  // per-class branch streams and fork/join events of the captured step
  std::vector<hipStream_t> br_stream;
  std::vector<hipEvent_t> br_join;
  hipEvent_t br_fork = nullptr;
  uint32_t flags = 0;
  int n_refine_opt = -1;
  int max_vol_iter = 0;
  std::vector<ClassState> cls;
  int n_cells = 0;
  long long sumN = 0, total_cols = 0, total_elems = 0;
  void* pos = nullptr;
  void* vel = nullptr;
  void* delta = nullptr;
  void* delta2 = nullptr;  // the other iterate buffer (PD iterations alternate)
  void* cterm = nullptr;
  void* rhs = nullptr;
  void* res = nullptr;
  void* damp = nullptr;         // right-hand side with the stiffness damping term (columns)
  // quasi-Newton step (npfem_set_quasi_newton): history slots (-1: classic
  // PD), line-search rounds, buffers
  int qn_hist = -1;
  int qn_hist_cap = -1;  // history the column buffer holds
  int qn_ls = 3;
  void* qn_cols = nullptr;        // (4 + 2 hist) column sets: r, v, z, d, s_i, y_i
  double* qn_scal = nullptr;      // [n_cells][kQnStride]
  double* qn_e = nullptr;         // [2][n_cells] objective: current, trial
  int* qn_done = nullptr;         // [n_cells]
  // immersed-boundary spreading: 64-bit fixed-point accumulators [3][nodes]
  // and the max |F| word in front of them
  unsigned long long* ibm_acc = nullptr;
  long long ibm_cap = 0;  // nodes the accumulators hold
  // contact data (caller-owned device arrays, npfem_set_contacts)
  const void* ct_points = nullptr;
  const void* ct_normals = nullptr;
  const int* ct_off = nullptr;
  long long ct_np = 0;
  float* colmax = nullptr;      // max |r| per column (16-bit products)
  float* colmax_res = nullptr;  // max |res| per column of the correction sweeps
  int* status = nullptr;
  double* energy = nullptr;
  int energy_cap = 0;    // iterations the energy buffer holds
  int energy_iters = 0;  // iterations recorded by the last step
  double* volume_buf = nullptr;
  void* weights_dev = nullptr;
  bool per_cell = false;
  std::vector<double> weights_host;  // [n_cells][4] effective weights
  std::vector<int> cell_class;       // [n_cells] mesh class of each cell
  double dt = -1.0;
  int n_refine = 0;
  double rho = 0.0, rho_w = 0.0;  // contraction estimates of the sweeps (choose_refine)
  bool tuned = false;
  hipGraphExec_t graph = nullptr;
  const void* graph_forces = nullptr;
  int graph_iters = 0;
  // npfem_run: n_steps steps captured as one graph
  hipGraphExec_t run_graph = nullptr;
  const void* run_forces = nullptr;
  int run_iters = 0, run_steps = 0;
  std::vector<void*> allocs;
  // differentiable rollout: checkpoints and recompute workspace
  void* ckpt = nullptr;          // [n_seg][2][3][sumN] positions then velocities
  size_t ckpt_bytes = 0;
  void* tape = nullptr;          // [ckpt_every][3 sumN + (n_iter + 1) total_elems]
  size_t tape_bytes = 0;
  void* adj_work = nullptr;      // xs, vs, xbar, vbar (3 sumN each); lam, gbar, sbar (columns)
  size_t adj_work_bytes = 0;
  int ro_steps = 0, ro_iter = 0, ro_every = 0;
  double ro_dt = 0.0;
  const void* ro_forces = nullptr;
  bool ro_valid = false;
  // kernel timing (NPFEM_OPT_KERNEL_TIMING): event pairs around launches
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_pending;  // (kind, start event index)
  size_t ev_used = 0;
  double kt_ms[NPFEM_KERNEL_KINDS] = {};
  long long kt_n[NPFEM_KERNEL_KINDS] = {};

  int ev_begin(hipStream_t st) {
    if (ev_used + 2 > ev_pool.size()) {
      for (int i = 0; i < 2; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        ev_pool.push_back(e);
      }
    }
    const int idx = (int)ev_used;
    ev_used += 2;
    if (hipEventRecord(ev_pool[idx], st) != hipSuccess) return -1;
    return idx;
  }
  void ev_end(int idx, int kind, hipStream_t st) {
    if (hipEventRecord(ev_pool[idx + 1], st) == hipSuccess) ev_pending.push_back({kind, idx});
  }
  hipError_t ev_harvest() {
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    for (auto& p : ev_pending) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev_pool[p.second], ev_pool[p.second + 1]);
      if (e != hipSuccess) return e;
      kt_ms[p.first] += ms;
      kt_n[p.first] += 1;
    }
    ev_pending.clear();
    ev_used = 0;
    return hipSuccess;
  }

  int ensure_branches() {
    if (!br_fork) {
      hipError_t e0 = hipEventCreateWithFlags(&br_fork, hipEventDisableTiming);
      if (e0 != hipSuccess) {
        br_fork = nullptr;
        return hip_fail(e0, "branch events");
      }
    }
    while (br_stream.size() < cls.size()) {
      hipStream_t s = nullptr;
      hipError_t er = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
      if (er != hipSuccess) return hip_fail(er, "branch streams");
      br_stream.push_back(s);
    }
    while (br_join.size() < cls.size()) {
      hipEvent_t e = nullptr;
      hipError_t er = hipEventCreateWithFlags(&e, hipEventDisableTiming);
      if (er != hipSuccess) return hip_fail(er, "branch events");
      br_join.push_back(e);
    }
    return NPFEM_OK;
  }

  ~npfem_batch_s() {
    if (graph) hipGraphExecDestroy(graph);
    if (run_graph) hipGraphExecDestroy(run_graph);
    for (hipStream_t s : br_stream) hipStreamDestroy(s);
    for (hipEvent_t e : br_join) hipEventDestroy(e);
    if (br_fork) hipEventDestroy(br_fork);
    for (hipEvent_t e : ev_pool) hipEventDestroy(e);
    for (auto& c : cls) {
      for (void* p : c.dev) hipFree(p);
      if (c.op) hipFree(c.op);
      if (c.op_frag) hipFree(c.op_frag);
      if (c.op_adj) hipFree(c.op_adj);
    }
    for (void* p : allocs) hipFree(p);
    if (ckpt) hipFree(ckpt);
    if (tape) hipFree(tape);
    if (adj_work) hipFree(adj_work);
    if (cap_stream) hipStreamDestroy(cap_stream);
  }
};

namespace {

int dalloc(npfem_batch_s* b, void** p, size_t bytes, const char* what) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return hip_fail(e, what);
  b->allocs.push_back(*p);
  return NPFEM_OK;
}

template <typename T>
int upload_vec(ClassState& c, const std::vector<T>& h, void** out, const char* what) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(16, h.size() * sizeof(T));
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return hip_fail(e, what);
  c.dev.push_back(p);
  if (!h.empty()) {
    e = hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, what);
  }
  *out = p;
  return NPFEM_OK;
}

template <typename T>
std::vector<T> cast_vec(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

// Uploads the class operators in the working precision T.
template <typename T>
int upload_class(ClassState& c) {
  const MeshOps& M = c.ops;
  // Device triangle order: by first appearance in the vertex-major incidence
  // lists, so that the triangles that consecutive vertices gather (the k-th
  // of each) sit close together in LDS, which spreads one wave's reads over
  // the banks. Only storage moves: each vertex still sums its triangles in
  // ascending mesh order, so results do not depend on it.
  std::vector<int> tord, tpos(M.F, -1);
  tord.reserve(M.F);
  for (int i = 0; i < M.N; ++i)
    for (int e = M.vt_ptr[i]; e < M.vt_ptr[i + 1]; ++e)
      if (tpos[M.vt_tri[e]] < 0) {
        tpos[M.vt_tri[e]] = (int)tord.size();
        tord.push_back(M.vt_tri[e]);
      }
  for (int t = 0; t < M.F; ++t)
    if (tpos[t] < 0) {  // (a triangle no vertex lists: not on a valid mesh)
      tpos[t] = (int)tord.size();
      tord.push_back(t);
    }
  std::vector<int> tri_v(4 * (size_t)M.F), hin_v(4 * (size_t)M.E);
  std::vector<T> tri_rec(8 * (size_t)M.F, T(0)), hin_rec(8 * (size_t)M.E, T(0));
  for (int i = 0; i < M.F; ++i) {
    const int t = tord[i];
    for (int r = 0; r < 3; ++r) tri_v[4 * (size_t)i + r] = M.tris[3 * (size_t)t + r];
    tri_v[4 * (size_t)i + 3] = 0;
    for (int k = 0; k < 6; ++k) tri_rec[8 * (size_t)i + k] = T(M.G[6 * (size_t)t + k]);
    tri_rec[8 * (size_t)i + 6] = T(M.area[t]);
  }
  for (int e = 0; e < M.E; ++e) {
    for (int r = 0; r < 4; ++r) {
      hin_v[4 * (size_t)e + r] = M.hin[4 * (size_t)e + r];
      hin_rec[8 * (size_t)e + r] = T(M.K[4 * (size_t)e + r]);
    }
    hin_rec[8 * (size_t)e + 4] = T(M.cw[e]);
    hin_rec[8 * (size_t)e + 5] = T(M.rr[e]);
  }
  int rc;
  void** v = c.view_ptrs;
  if ((rc = upload_vec(c, tri_v, &v[0], "tri_v"))) return rc;
  if ((rc = upload_vec(c, tri_rec, &v[1], "tri_rec"))) return rc;
  if ((rc = upload_vec(c, hin_v, &v[2], "hin_v"))) return rc;
  if ((rc = upload_vec(c, hin_rec, &v[3], "hin_rec"))) return rc;
  if constexpr (sizeof(T) == 8) {
    v[15] = v[1];
    v[16] = v[3];
  } else {
    std::vector<double> tri64(8 * (size_t)M.F, 0.0), hin64(8 * (size_t)M.E, 0.0);
    for (int i = 0; i < M.F; ++i) {
      const int t = tord[i];
      for (int k = 0; k < 6; ++k) tri64[8 * (size_t)i + k] = M.G[6 * (size_t)t + k];
      tri64[8 * (size_t)i + 6] = M.area[t];
    }
    for (int e = 0; e < M.E; ++e) {
      for (int r = 0; r < 4; ++r) hin64[8 * (size_t)e + r] = M.K[4 * (size_t)e + r];
      hin64[8 * (size_t)e + 4] = M.cw[e];
      hin64[8 * (size_t)e + 5] = M.rr[e];
    }
    if ((rc = upload_vec(c, tri64, &v[15], "tri_rec64"))) return rc;
    if ((rc = upload_vec(c, hin64, &v[16], "hin_rec64"))) return rc;
  }
  // fixed-width, vertex-major incidence ([N][slot]); entries keep ascending
  // element order, padding contributes zero
  const int N = M.N;
  {
    double cen[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
    for (int i = 0; i < N; ++i)
      for (int d = 0; d < 3; ++d) cen[d] += M.X[3 * (size_t)i + d] / N;
    for (int i = 0; i < N; ++i) {
      double q = 0.0;
      for (int d = 0; d < 3; ++d) q += (M.X[3 * (size_t)i + d] - cen[d]) * (M.X[3 * (size_t)i + d] - cen[d]);
      r2 = std::max(r2, q);
    }
    c.r_rest = std::sqrt(r2);
  }
  c.DT = 0;
  c.DH = 0;
  for (int i = 0; i < N; ++i) {
    c.DT = std::max(c.DT, M.vt_ptr[i + 1] - M.vt_ptr[i]);
    c.DH = std::max(c.DH, M.vh_ptr[i + 1] - M.vh_ptr[i]);
  }
  std::vector<int> pt_tri((size_t)c.DT * N, 0), pt_fan((size_t)c.DT * N, N | (N << 16));
  std::vector<T> pt_g(2 * (size_t)c.DT * N, T(0));
  for (int i = 0; i < N; ++i) {
    for (int e = M.vt_ptr[i], k = 0; e < M.vt_ptr[i + 1]; ++e, ++k) {
      const size_t s = (size_t)i * c.DT + k;
      pt_tri[s] = tpos[M.vt_tri[e]];
      pt_fan[s] = M.vt_fan[e];
      pt_g[2 * s] = T(M.vt_g[2 * (size_t)e]);
      pt_g[2 * s + 1] = T(M.vt_g[2 * (size_t)e + 1]);
    }
  }
  std::vector<int> ph_hin((size_t)c.DH * N, 0);
  std::vector<T> ph_k((size_t)c.DH * N, T(0));
  for (int i = 0; i < N; ++i) {
    for (int e = M.vh_ptr[i], k = 0; e < M.vh_ptr[i + 1]; ++e, ++k) {
      const size_t s = (size_t)i * c.DH + k;
      ph_hin[s] = M.vh_hin[e];
      ph_k[s] = T(M.vh_k[e]);
    }
  }
  if ((rc = upload_vec(c, pt_tri, &v[5], "vt_tri"))) return rc;
  if ((rc = upload_vec(c, pt_g, &v[6], "vt_g"))) return rc;
  if ((rc = upload_vec(c, pt_fan, &v[7], "vt_fan"))) return rc;
  // one-ring in fan order, when every vertex's fan closes into a single cycle
  // of distinct neighbours (closed manifold): the volume gradient then reads
  // each neighbour once, (1/6) sum_k n_k x n_k+1
  {
    std::vector<int> pt_ring((size_t)c.DT * N, 0);
    bool ok = c.DT >= 3;
    for (int i = 0; i < N && ok; ++i) {
      const int e0 = M.vt_ptr[i], deg = M.vt_ptr[i + 1] - e0;
      int* ring = &pt_ring[(size_t)i * c.DT];
      if (deg < 3) {
        ok = false;
        break;
      }
      ring[0] = M.vt_fan[e0] & 0xffff;
      int cur = M.vt_fan[e0] >> 16;
      for (int k = 1; k < deg && ok; ++k) {
        for (int j = 0; j < k; ++j) ok = ok && ring[j] != cur;
        ring[k] = cur;
        int nxt = -1;
        for (int e = e0; e < e0 + deg; ++e)
          if ((M.vt_fan[e] & 0xffff) == cur) nxt = M.vt_fan[e] >> 16;
        ok = ok && nxt >= 0;
        cur = nxt;
      }
      ok = ok && cur == ring[0];
      for (int k = deg; k < c.DT; ++k) ring[k] = ring[0];
    }
    if (ok && (rc = upload_vec(c, pt_ring, &v[8], "vt_ring"))) return rc;
  }
  if ((rc = upload_vec(c, ph_hin, &v[9], "vh_hin"))) return rc;
  if ((rc = upload_vec(c, ph_k, &v[10], "vh_k"))) return rc;
  c.DL = 0;
  for (int i = 0; i < N; ++i) c.DL = std::max(c.DL, M.lap_ptr[i + 1] - M.lap_ptr[i]);
  std::vector<int> pl_col((size_t)c.DL * N, N);
  std::vector<T> pl_t((size_t)c.DL * N, T(0)), pl_b((size_t)c.DL * N, T(0));
  for (int i = 0; i < N; ++i) {
    for (int e = M.lap_ptr[i], k = 0; e < M.lap_ptr[i + 1]; ++e, ++k) {
      const size_t s = (size_t)k * N + i;
      pl_col[s] = M.lap_col[e];
      pl_t[s] = T(M.lap_t[e]);
      pl_b[s] = T(M.lap_b[e]);
    }
  }
  if ((rc = upload_vec(c, pl_col, &v[12], "lap_col"))) return rc;
  if ((rc = upload_vec(c, pl_t, &v[13], "lap_t"))) return rc;
  if ((rc = upload_vec(c, pl_b, &v[14], "lap_b"))) return rc;
  return NPFEM_OK;
}

template <typename T>
ClassSlice<T> slice_of(const ClassState& c) {
  ClassSlice<T> s;
  ClassView<T>& v = s.cv;
  v.N = c.N;
  v.Npad = c.Npad;
  v.F = c.F;
  v.E = c.E;
  v.tri_v = (const int4*)c.view_ptrs[0];
  v.tri_rec = (const T*)c.view_ptrs[1];
  v.hin_v = (const int4*)c.view_ptrs[2];
  v.hin_rec = (const T*)c.view_ptrs[3];
  v.tri_rec64 = (const double*)c.view_ptrs[15];
  v.hin_rec64 = (const double*)c.view_ptrs[16];
  v.DT = c.DT;
  v.DH = c.DH;
  v.vt_tri = (const int*)c.view_ptrs[5];
  v.vt_g = (const T*)c.view_ptrs[6];
  v.vt_fan = (const int*)c.view_ptrs[7];
  v.vt_ring = (const int*)c.view_ptrs[8];
  v.vh_hin = (const int*)c.view_ptrs[9];
  v.vh_k = (const T*)c.view_ptrs[10];
  v.DL = c.DL;
  v.lap_col = (const int*)c.view_ptrs[12];
  v.lap_t = (const T*)c.view_ptrs[13];
  v.lap_b = (const T*)c.view_ptrs[14];
  v.vol_rest = c.ops.vol_rest;
  s.n_cells = c.n_cells;
  s.cell0 = c.cell0;
  s.col0 = c.col0;
  s.elem0 = c.elem0;
  s.vert0 = c.vert0;
  s.mass = T(c.mat.vertex_mass);
  s.w_nom[0] = T(c.mat.w_stretch);
  s.w_nom[1] = T(c.mat.w_area);
  s.w_nom[2] = T(c.mat.w_bend);
  s.w_nom[3] = T(c.mat.w_volume);
  return s;
}

// Settling tests of the volume projection's multiplier: relative to the
// correction itself, and absolute as an RMS vertex displacement that is a
// small fraction of the cell radius (FP32: 4e-9 R, far below one ulp of the
// coordinates; FP64: 1e-15 R). At rest-like states the multiplier sits at
// the rounding noise of the volume sum, where only the absolute test can fire.
template <typename T>
void set_volume_tolerances(LocalArgs<T>& a, const ClassState& c, bool fp64) {
  a.vol_tol = fp64 ? 1e-14 : 1e-4;
  a.vol_abs = (fp64 ? 1e-15 : 4e-9) * c.ops.radius * std::sqrt((double)c.N);
}

int precision_of_gemm(int prec) {
  switch (prec) {
    case NPFEM_FP64: return 1;
    case NPFEM_FP32: return 0;
    case NPFEM_BF16_REFINE: return 2;
    case NPFEM_FP16_REFINE: return 3;
  }
  return -1;
}

// Number of correction sweeps after each global solve. Per-cell weights make
// the cell matrix A_c differ from the shared nominal A_0; the sweep
// delta <- delta + A_0^-1 (r - A_c delta) contracts the error by at most
// rho = max_c |A_c - A_0| / lambda_min(A_0), with lambda_min(A_0) >= m/h^2 + w_v
// (both Laplacians are positive semi-definite). Low-precision operators add
// two sweeps.
// Correction sweeps after the global-step GEMM. Each sweep multiplies the
// error of the solve by at most rho = rho_w + rho_lp + rho_w rho_lp, where
// rho_w = max_c |A_c - A_0| / (m/h^2 + w_v) bounds ||A_0^-1 (A_c - A_0)|| for
// per-cell weights (A_0 the class matrix, m/h^2 + w_v its smallest
// eigenvalue) and rho_lp bounds the relative error of the 16-bit product:
// 2 u kappa for the rounding of both operands (u = 2^-8 BF16, 2^-11 FP16)
// plus, for FP16, N 2^-25 beta for operator entries in the subnormal range.
// The GEMM plus s sweeps leave rho^(s+1) of the solution; s is the least
// count that brings this to the unit roundoff of the state type (2^-24 FP32,
// 2^-53 FP64). n_refine >= 0 in the options fixes the count instead.
int choose_refine(npfem_batch_s* b, double dt, int* out) {
  if (b->n_refine_opt >= 0) {
    *out = b->n_refine_opt;
    return NPFEM_OK;
  }
  double rho_w = 0.0, rho_lp = 0.0;
  if (b->gemm_kind >= 2) {
    const double u = b->gemm_kind == 2 ? std::ldexp(1.0, -8) : std::ldexp(1.0, -11);
    for (const ClassState& c : b->cls) {
      if (c.n_cells == 0) continue;
      double r = 2.0 * u * c.kappa;
      if (b->gemm_kind == 3) r += c.N * std::ldexp(1.0, -25) * c.beta;
      rho_lp = std::max(rho_lp, r);
    }
  }
  if (b->per_cell) {
    for (const ClassState& c : b->cls) {
      const double w0[4] = {c.mat.w_stretch, c.mat.w_area, c.mat.w_bend, c.mat.w_volume};
      const double lmin = c.diag_mass(dt) / (dt * dt) + c.mat.w_volume;
      const double ls = c.lap_scale(dt);
      for (int i = 0; i < c.n_cells; ++i) {
        const double* w = &b->weights_host[4 * (size_t)(c.cell0 + i)];
        const double dev = ls * (std::fabs(w[0] + w[1] - w0[0] - w0[1]) * c.ops.norm_t +
                                 std::fabs(w[2] - w0[2]) * c.ops.norm_b) +
                           std::fabs(w[3] - w0[3]);
        rho_w = std::max(rho_w, dev / lmin);
      }
    }
  }
  const double rho = rho_w + rho_lp + rho_w * rho_lp;
  b->rho = rho;
  b->rho_w = rho_w;
  if (rho >= 0.9)
    return fail(NPFEM_ERR_INVALID_ARG,
                "the shared operator does not contract the correction (estimate %.3g: per-cell "
                "weights too far from the class material, or the time step too large for the "
                "16-bit product); set n_refine explicitly or split the class", rho);
  int n = 0;
  if (rho > 0.0) {
    const double tol = b->fp64 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
    n = std::max(0, (int)std::ceil(std::log(tol) / std::log(rho)) - 1);
    n = std::min(n, 60);
  }
  *out = n;
  return NPFEM_OK;
}

// Sets the effective per-cell weights (NULL = nominal), uploads them when any
// differs from its class material and re-derives the correction sweeps.
int apply_weights(npfem_batch_s* b, const double* cell_weights) {
  const int n = b->n_cells;
  b->weights_host.resize(4 * (size_t)n);
  b->per_cell = false;
  for (int c = 0; c < n; ++c) {
    const npfem_material& m = b->cls[b->cell_class[c]].mat;
    const double nom[4] = {m.w_stretch, m.w_area, m.w_bend, m.w_volume};
    for (int i = 0; i < 4; ++i) {
      const double w = cell_weights ? cell_weights[4 * (size_t)c + i] : nom[i];
      b->weights_host[4 * (size_t)c + i] = w;
      if (w != nom[i]) b->per_cell = true;
    }
  }
  if (b->per_cell) {
    const size_t tsz = b->fp64 ? sizeof(double) : sizeof(float);
    if (!b->weights_dev) {
      const int rc = dalloc(b, &b->weights_dev, tsz * 4 * (size_t)n, "weights");
      if (rc) return rc;
    }
    hipError_t e;
    if (b->fp64) {
      e = hipMemcpy(b->weights_dev, b->weights_host.data(), 8 * 4 * (size_t)n,
                    hipMemcpyHostToDevice);
    } else {
      std::vector<float> wf(b->weights_host.begin(), b->weights_host.end());
      e = hipMemcpy(b->weights_dev, wf.data(), 4 * 4 * (size_t)n, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_fail(e, "weights upload");
  }
  if (b->dt > 0.0) {
    const int rc = choose_refine(b, b->dt, &b->n_refine);
    if (rc) return rc;
  }
  return NPFEM_OK;
}

int factorise(npfem_batch_s* b, double dt) {
  int Nmax = 0;
  for (auto& c : b->cls) Nmax = std::max(Nmax, c.Npad);
  double* dA = nullptr;
  double* scratch = nullptr;
  int* dfail = nullptr;
  double* dbeta = nullptr;
  auto cleanup = [&]() {
    if (dA) hipFree(dA);
    if (scratch) hipFree(scratch);
    if (dfail) hipFree(dfail);
    if (dbeta) hipFree(dbeta);
  };
  hipError_t e = hipMalloc(&dA, sizeof(double) * (size_t)Nmax * Nmax);
  if (e == hipSuccess) e = hipMalloc(&scratch, sizeof(double) * 2 * (size_t)Nmax);
  if (e == hipSuccess) e = hipMalloc(&dfail, sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&dbeta, sizeof(double));
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "factorisation workspace");
  }
  std::vector<double> hA;
  const size_t esz = b->gemm_kind == 1 ? 8 : (b->gemm_kind == 0 ? 4 : 2);
  for (auto& c : b->cls) {
    if (c.n_cells == 0) continue;
    hA.assign((size_t)c.Npad * c.Npad, 0.0);
    // (damped: A + C/h, the system matrix of the scaled mass and weights)
    const double ls = c.lap_scale(dt);
    const double w0[4] = {ls * c.mat.w_stretch, ls * c.mat.w_area, ls * c.mat.w_bend,
                          c.mat.w_volume};
    dense_system_matrix(c.ops, w0, c.diag_mass(dt), dt, hA.data(), c.Npad);
    int hfail = 0;
    e = hipMemcpy(dA, hA.data(), sizeof(double) * hA.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(dfail, 0, sizeof(int));
    if (e == hipSuccess) e = launch_spd_inverse(dA, c.N, c.Npad, scratch, dfail, nullptr);
    if (e == hipSuccess) e = hipMemcpy(&hfail, dfail, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      cleanup();
      return hip_fail(e, "FP64 inverse");
    }
    if (hfail) {
      cleanup();
      return fail(NPFEM_ERR_NOT_SPD, "system matrix of a %d-vertex class is not SPD", c.N);
    }
    const double hm = c.hm_eff(dt);
    c.beta = 0.0;
    c.kappa = 0.0;
    if (b->gemm_kind != 1) {
      if (b->gemm_kind >= 2) {
        e = launch_max_abs_split(dA, c.N, c.Npad, hm, dbeta, nullptr);
        if (e == hipSuccess) e = hipMemcpy(&c.beta, dbeta, sizeof(double), hipMemcpyDeviceToHost);
      }
      // kappa = max_i sum_j |Ainv_ij - hm delta_ij| / hm: the size of the part
      // of the operator that passes through the 16-bit product; with it,
      // |A^-1|_inf <= hm (1 + kappa) bounds the solve for the sweep test
      if (e == hipSuccess)
        e = hipMemcpy(hA.data(), dA, sizeof(double) * hA.size(), hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "operator scale");
      }
      for (int i = 0; i < c.N; ++i) {
        double rs = 0.0;
        for (int j = 0; j < c.N; ++j)
          rs += std::fabs(hA[(size_t)i * c.Npad + j] - (i == j ? hm : 0.0));
        c.kappa = std::max(c.kappa, rs / hm);
      }
    }
    if (!c.op) {
      e = hipMalloc(&c.op, esz * (size_t)c.Npad * c.Npad);
      if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "operator storage");
      }
    }
    e = launch_convert_operator(b->gemm_kind, dA, c.Npad, hm, c.beta, c.op, nullptr);
    // the adjoint's operator for FP32 state: A^-1 without its identity part
    if (e == hipSuccess && b->gemm_kind != 1) {
      if (!c.op_adj) e = hipMalloc(&c.op_adj, sizeof(float) * (size_t)c.Npad * c.Npad);
      c.adj_s = hm;
      if (e == hipSuccess) e = launch_convert_offdiag(dA, c.Npad, hm, static_cast<float*>(c.op_adj), nullptr);
    }
    // fragment copy for the column-stationary kernel, where it takes the
    // class (FP32: 48 columns of Npad values in LDS; 16-bit: k-steps <= 24)
    const bool frag = b->gemm_kind == 0 ? (size_t)48 * c.Npad * 4 <= 160 * 1024
                    : b->gemm_kind >= 2 && gemm_rs_nks(c.Npad) > 0;
    if (e == hipSuccess && frag) {
      const size_t nfrag = b->gemm_kind == 0 ? (size_t)(c.Npad / 16) * (c.Npad / 16) * 256
                                             : (size_t)(c.Npad / 16) * gemm_rs_nks(c.Npad) * 512;
      if (!c.op_frag) e = hipMalloc(&c.op_frag, esz * nfrag);
      if (e == hipSuccess) e = launch_convert_fragments(b->gemm_kind, c.op, c.Npad, c.op_frag, nullptr);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      cleanup();
      return hip_fail(e, "operator conversion");
    }
  }
  cleanup();
  int rc = choose_refine(b, dt, &b->n_refine);
  if (rc) return rc;
  b->dt = dt;
  return NPFEM_OK;
}

#define NPFEM_TIMED(kind, expr, what)                           \
  do {                                                          \
    const bool t_ = (b->flags & NPFEM_OPT_KERNEL_TIMING) != 0;  \
    const int idx_ = t_ ? b->ev_begin(st) : -1;                 \
    HIP_TRY(expr, what);                                        \
    if (idx_ >= 0) b->ev_end(idx_, kind, st);                   \
  } while (0)

// Correction sweeps that a cell does not need are skipped on the device:
// FP32 state (FP32 or 16-bit products) with the automatic count.
bool sweeps_adaptive(const npfem_batch_s* b) {
  return b->n_refine > 0 && b->n_refine_opt < 0 && !b->fp64;
}

// C = D + A_c^-1 B for one class (D = nullptr: none; D may be C): one GEMM
// with the stored class operator, then the correction sweeps
// C += A_0^-1 (B - A_c (C - D)) (per-cell weights, low precision). B, C and D
// are batch column buffers.
template <typename T>
int enqueue_solve(npfem_batch_s* b, ClassState& c, T* B, T* C, const T* D, double h,
                  hipStream_t st, bool step_solve, T* adj_sb = nullptr) {
  T* res = static_cast<T*>(b->res);
  const T* w = b->per_cell ? static_cast<const T*>(b->weights_dev) : nullptr;
  const bool lp = b->gemm_kind >= 2;
  float* colmax = lp ? b->colmax : nullptr;
  // (only the step's own solves: the per-column maxima describe its
  // right-hand side)
  const bool adapt = step_solve && sweeps_adaptive(b);
  GemmArgs g;
  g.A = c.op;
  g.A_frag = c.op_frag;
  g.B = B + c.elem0;
  g.C = C + c.elem0;
  g.D = D ? D + c.elem0 : nullptr;
  g.colscale = colmax ? colmax + c.col0 : nullptr;
  g.Npad = c.Npad;
  g.ncols = 3 * c.n_cells;
  g.mode = lp ? EPI_SPLIT_SET : EPI_SET;
  g.hm = c.hm_eff(h);
  g.beta = c.beta;
  if (adj_sb && c.op_adj) {
    // the adjoint's solve for FP32 state: C = (A^-1 - s I) B + s B with the
    // FP32 operator that keeps the constraints' coupling to FP32 precision
    // (adj_sb: workspace for s B)
    const long long n = 3LL * c.n_cells * c.Npad;
    HIP_TRY(launch_scale<T>(B + c.elem0, adj_sb + c.elem0, n, c.adj_s, st), "adjoint solve");
    GemmArgs a = g;
    a.A = c.op_adj;
    a.A_frag = nullptr;
    a.D = adj_sb + c.elem0;
    a.colscale = nullptr;
    a.mode = EPI_SET;
    HIP_TRY(launch_gemm(0, 0, a, st), "adjoint solve");
  } else {
    NPFEM_TIMED(NPFEM_KERNEL_GLOBAL, launch_gemm(b->gemm_kind, c.gemm_tile, g, st), "global step");
  }
  // FP32 state with the automatic sweep count: sweep s + 1 runs for a cell
  // only while the bound rho^(s+1) |delta| on the error left in its delta
  // exceeds the FP32 rounding of the cell's coordinates (2^-24 of its rest
  // radius), with |delta| <= |A_c^-1| max |r| <= hm (1 + kappa) / (1 - rho_w)
  // max |r| (max |r| per column from the local step); the per-cell test runs
  // on the device (residual step), which marks the columns that need no
  // correction with a zero maximum.
  double bound = g.hm * (1.0 + c.kappa) / std::max(1e-300, 1.0 - b->rho_w);
  for (int s = 0; s < b->n_refine; ++s) {
    bound *= b->rho;
    NPFEM_TIMED(NPFEM_KERNEL_RESIDUAL,
                launch_residual<T>(slice_of<T>(c), B, C, D, res, w,
                                   (lp || adapt) ? b->colmax_res : nullptr,
                                   adapt ? b->colmax : nullptr, bound,
                                   std::ldexp(1.0, -24) * c.r_rest,
                                   c.diag_mass(h) / (h * h * c.mat.vertex_mass), c.lap_scale(h),
                                   1.0, st),
                "residual");
    GemmArgs r = g;
    r.B = res + c.elem0;
    r.colscale = (lp || adapt) ? b->colmax_res + c.col0 : nullptr;
    r.mode = lp ? EPI_SPLIT_ADD : EPI_ADD;
    NPFEM_TIMED(NPFEM_KERNEL_GLOBAL, launch_gemm(b->gemm_kind, c.gemm_tile, r, st), "refinement");
  }
  return NPFEM_OK;
}

// One time step of the cells of class c on state (pos, vel): predict, n_iter
// (local step, global solve) iterations, update. dslots, if given, holds
// n_iter + 1 column buffers: iterate k is read from dslots[k] and the solve
// writes dslots[k + 1] (recording every PD iterate for the adjoint);
// otherwise the iterates alternate between the batch's two iterate buffers.
// The solve of iteration k forms iterate k + 1 as iterate k plus
// A^-1 (cterm - (m/h^2) delta_k + R(q_k)) (the local step's increment form,
// see kernels_local.hip). Classes touch
// disjoint parts of every batch buffer, so their chains are independent.
template <typename T>
int enqueue_class_step_qn(npfem_batch_s* b, ClassState& c, T* pos, T* vel, const T* forces,
                          double h, int n_iter, hipStream_t st);

template <typename T>
int enqueue_class_step(npfem_batch_s* b, ClassState& c, T* pos, T* vel, const T* forces,
                       double h, int n_iter, hipStream_t st, T* const* dslots) {
  if (b->qn_hist >= 0 && !dslots) return enqueue_class_step_qn<T>(b, c, pos, vel, forces, h, n_iter, st);
  T* delta = static_cast<T*>(b->delta);
  T* delta2 = static_cast<T*>(b->delta2);
  T* cterm = static_cast<T*>(b->cterm);
  T* rhs = static_cast<T*>(b->rhs);
  const T* w = b->per_cell ? static_cast<const T*>(b->weights_dev) : nullptr;
  float* colmax = (b->gemm_kind >= 2 || sweeps_adaptive(b)) ? b->colmax : nullptr;
  const bool want_energy = (b->flags & NPFEM_OPT_ENERGY) != 0 && !dslots;
  // iterate k: dslots[k], else the two iterate buffers in turn (the solve
  // reads iterate k and writes k + 1 = k + A^-1 r)
  auto slot = [&](int k) { return dslots ? dslots[k] : (k & 1) ? delta2 : delta; };
  NPFEM_TIMED(NPFEM_KERNEL_PREDICT,
              launch_predict<T>(slice_of<T>(c), pos, vel, forces, b->sumN, slot(0), cterm,
                                b->status, h, c.alpha, st),
              "predict");
  for (int it = 0; it < n_iter; ++it) {
    LocalArgs<T> a;
    a.cs = slice_of<T>(c);
    a.pos = pos;
    a.sumN = b->sumN;
    a.delta = slot(it);
    a.cterm = cterm;
    a.rhs = rhs;
    a.weights = w;
    a.energy = want_energy ? b->energy + (size_t)it * b->n_cells : nullptr;
    a.colmax = colmax;
    a.status = b->status;
    a.h = h;
    a.m = c.mat.vertex_mass;
    a.mdelta = c.mat.vertex_mass * c.mass_scale(h) / (h * h);
    if (c.wc != 0.0) {
      a.contact_w = c.wc;
      a.contact_p = static_cast<const T*>(b->ct_points);
      a.contact_n = static_cast<const T*>(b->ct_normals);
      a.contact_off = b->ct_off;
      a.contact_np = b->ct_np;
    }
    a.max_vol_iter = b->max_vol_iter;
    set_volume_tolerances(a, c, b->fp64);
    NPFEM_TIMED(NPFEM_KERNEL_LOCAL, launch_local<T>(a, c.local_block, st), "local step");
    T* B = rhs;
    if (c.beta_d != 0.0) {
      // stiffness-proportional damping: r -= (beta/h) K_d delta (K_d =
      // (w_s + w_a) L_tri + w_b L_bend), the part of C delta/h that the local
      // step does not form (its alpha m delta/h part is in mdelta)
      B = static_cast<T*>(b->damp);
      NPFEM_TIMED(NPFEM_KERNEL_RESIDUAL,
                  launch_residual<T>(slice_of<T>(c), rhs, slot(it), nullptr, B, w, colmax,
                                     nullptr, 0.0, 0.0, 0.0, c.beta_d / h, 0.0, st),
                  "damping term");
    }
    const int rc = enqueue_solve<T>(b, c, B, slot(it + 1), slot(it), h, st, true);
    if (rc) return rc;
  }
  NPFEM_TIMED(NPFEM_KERNEL_UPDATE,
              launch_update<T>(slice_of<T>(c), pos, vel, b->sumN, slot(n_iter), h, st),
              "update");
  return NPFEM_OK;
}

// The quasi-Newton form of a class's step (kernels_qn.hip): predict; the
// local step at q^0 gives r and the objective; then n_iter times: first loop,
// product with the class operator, second loop and full-step trial, and up to
// qn_ls rounds of (local step at the trial for the cells still searching,
// Armijo test / halving); update. The iterates live in the delta buffer, the
// trials in delta2, the local step writes r to the QN r buffer (initial) or
// rhs (trials).
template <typename T>
int enqueue_class_step_qn(npfem_batch_s* b, ClassState& c, T* pos, T* vel, const T* forces,
                          double h, int n_iter, hipStream_t st) {
  T* delta = static_cast<T*>(b->delta);
  T* trial = static_cast<T*>(b->delta2);
  T* cterm = static_cast<T*>(b->cterm);
  const size_t cs_elems = (size_t)b->total_elems;
  T* cols = static_cast<T*>(b->qn_cols);
  QnArgs<T> q{};
  q.hist = b->qn_hist;
  q.r_cur = cols;
  q.v = cols + cs_elems;
  q.z = cols + 2 * cs_elems;
  q.d = cols + 3 * cs_elems;
  for (int i = 0; i < q.hist; ++i) {
    q.s[i] = cols + (4 + 2 * (size_t)i) * cs_elems;
    q.y[i] = cols + (5 + 2 * (size_t)i) * cs_elems;
  }
  q.r_trial = static_cast<T*>(b->rhs);
  q.delta = delta;
  q.delta_trial = trial;
  q.scal = b->qn_scal;
  q.stride = kQnStride;
  q.e_cur = b->qn_e;
  q.e_trial = b->qn_e + b->n_cells;
  q.done = b->qn_done;
  // an FP32 state rounds the objective to ~1e-7 of itself: near convergence
  // the Armijo decrease falls below that, and without an allowance every
  // trial would be rejected
  q.e_tol = b->fp64 ? 0.0 : std::ldexp(1.0, -20);
  const bool want_energy = (b->flags & NPFEM_OPT_ENERGY) != 0;
  q.energy = want_energy ? b->energy : nullptr;
  q.energy_iters = n_iter;
  q.n_cells = b->n_cells;
  const T* w = b->per_cell ? static_cast<const T*>(b->weights_dev) : nullptr;
  NPFEM_TIMED(NPFEM_KERNEL_PREDICT,
              launch_predict<T>(slice_of<T>(c), pos, vel, forces, b->sumN, delta, cterm,
                                b->status, h, 0.0, st),
              "predict");
  LocalArgs<T> a;
  a.cs = slice_of<T>(c);
  a.pos = pos;
  a.sumN = b->sumN;
  a.cterm = cterm;
  a.weights = w;
  a.colmax = nullptr;
  a.status = b->status;
  a.h = h;
  a.m = c.mat.vertex_mass;
  a.mdelta = c.mat.vertex_mass / (h * h);
  a.max_vol_iter = b->max_vol_iter;
  set_volume_tolerances(a, c, b->fp64);
  // objective and r at q^0 (recorded as the energy of iterate 0)
  a.delta = delta;
  a.rhs = q.r_cur;
  a.energy = q.e_cur;
  NPFEM_TIMED(NPFEM_KERNEL_LOCAL, launch_local<T>(a, c.local_block, st), "local step");
  if (want_energy)
    HIP_TRY(hipMemcpyAsync(b->energy + c.cell0, q.e_cur + c.cell0, sizeof(double) * c.n_cells,
                           hipMemcpyDeviceToDevice, st),
            "energy record");
  for (int it = 0; it < n_iter; ++it) {
    const int count = std::min(it, q.hist);
    const int head = q.hist > 0 ? it % q.hist : 0;
    HIP_TRY(launch_qn_loop1<T>(slice_of<T>(c), q, count, head, st), "quasi-Newton first loop");
    GemmArgs g;
    g.A = c.op;
    g.A_frag = c.op_frag;
    g.B = q.v + c.elem0;
    g.C = q.z + c.elem0;
    g.D = nullptr;
    g.colscale = nullptr;
    g.Npad = c.Npad;
    g.ncols = 3 * c.n_cells;
    g.mode = EPI_SET;
    g.hm = c.hm_eff(h);
    g.beta = c.beta;
    NPFEM_TIMED(NPFEM_KERNEL_GLOBAL, launch_gemm(b->gemm_kind, c.gemm_tile, g, st), "global step");
    HIP_TRY(launch_qn_loop2<T>(slice_of<T>(c), q, count, head, st), "quasi-Newton second loop");
    for (int t = 0; t < b->qn_ls; ++t) {
      a.delta = trial;
      a.rhs = q.r_trial;
      a.energy = q.e_trial;
      a.skip = q.done;
      NPFEM_TIMED(NPFEM_KERNEL_LOCAL, launch_local<T>(a, c.local_block, st), "local step");
      HIP_TRY(launch_qn_accept<T>(slice_of<T>(c), q, head, t == b->qn_ls - 1 ? 1 : 0, it, st),
              "quasi-Newton line search");
    }
  }
  NPFEM_TIMED(NPFEM_KERNEL_UPDATE,
              launch_update<T>(slice_of<T>(c), pos, vel, b->sumN, delta, h, st),
              "update");
  return NPFEM_OK;
}

// One time step of every cell. With fork set (graph capture of a batch of
// several mesh classes) each class chain goes on a stream of its own that
// forks from and joins back into st, so the captured graph holds one
// parallel branch per class and small classes fill the CUs that a large
// class leaves idle; otherwise the chains run one after the other on st.
template <typename T>
int enqueue_step(npfem_batch_s* b, T* pos, T* vel, const T* forces, double h, int n_iter,
                 hipStream_t st, T* const* dslots = nullptr, bool fork = false) {
  if ((b->flags & NPFEM_OPT_KERNEL_TIMING) && b->ev_used > 60000)
    HIP_TRY(b->ev_harvest(), "kernel timing");
  int active = 0;
  for (auto& c : b->cls) active += c.n_cells > 0;
  if (!fork || active < 2) {
    for (auto& c : b->cls) {
      if (c.n_cells == 0) continue;
      const int rc = enqueue_class_step<T>(b, c, pos, vel, forces, h, n_iter, st, dslots);
      if (rc) return rc;
    }
    return NPFEM_OK;
  }
  int rc = b->ensure_branches();
  if (rc) return rc;
  HIP_TRY(hipEventRecord(b->br_fork, st), "fork event");
  for (size_t k = 0; k < b->cls.size(); ++k) {
    ClassState& c = b->cls[k];
    if (c.n_cells == 0) continue;
    hipStream_t s = b->br_stream[k];
    HIP_TRY(hipStreamWaitEvent(s, b->br_fork, 0), "fork wait");
    rc = enqueue_class_step<T>(b, c, pos, vel, forces, h, n_iter, s, dslots);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(b->br_join[k], s), "join event");
    HIP_TRY(hipStreamWaitEvent(st, b->br_join[k], 0), "join wait");
  }
  return NPFEM_OK;
}

int enqueue_any(npfem_batch_s* b, const void* forces, double h, int n_iter, hipStream_t st,
                bool fork = false) {
  if (b->fp64)
    return enqueue_step<double>(b, static_cast<double*>(b->pos), static_cast<double*>(b->vel),
                                static_cast<const double*>(forces), h, n_iter, st, nullptr, fork);
  return enqueue_step<float>(b, static_cast<float*>(b->pos), static_cast<float*>(b->vel),
                             static_cast<const float*>(forces), h, n_iter, st, nullptr, fork);
}

int prepare_kernels(npfem_batch_s* b) {
  for (auto& c : b->cls) {
    if (c.n_cells == 0) continue;
    hipError_t e = b->fp64 ? local_prepare<double>(slice_of<double>(c).cv, c.local_block)
                           : local_prepare<float>(slice_of<float>(c).cv, c.local_block);
    if (e != hipSuccess) return hip_fail(e, "local step attributes");
    e = gemm_prepare(b->gemm_kind, c.gemm_tile, c.Npad);
    if (e != hipSuccess) return hip_fail(e, "global step attributes");
  }
  return NPFEM_OK;
}

// Drops the captured step and run graphs (their kernels' arguments or the
// work they enqueue changed).
void drop_graphs(npfem_batch_s* b) {
  if (b->graph) {
    hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  if (b->run_graph) {
    hipGraphExecDestroy(b->run_graph);
    b->run_graph = nullptr;
  }
}

// Captures n_steps consecutive steps (each with its branch per class) as one
// graph: a run replays as a single launch.
int capture_run_graph(npfem_batch_s* b, const void* forces, double h, int n_iter, int n_steps) {
  if (b->run_graph) {
    hipGraphExecDestroy(b->run_graph);
    b->run_graph = nullptr;
  }
  int rc = prepare_kernels(b);
  if (rc) return rc;
  HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  for (int i = 0; i < n_steps && !rc; ++i) rc = enqueue_any(b, forces, h, n_iter, b->cap_stream, true);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (rc) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  e = hipGraphInstantiate(&b->run_graph, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->run_graph = nullptr;
    return hip_fail(e, "graph instantiate");
  }
  b->run_forces = forces;
  b->run_iters = n_iter;
  b->run_steps = n_steps;
  return NPFEM_OK;
}

int capture_graph(npfem_batch_s* b, const void* forces, double h, int n_iter) {
  if (b->graph) {
    hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  int rc = prepare_kernels(b);
  if (rc) return rc;
  HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  rc = enqueue_any(b, forces, h, n_iter, b->cap_stream, true);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (rc) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->graph = nullptr;
    return hip_fail(e, "graph instantiate");
  }
  b->graph_forces = forces;
  b->graph_iters = n_iter;
  return NPFEM_OK;
}

int default_local_block(int N) {
  if (N <= 256) return 128;
  if (N <= 1536) return 256;
  return 512;
}

// Autotuner: times every GEMM tile shape and every local-step workgroup size
// for each class on the batch's own buffers and keeps the fastest. It runs
// before the first predict, which overwrites everything the trials write;
// positions and velocities are only read.
template <typename T>
int autotune(npfem_batch_s* b, double h) {
  hipStream_t st = b->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0), "autotune events");
  HIP_TRY(hipEventCreate(&e1), "autotune events");
  // best of three rounds of three launches, after one warm-up launch (that
  // also checks that the candidate launches at all)
  auto timed = [&](auto&& launch, float* ms) -> hipError_t {
    hipError_t e = launch();
    if (e != hipSuccess) return e;
    *ms = 1e30f;
    for (int r = 0; r < 3; ++r) {
      if ((e = hipEventRecord(e0, st)) != hipSuccess) return e;
      for (int i = 0; i < 3; ++i)
        if ((e = launch()) != hipSuccess) return e;
      if ((e = hipEventRecord(e1, st)) != hipSuccess) return e;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
      float t = 0.f;
      if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return e;
      *ms = std::min(*ms, t);
    }
    return hipSuccess;
  };
  int rc = NPFEM_OK;
  for (auto& c : b->cls) {
    if (c.n_cells == 0) continue;
    GemmArgs g;
    g.A = c.op;
    g.A_frag = c.op_frag;
    g.B = static_cast<T*>(b->rhs) + c.elem0;
    g.C = static_cast<T*>(b->delta) + c.elem0;
    // (the step's solve adds the previous iterate; the other iterate buffer
    // stands in for it, so that repeated trials do not accumulate)
    g.D = static_cast<T*>(b->delta2) + c.elem0;
    g.colscale = nullptr;
    g.Npad = c.Npad;
    g.ncols = 3 * c.n_cells;
    g.mode = b->gemm_kind >= 2 ? EPI_SPLIT_SET : EPI_SET;
    g.hm = c.hm_eff(h);
    g.beta = c.beta;
    float best = 1e30f;
    for (int tile = 0; tile < gemm_num_tiles(b->gemm_kind); ++tile) {
      float ms = 0.f;
      if (gemm_prepare(b->gemm_kind, tile, c.Npad) != hipSuccess) continue;
      if (timed([&]() { return launch_gemm(b->gemm_kind, tile, g, st); }, &ms) == hipSuccess &&
          ms < best) {
        best = ms;
        c.gemm_tile = tile;
      }
    }
    LocalArgs<T> a;
    a.cs = slice_of<T>(c);
    a.pos = static_cast<const T*>(b->pos);
    a.sumN = b->sumN;
    a.delta = static_cast<const T*>(b->delta);
    a.cterm = static_cast<const T*>(b->cterm);
    a.rhs = static_cast<T*>(b->rhs);
    a.weights = b->per_cell ? static_cast<const T*>(b->weights_dev) : nullptr;
    a.energy = nullptr;
    a.colmax = nullptr;
    a.status = b->status;
    a.h = h;
    a.m = c.mat.vertex_mass;
    a.mdelta = c.mat.vertex_mass * c.mass_scale(h) / (h * h);
    a.max_vol_iter = b->max_vol_iter;
    set_volume_tolerances(a, c, b->fp64);
    best = 1e30f;
    // (1024 threads is left to set_config: it wins for a large mesh alone,
    // but its 16-wave workgroups wait longer for a free CU beside other
    // classes' branches, and the trials here time each class alone)
    for (int block : {128, 256, 512}) {
      if (local_prepare<T>(a.cs.cv, block) != hipSuccess) continue;
      float ms = 0.f;
      if (timed([&]() { return launch_local<T>(a, block, st); }, &ms) == hipSuccess && ms < best) {
        best = ms;
        c.local_block = block;
      }
    }
    hipGetLastError();  // clear launch-configuration errors of rejected candidates
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  HIP_TRY(hipStreamSynchronize(st), "autotune");
  return rc;
}

int grow(void** p, size_t* have, size_t need, const char* what) {
  if (*have >= need && *p) return NPFEM_OK;
  if (*p) hipFree(*p);
  *p = nullptr;
  *have = 0;
  hipError_t e = hipMalloc(p, std::max<size_t>(need, 16));
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_fail(e, what);
  }
  *have = need;
  return NPFEM_OK;
}

// Reverse of the last rollout (see npfem_rollout_adjoint). Segment by
// segment, backwards: recompute the segment from its checkpoint recording x_n
// and every PD iterate, then reverse its steps and iterations.
template <typename T>
int adjoint_impl(npfem_batch_s* b, const void* dL_dx, const void* dL_dv, void* dL_dw, void* dL_df,
                 void* dL_dx0, void* dL_dv0) {
  hipStream_t st = b->stream;
  const double h = b->ro_dt;
  const int K = b->ro_iter, ce = b->ro_every, S = b->ro_steps;
  const int n_seg = (S + ce - 1) / ce;
  const size_t sv = 3 * (size_t)b->sumN, cols = (size_t)b->total_elems;
  const size_t per_step = sv + (size_t)(K + 1) * cols;
  int rc;
  if ((rc = grow(&b->tape, &b->tape_bytes, sizeof(T) * per_step * ce, "adjoint tape"))) return rc;
  const size_t wbytes = sizeof(double) * 4 * (size_t)b->n_cells;
  if ((rc = grow(&b->adj_work, &b->adj_work_bytes, sizeof(T) * (4 * sv + 4 * cols) + wbytes + 256,
                 "adjoint workspace")))
    return rc;
  double* wbar = static_cast<double*>(b->adj_work);
  T* xs = reinterpret_cast<T*>(reinterpret_cast<char*>(b->adj_work) + ((wbytes + 255) / 256) * 256);
  T* vs = xs + sv;
  T* xbar = vs + sv;
  T* vbar = xbar + sv;
  T* lam = vbar + sv;
  T* gbar = lam + cols;
  T* sbar = gbar + cols;
  T* sgbar = sbar + cols;  // s gbar (the FP32-state solve, enqueue_solve)
  T* tape = static_cast<T*>(b->tape);
  T* ckpt = static_cast<T*>(b->ckpt);
  T* fbar = static_cast<T*>(dL_df);
  const T* forces = static_cast<const T*>(b->ro_forces);
  const T* w = b->per_cell ? static_cast<const T*>(b->weights_dev) : nullptr;

  for (auto& c : b->cls) {
    hipError_t e = local_prepare<T>(slice_of<T>(c).cv, c.local_block);
    if (e == hipSuccess) e = adjoint_prepare<T>(slice_of<T>(c).cv);
    if (e == hipSuccess) e = gemm_prepare(b->gemm_kind, c.gemm_tile, c.Npad);
    if (e != hipSuccess) return hip_fail(e, "adjoint kernel attributes");
  }
  HIP_TRY(hipMemcpyAsync(xbar, dL_dx, sizeof(T) * sv, hipMemcpyDeviceToDevice, st), "adjoint");
  if (dL_dv)
    HIP_TRY(hipMemcpyAsync(vbar, dL_dv, sizeof(T) * sv, hipMemcpyDeviceToDevice, st), "adjoint");
  else
    HIP_TRY(hipMemsetAsync(vbar, 0, sizeof(T) * sv, st), "adjoint");
  HIP_TRY(hipMemsetAsync(wbar, 0, wbytes, st), "adjoint");
  if (fbar) HIP_TRY(hipMemsetAsync(fbar, 0, sizeof(T) * sv, st), "adjoint");

  std::vector<T*> slots(K + 1);
  for (int seg = n_seg - 1; seg >= 0; --seg) {
    const int s0 = seg * ce, ns = std::min(ce, S - s0);
    HIP_TRY(hipMemcpyAsync(xs, ckpt + 2 * (size_t)seg * sv, sizeof(T) * sv,
                           hipMemcpyDeviceToDevice, st), "recompute");
    HIP_TRY(hipMemcpyAsync(vs, ckpt + (2 * (size_t)seg + 1) * sv, sizeof(T) * sv,
                           hipMemcpyDeviceToDevice, st), "recompute");
    for (int j = 0; j < ns; ++j) {
      T* tj = tape + (size_t)j * per_step;
      HIP_TRY(hipMemcpyAsync(tj, xs, sizeof(T) * sv, hipMemcpyDeviceToDevice, st), "recompute");
      for (int k = 0; k <= K; ++k) slots[k] = tj + sv + (size_t)k * cols;
      if ((rc = enqueue_step<T>(b, xs, vs, forces, h, K, st, slots.data()))) return rc;
    }
    for (int j = ns - 1; j >= 0; --j) {
      T* tj = tape + (size_t)j * per_step;
      for (int k = 0; k <= K; ++k) slots[k] = tj + sv + (size_t)k * cols;
      for (auto& c : b->cls)
        HIP_TRY(launch_adj_begin<T>(slice_of<T>(c), xbar, vbar, b->sumN, gbar, sbar, h, st),
                "adjoint step");
      for (int k = K - 1; k >= 0; --k) {
        for (auto& c : b->cls) {
          if (c.n_cells == 0) continue;
          if ((rc = enqueue_solve<T>(b, c, gbar, lam, nullptr, h, st, false,
                                     b->fp64 ? nullptr : sgbar)))
            return rc;
          AdjArgs<T> a;
          a.cs = slice_of<T>(c);
          a.xn = tj;
          a.sumN = b->sumN;
          a.delta_k = slots[k];
          a.delta_k1 = slots[k + 1];
          a.lam = lam;
          a.gbar = gbar;
          a.sbar = sbar;
          a.wbar = wbar;
          a.weights = w;
          a.status = b->status;
          a.h = h;
          a.m = c.mat.vertex_mass;
          a.max_vol_iter = b->max_vol_iter;
          LocalArgs<T> tol;
          set_volume_tolerances(tol, c, b->fp64);
          a.vol_tol = tol.vol_tol;
          a.vol_abs = tol.vol_abs;
          HIP_TRY(launch_adjoint_local<T>(a, st), "adjoint iteration");
        }
      }
      for (auto& c : b->cls)
        HIP_TRY(launch_adj_end<T>(slice_of<T>(c), xbar, vbar, b->sumN, gbar, sbar, fbar, h, st),
                "adjoint step");
    }
  }
  if (dL_dw)
    HIP_TRY(hipMemcpyAsync(dL_dw, wbar, wbytes, hipMemcpyDeviceToDevice, st), "adjoint outputs");
  if (dL_dx0)
    HIP_TRY(hipMemcpyAsync(dL_dx0, xbar, sizeof(T) * sv, hipMemcpyDeviceToDevice, st),
            "adjoint outputs");
  if (dL_dv0)
    HIP_TRY(hipMemcpyAsync(dL_dv0, vbar, sizeof(T) * sv, hipMemcpyDeviceToDevice, st),
            "adjoint outputs");
  HIP_TRY(hipStreamSynchronize(st), "adjoint");
  return NPFEM_OK;
}

}  // namespace

extern "C" {

const char* npfem_last_error(void) { return g_err.c_str(); }

int npfem_create_mesh(const double* rest_xyz, int32_t n_verts, const int32_t* tris,
                      int32_t n_tris, const npfem_material* mat, npfem_mesh* out) {
  g_err.clear();
  if (!out) return fail(NPFEM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!rest_xyz || !tris || !mat) return fail(NPFEM_ERR_INVALID_ARG, "NULL mesh argument");
  const double wv[5] = {mat->w_stretch, mat->w_area, mat->w_bend, mat->w_volume, mat->vertex_mass};
  for (int i = 0; i < 5; ++i) {
    if (!std::isfinite(wv[i]) || wv[i] < 0.0)
      return fail(NPFEM_ERR_INVALID_ARG, "material entries must be finite and non-negative");
  }
  if (!(mat->vertex_mass > 0.0)) return fail(NPFEM_ERR_INVALID_ARG, "vertex_mass must be > 0");
  std::unique_ptr<npfem_mesh_s> m(new (std::nothrow) npfem_mesh_s);
  if (!m) return fail(NPFEM_ERR_OOM, "host allocation");
  std::string err;
  const int rc = build_mesh_ops(rest_xyz, n_verts, tris, n_tris, m->ops, err);
  if (rc) return fail(rc, "%s", err.c_str());
  m->mat = *mat;
  *out = m.release();
  return NPFEM_OK;
}

int npfem_mesh_info(npfem_mesh m, int32_t* n_verts, int32_t* n_tris, int32_t* n_hinges,
                    double* rest_volume) {
  if (!m || m->tag != kMeshTag) return fail(NPFEM_ERR_INVALID_ARG, "not a mesh handle");
  if (n_verts) *n_verts = m->ops.N;
  if (n_tris) *n_tris = m->ops.F;
  if (n_hinges) *n_hinges = m->ops.E;
  if (rest_volume) *rest_volume = m->ops.vol_rest;
  return NPFEM_OK;
}

int npfem_mesh_system_matrix(npfem_mesh m, const double* weights4, double dt, double* A_out) {
  if (!m || m->tag != kMeshTag) return fail(NPFEM_ERR_INVALID_ARG, "not a mesh handle");
  if (!A_out) return fail(NPFEM_ERR_INVALID_ARG, "A_out is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(NPFEM_ERR_INVALID_ARG, "dt must be > 0");
  const double w0[4] = {m->mat.w_stretch, m->mat.w_area, m->mat.w_bend, m->mat.w_volume};
  dense_system_matrix(m->ops, weights4 ? weights4 : w0, m->mat.vertex_mass, dt, A_out, m->ops.N);
  return NPFEM_OK;
}

int npfem_create_batch(const npfem_mesh* meshes, int32_t n_meshes, const int32_t* cell_mesh,
                       int32_t n_cells, const double* cell_weights, void* pos, void* vel,
                       const npfem_options* opt, npfem_batch* out) {
  g_err.clear();
  if (!out) return fail(NPFEM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!meshes || n_meshes < 1 || !cell_mesh || n_cells < 1)
    return fail(NPFEM_ERR_INVALID_ARG, "need at least one mesh and one cell");
  if (!pos || !vel) return fail(NPFEM_ERR_INVALID_ARG, "pos and vel must be device pointers");
  for (int i = 0; i < n_meshes; ++i)
    if (!meshes[i] || meshes[i]->tag != kMeshTag)
      return fail(NPFEM_ERR_INVALID_ARG, "meshes[%d] is not a mesh handle", i);
  for (int c = 0; c < n_cells; ++c) {
    if (cell_mesh[c] < 0 || cell_mesh[c] >= n_meshes)
      return fail(NPFEM_ERR_INVALID_ARG, "cell_mesh[%d] out of range", c);
    if (c > 0 && cell_mesh[c] < cell_mesh[c - 1])
      return fail(NPFEM_ERR_INVALID_ARG, "cell_mesh must be non-decreasing (class-major order)");
  }
  npfem_options o{};
  o.precision = NPFEM_FP32;
  o.n_refine = -1;
  if (opt) o = *opt;
  const int kind = precision_of_gemm(o.precision);
  if (kind < 0) return fail(NPFEM_ERR_INVALID_ARG, "unknown precision %d", o.precision);
  if (o.n_refine < -1 || o.n_refine > 100) return fail(NPFEM_ERR_INVALID_ARG, "n_refine out of range");
  if (o.max_vol_iter < 0 || o.max_vol_iter > 200)
    return fail(NPFEM_ERR_INVALID_ARG, "max_vol_iter out of range");
  if (cell_weights) {
    for (long long i = 0; i < 4LL * n_cells; ++i)
      if (!std::isfinite(cell_weights[i]) || cell_weights[i] < 0.0)
        return fail(NPFEM_ERR_INVALID_ARG, "cell_weights must be finite and non-negative");
  }

  std::unique_ptr<npfem_batch_s> b(new (std::nothrow) npfem_batch_s);
  if (!b) return fail(NPFEM_ERR_OOM, "host allocation");
  HIP_TRY(hipGetDevice(&b->device), "hipGetDevice");
  b->precision = o.precision;
  b->gemm_kind = kind;
  b->fp64 = (o.precision == NPFEM_FP64);
  b->stream = static_cast<hipStream_t>(o.stream);
  b->flags = o.flags;
  b->n_refine_opt = o.n_refine;
  b->max_vol_iter = o.max_vol_iter > 0 ? o.max_vol_iter : (b->fp64 ? 12 : 6);
  b->n_cells = n_cells;
  b->pos = pos;
  b->vel = vel;
  HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "capture stream");

  const size_t tsz = b->fp64 ? sizeof(double) : sizeof(float);
  // classes in mesh order; cells are class-major
  b->cls.resize(n_meshes);
  long long col = 0, elem = 0, vert = 0;
  int c0 = 0;
  for (int k = 0; k < n_meshes; ++k) {
    ClassState& c = b->cls[k];
    c.ops = meshes[k]->ops;
    c.mat = meshes[k]->mat;
    c.N = c.ops.N;
    c.Npad = (c.N + 15) / 16 * 16;
    c.F = c.ops.F;
    c.E = c.ops.E;
    int n = 0;
    while (c0 + n < n_cells && cell_mesh[c0 + n] == k) ++n;
    c.n_cells = n;
    c.cell0 = c0;
    c.col0 = col;
    c.elem0 = elem;
    c.vert0 = vert;
    c.local_block = default_local_block(c.N);
    // default product (the autotuner may pick another): FP32 classes of 512
    // to 853 rows (48 columns fit the LDS) take the column-stationary kernel
    // (it splits the rows over several workgroups when the columns are few),
    // else 128 x 128 tiles from 1024 columns on, 64 x 64 below
    const bool rs_fp32 = b->gemm_kind == 0 && c.Npad % 16 == 0 && c.Npad >= 512 &&
                         (size_t)48 * c.Npad * 4 <= 160 * 1024;
    c.gemm_tile = (3LL * n >= 1024) ? (rs_fp32 ? gemm_num_tiles(0) - 1 : 3) : 0;
    if (n > 0 && c.N > kLocalMaxBlock * kLocalMaxVertsPerThread)
      return fail(NPFEM_ERR_INVALID_ARG,
                  "a batch takes meshes of at most %d vertices (the local step holds at most %d "
                  "vertices per thread of a %d-thread workgroup); this class has %d",
                  kLocalMaxBlock * kLocalMaxVertsPerThread, kLocalMaxVertsPerThread,
                  kLocalMaxBlock, c.N);
    if (b->fp64 && n > 0) {
      // the FP64 local step keeps q and the volume iterate as 32-byte
      // records of N + 1 vertices each in LDS
      ClassView<double> cv{};
      cv.N = c.N;
      cv.F = c.F;
      cv.E = c.E;
      const size_t need = local_smem_bytes<double>(cv, c.local_block);
      if (need > 160 * 1024)
        return fail(NPFEM_ERR_INVALID_ARG,
                    "an FP64 batch takes meshes of at most 2550 vertices (the local step of a "
                    "%d-vertex class needs %zu bytes of LDS, 163840 available)",
                    c.N, need);
    }
    col += 3LL * n;
    elem += 3LL * n * c.Npad;
    vert += (long long)n * c.N;
    c0 += n;
    int rc = b->fp64 ? upload_class<double>(c) : upload_class<float>(c);
    if (rc) return rc;
  }
  b->sumN = vert;
  b->total_cols = col;
  b->total_elems = elem;

  b->cell_class.assign(cell_mesh, cell_mesh + n_cells);
  int rc;
  if ((rc = apply_weights(b.get(), cell_weights))) return rc;
  const size_t colbytes = tsz * (size_t)b->total_elems;
  if ((rc = dalloc(b.get(), &b->delta, colbytes, "delta"))) return rc;
  if ((rc = dalloc(b.get(), &b->delta2, colbytes, "delta2"))) return rc;
  if ((rc = dalloc(b.get(), &b->cterm, colbytes, "cterm"))) return rc;
  if ((rc = dalloc(b.get(), &b->rhs, colbytes, "rhs"))) return rc;
  if ((rc = dalloc(b.get(), &b->res, colbytes, "res"))) return rc;
  void* p;
  if ((rc = dalloc(b.get(), &p, sizeof(float) * (size_t)b->total_cols, "colmax"))) return rc;
  b->colmax = static_cast<float*>(p);
  if ((rc = dalloc(b.get(), &p, sizeof(float) * (size_t)b->total_cols, "colmax_res"))) return rc;
  b->colmax_res = static_cast<float*>(p);
  if ((rc = dalloc(b.get(), &p, 64, "status"))) return rc;
  b->status = static_cast<int*>(p);
  if ((rc = dalloc(b.get(), &p, sizeof(double) * (size_t)n_cells, "volume"))) return rc;
  b->volume_buf = static_cast<double*>(p);
  HIP_TRY(hipMemset(b->delta, 0, colbytes), "memset");
  HIP_TRY(hipMemset(b->delta2, 0, colbytes), "memset");
  HIP_TRY(hipMemset(b->rhs, 0, colbytes), "memset");
  HIP_TRY(hipMemset(b->res, 0, colbytes), "memset");
  HIP_TRY(hipMemset(b->cterm, 0, colbytes), "memset");
  HIP_TRY(hipMemset(b->status, 0, 64), "memset");
  HIP_TRY(hipDeviceSynchronize(), "create_batch");
  *out = b.release();
  return NPFEM_OK;
}

// Whole-step trial of the 1024-thread local step for large meshes (FP32
// state, several mesh classes). The autotuner times each class alone, but a
// 1024-thread workgroup's cost depends on the other classes' branches that
// run beside it (it waits longer for a CU with 16 free wave slots), so this
// choice is made on whole steps with the class branches forked as in the
// captured graph: launched eagerly from the state saved here, which is
// restored after every trial.
static int joint_tune(npfem_batch_s* b, const void* forces, double h, int n_iter) {
  if (b->fp64 || b->qn_hist >= 0 || (b->flags & NPFEM_OPT_KERNEL_TIMING)) return NPFEM_OK;
  int active = 0;
  std::vector<int> cand;
  for (size_t k = 0; k < b->cls.size(); ++k) {
    const ClassState& c = b->cls[k];
    if (c.n_cells == 0) continue;
    ++active;
    if (c.N > 1536 && c.N <= 3072 && c.local_block != 1024 &&
        local_prepare<float>(slice_of<float>(c).cv, 1024) == hipSuccess)
      cand.push_back((int)k);
  }
  hipGetLastError();
  if (active < 2 || cand.empty()) return NPFEM_OK;
  hipStream_t st = b->stream;
  const size_t bytes = sizeof(float) * 3 * (size_t)b->sumN;
  void* sx = nullptr;
  void* sv = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    if (sx) hipFree(sx);
    if (sv) hipFree(sv);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  };
  hipError_t e = hipMalloc(&sx, bytes);
  if (e == hipSuccess) e = hipMalloc(&sv, bytes);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemcpyAsync(sx, b->pos, bytes, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(sv, b->vel, bytes, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) {
    release();
    return hip_fail(e, "joint tuning");
  }
  auto restore = [&]() {
    hipError_t r = hipMemcpyAsync(b->pos, sx, bytes, hipMemcpyDeviceToDevice, st);
    if (r == hipSuccess) r = hipMemcpyAsync(b->vel, sv, bytes, hipMemcpyDeviceToDevice, st);
    return r;
  };
  // one warm-up step, then the best of three timed steps
  auto step_ms = [&](float* best) -> int {
    int rc = prepare_kernels(b);
    if (!rc) rc = enqueue_any(b, forces, h, n_iter, st, true);
    if (rc) return rc;
    *best = 1e30f;
    for (int r = 0; r < 3; ++r) {
      hipError_t x = restore();
      if (x == hipSuccess) x = hipEventRecord(e0, st);
      if (x != hipSuccess) return hip_fail(x, "joint tuning");
      if ((rc = enqueue_any(b, forces, h, n_iter, st, true))) return rc;
      float ms = 0.f;
      x = hipEventRecord(e1, st);
      if (x == hipSuccess) x = hipEventSynchronize(e1);
      if (x == hipSuccess) x = hipEventElapsedTime(&ms, e0, e1);
      if (x != hipSuccess) return hip_fail(x, "joint tuning");
      *best = std::min(*best, ms);
    }
    return NPFEM_OK;
  };
  int rc = NPFEM_OK;
  for (int k : cand) {
    ClassState& c = b->cls[k];
    const int keep = c.local_block;
    float t_keep = 0.f, t_wide = 0.f;
    if ((rc = step_ms(&t_keep))) break;
    c.local_block = 1024;
    if ((rc = step_ms(&t_wide))) break;
    if (!(t_wide < t_keep)) c.local_block = keep;
  }
  e = restore();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  release();
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "joint tuning");
  return prepare_kernels(b);
}

// Argument checks, refactorisation on a new dt and the energy record's
// size, shared by npfem_step and npfem_run (b checked, device current).
static int step_prepare(npfem_batch b, const void* ext_forces, double dt, int32_t n_iter) {
  if (!ext_forces) return fail(NPFEM_ERR_INVALID_ARG, "ext_forces is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(NPFEM_ERR_INVALID_ARG, "dt must be finite and > 0");
  if (n_iter < 1 || n_iter > 1000) return fail(NPFEM_ERR_INVALID_ARG, "n_iter must be in [1, 1000]");
  if (b->qn_hist >= 0)
    for (const auto& c : b->cls)
      if (c.alpha != 0.0 || c.beta_d != 0.0 || c.wc != 0.0)
        return fail(NPFEM_ERR_INVALID_ARG,
                    "the quasi-Newton step covers the undamped, contact-free objective");
  int rc;
  bool tuned_now = false;
  if (dt != b->dt) {
    HIP_TRY(hipStreamSynchronize(b->stream), "sync before refactorisation");
    if ((rc = factorise(b, dt))) return rc;
    if ((b->flags & NPFEM_OPT_AUTOTUNE) && !b->tuned) {
      if ((rc = b->fp64 ? autotune<double>(b, dt) : autotune<float>(b, dt))) return rc;
      b->tuned = true;
      tuned_now = true;
    }
    drop_graphs(b);
  }
  if ((b->flags & NPFEM_OPT_ENERGY) && n_iter > b->energy_cap) {
    HIP_TRY(hipStreamSynchronize(b->stream), "sync before energy buffer");
    void* p = nullptr;
    HIP_TRY(hipMalloc(&p, sizeof(double) * (size_t)n_iter * b->n_cells), "energy buffer");
    if (b->energy) {
      auto it = std::find(b->allocs.begin(), b->allocs.end(), (void*)b->energy);
      if (it != b->allocs.end()) b->allocs.erase(it);
      hipFree(b->energy);
    }
    b->allocs.push_back(p);
    b->energy = static_cast<double*>(p);
    b->energy_cap = n_iter;
    drop_graphs(b);
  }
  // (after the energy record is sized: the trial steps write it)
  if (tuned_now && (rc = joint_tune(b, ext_forces, dt, n_iter))) return rc;
  return NPFEM_OK;
}

int npfem_step(npfem_batch b, const void* ext_forces, double dt, int32_t n_iter) {
  g_err.clear();
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  DeviceGuard guard(b->device);
  int rc;
  if ((rc = step_prepare(b, ext_forces, dt, n_iter))) return rc;
  if (b->flags & (NPFEM_OPT_NO_GRAPH | NPFEM_OPT_KERNEL_TIMING)) {
    if ((rc = prepare_kernels(b))) return rc;
    if ((rc = enqueue_any(b, ext_forces, dt, n_iter, b->stream))) return rc;
  } else {
    if (!b->graph || b->graph_forces != ext_forces || b->graph_iters != n_iter) {
      if ((rc = capture_graph(b, ext_forces, dt, n_iter))) return rc;
    }
    HIP_TRY(hipGraphLaunch(b->graph, b->stream), "graph launch");
  }
  b->energy_iters = n_iter;
  if (b->flags & NPFEM_OPT_SYNC_CHECK) return npfem_sync_status(b);
  return NPFEM_OK;
}

int npfem_run(npfem_batch b, const void* ext_forces, double dt, int32_t n_iter, int32_t n_steps) {
  g_err.clear();
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (n_steps < 1 || n_steps > 1000) return fail(NPFEM_ERR_INVALID_ARG, "n_steps must be in [1, 1000]");
  DeviceGuard guard(b->device);
  int rc;
  if ((rc = step_prepare(b, ext_forces, dt, n_iter))) return rc;
  if (b->flags & (NPFEM_OPT_NO_GRAPH | NPFEM_OPT_KERNEL_TIMING)) {
    if ((rc = prepare_kernels(b))) return rc;
    for (int i = 0; i < n_steps; ++i)
      if ((rc = enqueue_any(b, ext_forces, dt, n_iter, b->stream))) return rc;
  } else {
    if (!b->run_graph || b->run_forces != ext_forces || b->run_iters != n_iter ||
        b->run_steps != n_steps) {
      if ((rc = capture_run_graph(b, ext_forces, dt, n_iter, n_steps))) return rc;
    }
    HIP_TRY(hipGraphLaunch(b->run_graph, b->stream), "graph launch");
  }
  b->energy_iters = n_iter;
  if (b->flags & NPFEM_OPT_SYNC_CHECK) return npfem_sync_status(b);
  return NPFEM_OK;
}

int npfem_set_weights(npfem_batch b, const double* cell_weights) {
  g_err.clear();
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (cell_weights) {
    for (long long i = 0; i < 4LL * b->n_cells; ++i)
      if (!std::isfinite(cell_weights[i]) || cell_weights[i] < 0.0)
        return fail(NPFEM_ERR_INVALID_ARG, "cell_weights must be finite and non-negative");
  }
  DeviceGuard guard(b->device);
  HIP_TRY(hipStreamSynchronize(b->stream), "sync before weight update");
  const int rc = apply_weights(b, cell_weights);
  drop_graphs(b);
  b->ro_valid = false;
  return rc;
}

int npfem_set_damping(npfem_batch b, int32_t cls, double alpha, double beta) {
  g_err.clear();
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (cls < -1 || cls >= (int)b->cls.size())
    return fail(NPFEM_ERR_INVALID_ARG, "class index out of range");
  if (!std::isfinite(alpha) || !std::isfinite(beta) || alpha < 0.0 || beta < 0.0)
    return fail(NPFEM_ERR_INVALID_ARG, "damping coefficients must be finite and non-negative");
  DeviceGuard guard(b->device);
  HIP_TRY(hipStreamSynchronize(b->stream), "sync before damping update");
  bool any_beta = false;
  for (int k = 0; k < (int)b->cls.size(); ++k) {
    if (cls < 0 || k == cls) {
      b->cls[k].alpha = alpha;
      b->cls[k].beta_d = beta;
    }
    any_beta = any_beta || b->cls[k].beta_d != 0.0;
  }
  if (any_beta && !b->damp) {
    const size_t tsz = b->fp64 ? sizeof(double) : sizeof(float);
    const int rc = dalloc(b, &b->damp, tsz * (size_t)b->total_elems, "damping buffer");
    if (rc) return rc;
    HIP_TRY(hipMemset(b->damp, 0, tsz * (size_t)b->total_elems), "memset");
  }
  // the operator depends on the damping: refactor and re-capture at the next step
  b->dt = 0.0;
  drop_graphs(b);
  b->ro_valid = false;
  return NPFEM_OK;
}

int npfem_set_quasi_newton(npfem_batch b, int32_t history, int32_t line_search) {
  g_err.clear();
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (history > kQnMaxHist || line_search < 1 || line_search > 8)
    return fail(NPFEM_ERR_INVALID_ARG, "history must be <= 16 and line_search in [1, 8]");
  if (history >= 0 && b->gemm_kind >= 2)
    return fail(NPFEM_ERR_INVALID_ARG, "the quasi-Newton step runs FP64 and FP32 batches");
  DeviceGuard guard(b->device);
  HIP_TRY(hipStreamSynchronize(b->stream), "sync before solver change");
  if (history >= 0) {
    const size_t tsz = b->fp64 ? sizeof(double) : sizeof(float);
    const size_t need = (4 + 2 * (size_t)history) * tsz * (size_t)b->total_elems;
    auto drop = [&](void* p) {
      if (!p) return;
      auto it = std::find(b->allocs.begin(), b->allocs.end(), p);
      if (it != b->allocs.end()) b->allocs.erase(it);
      hipFree(p);
    };
    if (history > b->qn_hist_cap || !b->qn_cols) {
      drop(b->qn_cols);
      b->qn_cols = nullptr;
      int rc = dalloc(b, &b->qn_cols, need, "quasi-Newton columns");
      if (rc) return rc;
      HIP_TRY(hipMemset(b->qn_cols, 0, need), "memset");
      b->qn_hist_cap = history;
    }
    if (!b->qn_scal) {
      void* p = nullptr;
      int rc = dalloc(b, &p, sizeof(double) * kQnStride * (size_t)b->n_cells, "quasi-Newton scalars");
      if (rc) return rc;
      b->qn_scal = static_cast<double*>(p);
      if ((rc = dalloc(b, &p, sizeof(double) * 2 * (size_t)b->n_cells, "quasi-Newton objective")))
        return rc;
      b->qn_e = static_cast<double*>(p);
      if ((rc = dalloc(b, &p, sizeof(int) * (size_t)b->n_cells, "quasi-Newton flags"))) return rc;
      b->qn_done = static_cast<int*>(p);
      HIP_TRY(hipMemset(b->qn_scal, 0, sizeof(double) * kQnStride * (size_t)b->n_cells), "memset");
    }
  }
  b->qn_hist = history < 0 ? -1 : history;
  b->qn_ls = line_search;
  drop_graphs(b);
  b->ro_valid = false;
  return NPFEM_OK;
}

int npfem_set_contacts(npfem_batch b, double weight, const void* points, const void* normals,
                       const int32_t* cell_offsets, int64_t n_points) {
  g_err.clear();
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (!std::isfinite(weight) || weight < 0.0)
    return fail(NPFEM_ERR_INVALID_ARG, "contact weight must be finite and non-negative");
  if (weight > 0.0 && (!points || !normals || !cell_offsets || n_points < 0))
    return fail(NPFEM_ERR_INVALID_ARG, "contact arrays are NULL or n_points < 0");
  DeviceGuard guard(b->device);
  HIP_TRY(hipStreamSynchronize(b->stream), "sync before contact update");
  bool refactor = false;
  for (auto& c : b->cls) {
    refactor = refactor || c.wc != weight;
    c.wc = weight;
  }
  b->ct_points = weight > 0.0 ? points : nullptr;
  b->ct_normals = weight > 0.0 ? normals : nullptr;
  b->ct_off = weight > 0.0 ? cell_offsets : nullptr;
  b->ct_np = weight > 0.0 ? n_points : 0;
  // the weight is in the operator (refactor); the arrays' addresses are in
  // the captured graph (re-capture)
  if (refactor) b->dt = 0.0;
  drop_graphs(b);
  b->ro_valid = false;
  return NPFEM_OK;
}

static int ibm_grid(const int32_t dims[3], double dx, const double origin[3], IbmGrid* g) {
  if (!dims || !origin) return fail(NPFEM_ERR_INVALID_ARG, "grid dims or origin is NULL");
  if (dims[0] < 4 || dims[1] < 4 || dims[2] < 4)
    return fail(NPFEM_ERR_INVALID_ARG, "grid must have at least 4 nodes per axis");
  if ((double)dims[0] * dims[1] * dims[2] > 2.0e9)
    return fail(NPFEM_ERR_INVALID_ARG, "grid too large (more than 2e9 nodes)");
  if (!(dx > 0.0) || !std::isfinite(dx) || !std::isfinite(origin[0]) ||
      !std::isfinite(origin[1]) || !std::isfinite(origin[2]))
    return fail(NPFEM_ERR_INVALID_ARG, "dx must be finite and > 0, the origin finite");
  *g = IbmGrid{dims[0], dims[1], dims[2], dx, origin[0], origin[1], origin[2]};
  return NPFEM_OK;
}

int npfem_ibm_interpolate(npfem_batch b, const double* cell_origins, const void* grid_u,
                          const int32_t dims[3], double dx, const double grid_origin[3],
                          void* out_u) {
  g_err.clear();
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (!cell_origins || !grid_u || !out_u) return fail(NPFEM_ERR_INVALID_ARG, "NULL array");
  IbmGrid g;
  int rc = ibm_grid(dims, dx, grid_origin, &g);
  if (rc) return rc;
  DeviceGuard guard(b->device);
  for (auto& c : b->cls) {
    hipError_t e =
        b->fp64 ? launch_ibm_interpolate<double>(slice_of<double>(c), (const double*)b->pos,
                                                 b->sumN, cell_origins, (const double*)grid_u, g,
                                                 (double*)out_u, b->stream)
                : launch_ibm_interpolate<float>(slice_of<float>(c), (const float*)b->pos,
                                                b->sumN, cell_origins, (const float*)grid_u, g,
                                                (float*)out_u, b->stream);
    if (e != hipSuccess) return hip_fail(e, "IBM interpolation");
  }
  return NPFEM_OK;
}

int npfem_ibm_spread(npfem_batch b, const double* cell_origins, const void* vertex_f,
                     const int32_t dims[3], double dx, const double grid_origin[3], void* grid_f) {
  g_err.clear();
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (!cell_origins || !vertex_f || !grid_f) return fail(NPFEM_ERR_INVALID_ARG, "NULL array");
  IbmGrid g;
  int rc = ibm_grid(dims, dx, grid_origin, &g);
  if (rc) return rc;
  DeviceGuard guard(b->device);
  const long long nodes = (long long)g.nx * g.ny * g.nz;
  if (nodes > b->ibm_cap) {
    HIP_TRY(hipStreamSynchronize(b->stream), "sync before IBM accumulators");
    if (b->ibm_acc) {
      auto it = std::find(b->allocs.begin(), b->allocs.end(), (void*)b->ibm_acc);
      if (it != b->allocs.end()) b->allocs.erase(it);
      hipFree(b->ibm_acc);
      b->ibm_acc = nullptr;
      b->ibm_cap = 0;
    }
    void* p = nullptr;
    if ((rc = dalloc(b, &p, sizeof(unsigned long long) * (size_t)(3 * nodes + 32), "IBM accumulators")))
      return rc;
    b->ibm_acc = static_cast<unsigned long long*>(p);
    b->ibm_cap = nodes;
  }
  unsigned long long* mx = b->ibm_acc;         // max |F| word (own 256-byte line)
  unsigned long long* acc = b->ibm_acc + 32;   // [3][nodes]
  HIP_TRY(launch_ibm_zero(b->ibm_acc, 3 * nodes + 32, b->stream), "IBM accumulators");
  const double n_total = (double)b->sumN;
  for (auto& c : b->cls) {
    hipError_t e = b->fp64 ? launch_ibm_maxabs<double>(slice_of<double>(c), (const double*)vertex_f,
                                                       b->sumN, mx, b->status, b->stream)
                           : launch_ibm_maxabs<float>(slice_of<float>(c), (const float*)vertex_f,
                                                      b->sumN, mx, b->status, b->stream);
    if (e != hipSuccess) return hip_fail(e, "IBM force scale");
  }
  for (auto& c : b->cls) {
    hipError_t e =
        b->fp64 ? launch_ibm_spread<double>(slice_of<double>(c), (const double*)b->pos, b->sumN,
                                            cell_origins, (const double*)vertex_f, g, mx, n_total,
                                            acc, b->stream)
                : launch_ibm_spread<float>(slice_of<float>(c), (const float*)b->pos, b->sumN,
                                           cell_origins, (const float*)vertex_f, g, mx, n_total,
                                           acc, b->stream);
    if (e != hipSuccess) return hip_fail(e, "IBM spreading");
  }
  hipError_t e = b->fp64 ? launch_ibm_convert<double>(acc, 3 * nodes, mx, n_total, dx,
                                                      (double*)grid_f, b->stream)
                         : launch_ibm_convert<float>(acc, 3 * nodes, mx, n_total, dx,
                                                     (float*)grid_f, b->stream);
  if (e != hipSuccess) return hip_fail(e, "IBM conversion");
  return NPFEM_OK;
}

int npfem_rollout(npfem_batch b, const void* ext_forces, double dt, int32_t n_iter,
                  int32_t n_steps, int32_t ckpt_every) {
  g_err.clear();
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (n_steps < 1 || ckpt_every < 1 || ckpt_every > n_steps)
    return fail(NPFEM_ERR_INVALID_ARG, "need n_steps >= 1 and 1 <= ckpt_every <= n_steps");
  if (b->qn_hist >= 0)
    return fail(NPFEM_ERR_INVALID_ARG, "the differentiable rollout runs the classic PD step");
  DeviceGuard guard(b->device);
  const size_t tsz = b->fp64 ? sizeof(double) : sizeof(float);
  const size_t sv = 3 * (size_t)b->sumN;
  const int n_seg = (n_steps + ckpt_every - 1) / ckpt_every;
  b->ro_valid = false;
  if (b->ckpt_bytes < tsz * 2 * sv * n_seg) HIP_TRY(hipStreamSynchronize(b->stream), "sync");
  int rc = grow(&b->ckpt, &b->ckpt_bytes, tsz * 2 * sv * n_seg, "checkpoints");
  if (rc) return rc;
  char* ck = static_cast<char*>(b->ckpt);
  for (int s = 0; s < n_steps; ++s) {
    if (s % ckpt_every == 0) {
      const size_t seg = s / ckpt_every;
      HIP_TRY(hipMemcpyAsync(ck + tsz * 2 * seg * sv, b->pos, tsz * sv, hipMemcpyDeviceToDevice,
                             b->stream), "checkpoint");
      HIP_TRY(hipMemcpyAsync(ck + tsz * (2 * seg + 1) * sv, b->vel, tsz * sv,
                             hipMemcpyDeviceToDevice, b->stream), "checkpoint");
    }
    if ((rc = npfem_step(b, ext_forces, dt, n_iter))) return rc;
  }
  b->ro_steps = n_steps;
  b->ro_iter = n_iter;
  b->ro_every = ckpt_every;
  b->ro_dt = dt;
  b->ro_forces = ext_forces;
  b->ro_valid = true;
  return NPFEM_OK;
}

int npfem_rollout_adjoint(npfem_batch b, const void* dL_dx, const void* dL_dv, void* dL_dw,
                          void* dL_df, void* dL_dx0, void* dL_dv0) {
  g_err.clear();
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (!dL_dx) return fail(NPFEM_ERR_INVALID_ARG, "dL_dx is NULL");
  if (!b->ro_valid || b->dt != b->ro_dt)
    return fail(NPFEM_ERR_INVALID_ARG,
                "no rollout to reverse (run npfem_rollout; weights and dt must not change)");
  if (b->gemm_kind == 3)
    return fail(NPFEM_ERR_INVALID_ARG, "the adjoint supports FP64, FP32 and BF16 batches");
  for (const auto& c : b->cls)
    if (c.alpha != 0.0 || c.beta_d != 0.0 || c.wc != 0.0)
      return fail(NPFEM_ERR_INVALID_ARG,
                  "the adjoint does not cover viscous damping or contact potentials");
  DeviceGuard guard(b->device);
  HIP_TRY(hipStreamSynchronize(b->stream), "sync before adjoint");
  const int rc = b->fp64 ? adjoint_impl<double>(b, dL_dx, dL_dv, dL_dw, dL_df, dL_dx0, dL_dv0)
                         : adjoint_impl<float>(b, dL_dx, dL_dv, dL_dw, dL_df, dL_dx0, dL_dv0);
  if (rc) return rc;
  return npfem_sync_status(b);
}

int npfem_sync_status(npfem_batch b) {
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  DeviceGuard guard(b->device);
  int st = 0;
  HIP_TRY(hipStreamSynchronize(b->stream), "sync");
  HIP_TRY(hipMemcpy(&st, b->status, sizeof(int), hipMemcpyDeviceToHost), "status read");
  HIP_TRY(hipMemset(b->status, 0, sizeof(int)), "status clear");
  HIP_TRY(hipDeviceSynchronize(), "status clear");
  if (st & ST_NONFINITE) return fail(NPFEM_ERR_NONFINITE, "non-finite value in state, forces or a reduction");
  return NPFEM_OK;
}

int npfem_get_energy(npfem_batch b, double* host_out, int32_t capacity, int32_t* n_iter_out) {
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (!(b->flags & NPFEM_OPT_ENERGY) || !b->energy)
    return fail(NPFEM_ERR_INVALID_ARG, "energy recording is off (NPFEM_OPT_ENERGY) or no step ran");
  const long long need = (long long)b->energy_iters * b->n_cells;
  if (!host_out || capacity < need) return fail(NPFEM_ERR_INVALID_ARG, "capacity below n_iter * n_cells");
  DeviceGuard guard(b->device);
  HIP_TRY(hipStreamSynchronize(b->stream), "sync");
  HIP_TRY(hipMemcpy(host_out, b->energy, sizeof(double) * need, hipMemcpyDeviceToHost), "energy read");
  if (n_iter_out) *n_iter_out = b->energy_iters;
  return NPFEM_OK;
}

int npfem_get_volume(npfem_batch b, double* host_out) {
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (!host_out) return fail(NPFEM_ERR_INVALID_ARG, "host_out is NULL");
  DeviceGuard guard(b->device);
  for (auto& c : b->cls) {
    hipError_t e = b->fp64 ? launch_volume<double>(slice_of<double>(c), (const double*)b->pos,
                                                   b->sumN, b->volume_buf, b->stream)
                           : launch_volume<float>(slice_of<float>(c), (const float*)b->pos,
                                                  b->sumN, b->volume_buf, b->stream);
    if (e != hipSuccess) return hip_fail(e, "volume");
  }
  HIP_TRY(hipStreamSynchronize(b->stream), "sync");
  HIP_TRY(hipMemcpy(host_out, b->volume_buf, sizeof(double) * b->n_cells, hipMemcpyDeviceToHost),
          "volume read");
  return NPFEM_OK;
}

int npfem_get_volume_noalloc(npfem_batch b, double* host_out) {
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (!host_out) return fail(NPFEM_ERR_INVALID_ARG, "host_out is NULL");
  if (b->n_cells > kVolumeScratchCells)
    return fail(NPFEM_ERR_INVALID_ARG,
                "more cells than the static staging buffer of npfem_get_volume_noalloc holds (65536)");
  DeviceGuard guard(b->device);
  double* stage = nullptr;
  HIP_TRY(volume_scratch(&stage), "staging buffer address");
  for (auto& c : b->cls) {
    hipError_t e = b->fp64 ? launch_volume<double>(slice_of<double>(c), (const double*)b->pos,
                                                   b->sumN, stage, b->stream)
                           : launch_volume<float>(slice_of<float>(c), (const float*)b->pos,
                                                  b->sumN, stage, b->stream);
    if (e != hipSuccess) return hip_fail(e, "volume");
  }
  HIP_TRY(hipMemcpyAsync(host_out, stage, sizeof(double) * b->n_cells, hipMemcpyDeviceToHost,
                         b->stream),
          "volume read");
  HIP_TRY(hipStreamSynchronize(b->stream), "sync");
  return NPFEM_OK;
}

int npfem_batch_config(npfem_batch b, int32_t cls, int32_t out[4]) {
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (!out || cls < 0 || cls >= (int)b->cls.size())
    return fail(NPFEM_ERR_INVALID_ARG, "class index out of range");
  const ClassState& c = b->cls[cls];
  int bm = 0, bn = 0;
  gemm_tile_shape(c.gemm_tile, &bm, &bn);
  out[0] = c.local_block;
  out[1] = bm;
  out[2] = bn;
  out[3] = b->n_refine;
  return NPFEM_OK;
}

int npfem_set_batch_config(npfem_batch b, int32_t cls, const int32_t in[4]) {
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (!in || cls < 0 || cls >= (int)b->cls.size())
    return fail(NPFEM_ERR_INVALID_ARG, "class index out of range");
  ClassState& c = b->cls[cls];
  if (in[0] != 128 && in[0] != 256 && in[0] != 512 && in[0] != 1024)
    return fail(NPFEM_ERR_INVALID_ARG, "local workgroup size must be 128, 256, 512 or 1024");
  if ((c.N + in[0] - 1) / in[0] > 11)
    return fail(NPFEM_ERR_INVALID_ARG, "workgroup too small for a %d-vertex mesh", c.N);
  if (in[0] == 1024 && (b->fp64 || c.N > 3072))
    return fail(NPFEM_ERR_INVALID_ARG,
                "1024-thread local steps take FP32 state and meshes of at most 3072 vertices");
  int tile = -1;
  for (int t = 0; t < gemm_num_tiles(b->gemm_kind); ++t) {
    int bm, bn;
    gemm_tile_shape(t, &bm, &bn);
    if (bm == in[1] && bn == in[2]) tile = t;
  }
  if (tile < 0) return fail(NPFEM_ERR_INVALID_ARG, "unsupported GEMM tile %dx%d", in[1], in[2]);
  if (in[3] > 100) return fail(NPFEM_ERR_INVALID_ARG, "too many correction sweeps");
  c.local_block = in[0];
  c.gemm_tile = tile;
  if (in[3] >= 0) {
    b->n_refine_opt = in[3];
    b->n_refine = in[3];
  }
  b->tuned = true;
  drop_graphs(b);
  return NPFEM_OK;
}

int npfem_kernel_times(npfem_batch b, double* ms_out, int64_t* launches_out, int32_t reset) {
  if (!b || b->tag != kBatchTag) return fail(NPFEM_ERR_INVALID_ARG, "not a batch handle");
  if (!(b->flags & NPFEM_OPT_KERNEL_TIMING))
    return fail(NPFEM_ERR_INVALID_ARG, "kernel timing is off (NPFEM_OPT_KERNEL_TIMING)");
  DeviceGuard guard(b->device);
  HIP_TRY(b->ev_harvest(), "kernel timing");
  for (int k = 0; k < NPFEM_KERNEL_KINDS; ++k) {
    if (ms_out) ms_out[k] = b->kt_ms[k];
    if (launches_out) launches_out[k] = b->kt_n[k];
    if (reset) {
      b->kt_ms[k] = 0.0;
      b->kt_n[k] = 0;
    }
  }
  return NPFEM_OK;
}

int npfem_free(void* handle) {
  if (!handle) return NPFEM_OK;
  const uint32_t tag = *static_cast<uint32_t*>(handle);
  if (tag == kMeshTag) {
    npfem_mesh_s* m = static_cast<npfem_mesh_s*>(handle);
    m->tag = 0;
    delete m;
    return NPFEM_OK;
  }
  if (tag == kBatchTag) {
    npfem_batch_s* b = static_cast<npfem_batch_s*>(handle);
    DeviceGuard guard(b->device);
    hipStreamSynchronize(b->stream);
    b->tag = 0;
    delete b;
    return NPFEM_OK;
  }
  return fail(NPFEM_ERR_INVALID_ARG, "unknown handle");
}

}  // extern "C"
