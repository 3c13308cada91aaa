/*
 * npfem.h - C ABI of the batched projective-dynamics membrane solver for
 * MI355X (gfx950).
 *
 * The library advances many deformable blood cells (closed triangulated
 * membranes) by implicit time steps of the elastodynamics equation (eq. 2:
 * rho0 phi'' = div P + rho0 b) discretised as a mass-lumped linear
 * finite-element membrane (Introduction) and integrated with projective
 * dynamics, the scheme the solid solver derives from (Implementation and
 * architecture). The fluid and the immersed-boundary coupling are outside
 * the library: the caller supplies external nodal forces and receives
 * positions and velocities, which is the data the fluid-solid exchange
 * carries (Implementation and architecture). Like the stand-alone solver
 * library driven from Python through ctypes (section "Rhino-Grasshopper
 * environment"), the calls are: load meshes with a material, build a batch,
 * add forces and run steps.
 *
 * One step, per cell, with lumped vertex mass m and time step h:
 *   s = x + h v + (h^2/m) f;  q = s
 *   repeat n_iter: local step (projections of every elemental potential),
 *                  global step  A q = (m/h^2) s + sum_i w_i S_i^T P_i
 *   x <- q;  v <- (q - x_old)/h
 * with A = (m/h^2) I + (w_s + w_a) sum_t A_t G_t G_t^T
 *        + w_b sum_e c_e K_e K_e^T + w_v I
 * (per-triangle strain and area, per-hinge bending, per-cell volume; the
 * body energy is the weighted sum of elemental potentials, section "Setting
 * up new materials").
 *
 * Conventions
 *  - Every function returns NPFEM_OK (0) or a negative NPFEM_ERR_* code; the
 *    thread-local message of the last failure is npfem_last_error(). No C++
 *    exception crosses the ABI.
 *  - Per-vertex device arrays are SoA [3][sum_N]: all x, then all y, then all
 *    z, cells class-major then cell-major. Element type is double for
 *    NPFEM_FP64 and float for every other precision.
 *  - Positions are cell-local: relative to an origin per cell that the caller
 *    keeps (in FP64 if it wants). The step is translation-equivariant, so the
 *    library never needs the origin; keeping coordinates small keeps FP32
 *    rounding at the scale of the cell, not of the domain.
 *  - Device buffers passed in (positions, velocities, forces, gradients) are
 *    owned by the caller and must outlive the batch. The library copies mesh
 *    data and owns its operators, workspace and graphs.
 *  - All device work of a batch is ordered on the stream given at creation;
 *    calls return without synchronising unless documented otherwise.
 *  - A batch is not thread-safe: one host thread at a time per batch.
 */
#ifndef NPFEM_H
#define NPFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NPFEM_ABI_VERSION 1

enum npfem_status {
  NPFEM_OK = 0,
  NPFEM_ERR_INVALID_ARG = -1,    /* bad pointer, size, order or option */
  NPFEM_ERR_MESH_OPEN = -2,      /* an edge has only one incident triangle */
  NPFEM_ERR_MESH_NONMANIFOLD = -3, /* edge used twice in one direction, >2 triangles, bad Euler characteristic */
  NPFEM_ERR_DEGENERATE_TRI = -4, /* zero-area rest triangle or repeated vertex */
  NPFEM_ERR_NOT_SPD = -5,        /* non-positive pivot in the FP64 factorisation */
  NPFEM_ERR_NONFINITE = -6,      /* NaN or Inf seen in state, forces or a reduction */
  NPFEM_ERR_HIP = -7,            /* HIP runtime error */
  NPFEM_ERR_OOM = -8             /* device or host allocation failed */
};

typedef enum npfem_precision {
  NPFEM_FP64 = 0,        /* state, local step and global step in FP64 */
  NPFEM_FP32 = 1,        /* FP32 state and kernels, FP32 MFMA global step */
  NPFEM_BF16_REFINE = 2, /* FP32 state; global step on BF16 MFMA (FP32 accumulate) + refinement */
  NPFEM_FP16_REFINE = 3  /* as above with FP16 MFMA operands */
} npfem_precision;

/* Nominal material of a mesh class: constraint weights and lumped mass per
 * vertex (units are the caller's; the bundled workloads use um, s and
 * consistent force units). */
typedef struct npfem_material {
  double w_stretch; /* strain potential weight (times rest triangle area) */
  double w_area;    /* area-preservation weight (times rest triangle area) */
  double w_bend;    /* hinge bending weight (times 3/(A1+A2)) */
  double w_volume;  /* cell volume-preservation weight (per vertex) */
  double vertex_mass;
} npfem_material;

#define NPFEM_OPT_ENERGY 1u     /* record per-cell FP64 energy of every PD iterate of the last step */
#define NPFEM_OPT_NO_GRAPH 2u   /* launch kernels one by one instead of replaying a captured hipGraph */
#define NPFEM_OPT_AUTOTUNE 4u   /* time candidate launch shapes per mesh class at the first
                                   step; FP32 batches of several classes also time whole
                                   steps (from a saved and restored state) with a
                                   1024-thread local step for meshes of 1537-3072 vertices */
#define NPFEM_OPT_SYNC_CHECK 8u /* npfem_step synchronises and reports NONFINITE itself */
#define NPFEM_OPT_KERNEL_TIMING 16u /* launch one by one with a HIP event pair around every
                                       kernel; read with npfem_kernel_times */

/* Kernel kinds reported by npfem_kernel_times. */
enum npfem_kernel_kind {
  NPFEM_KERNEL_PREDICT = 0,  /* start of step: inertia term and first iterate */
  NPFEM_KERNEL_LOCAL = 1,    /* local step + right-hand-side gather */
  NPFEM_KERNEL_GLOBAL = 2,   /* global-step GEMM (first solve and corrections) */
  NPFEM_KERNEL_RESIDUAL = 3, /* refinement residual */
  NPFEM_KERNEL_UPDATE = 4,   /* end of step: positions and velocities */
  NPFEM_KERNEL_KINDS = 5
};

typedef struct npfem_options {
  int32_t precision;    /* npfem_precision */
  int32_t n_refine;     /* correction sweeps after each global solve; -1 = automatic */
  int32_t max_vol_iter; /* cap on volume-projection sub-iterations; 0 = default */
  uint32_t flags;       /* NPFEM_OPT_* */
  void* stream;         /* hipStream_t for all work of the batch; NULL = null stream */
} npfem_options;

typedef struct npfem_mesh_s* npfem_mesh;
typedef struct npfem_batch_s* npfem_batch;

/* Host-only. Validates and copies one mesh class and precomputes its rest
 * operators in FP64: per-triangle G_t (3x2) and area, per-hinge cotangent
 * stencil K_e, weight c_e and rest magnitude, rest volume, vertex incidence
 * lists and the sparse Laplacians.
 *   rest_xyz  host [n_verts][3] rest shape (also the default initial shape)
 *   tris      host [n_tris][3] vertex indices, counter-clockwise seen from
 *             outside (positive enclosed volume)
 *   mat       nominal material
 * Errors: INVALID_ARG (NULL, n_verts < 4, n_verts > 65535, index out of
 * range, non-finite or non-positive weights/mass, negative volume),
 * MESH_OPEN, MESH_NONMANIFOLD, DEGENERATE_TRI, OOM. */
int npfem_create_mesh(const double* rest_xyz, int32_t n_verts, const int32_t* tris,
                      int32_t n_tris, const npfem_material* mat, npfem_mesh* out);

/* Host-only queries of a mesh (any output pointer may be NULL). */
int npfem_mesh_info(npfem_mesh m, int32_t* n_verts, int32_t* n_tris, int32_t* n_hinges,
                    double* rest_volume);

/* Host-only: the dense FP64 system matrix A (row-major [n_verts][n_verts])
 * for the given weights (host [4]: stretch, area, bend, volume; NULL =
 * nominal) and time step. For inspection and tests. */
int npfem_mesh_system_matrix(npfem_mesh m, const double* weights4, double dt, double* A_out);

/* Builds a batch of n_cells cells over n_meshes mesh classes and binds the
 * caller's state buffers.
 *   meshes        host [n_meshes]
 *   cell_mesh     host [n_cells] class index per cell, non-decreasing
 *   cell_weights  host [n_cells][4] per-cell (stretch, area, bend, volume)
 *                 weights, or NULL for each class's nominal material
 *   pos, vel      device SoA [3][sum_N] (double for NPFEM_FP64, else float),
 *                 updated in place by npfem_step
 *   opt           options (NULL = FP32, defaults)
 * Allocates device workspace; the FP64 factorisation happens at the first
 * step (it depends on the time step). Errors: INVALID_ARG (also for a mesh
 * of more than 5632 vertices, beyond the local step's widest workgroup of
 * 512 threads x 11 vertices, and for an FP64 batch with a mesh of more than
 * 2550 vertices, whose local step does not fit the 160 KB of LDS of a CU),
 * HIP, OOM. */
int npfem_create_batch(const npfem_mesh* meshes, int32_t n_meshes, const int32_t* cell_mesh,
                       int32_t n_cells, const double* cell_weights, void* pos, void* vel,
                       const npfem_options* opt, npfem_batch* out);

/* Advances every cell by one implicit step of length dt with n_iter
 * local/global iterations under constant external nodal forces.
 *   ext_forces  device SoA [3][sum_N], element type as pos
 * The first call, and any call with a dt different from the previous one,
 * rebuilds the system matrices, inverts them in FP64 on the GPU and
 * re-captures the step graph (synchronous, slow). Otherwise the call only
 * enqueues work on the batch stream. Non-finite inputs set a device flag read
 * by npfem_sync_status (or returned here with NPFEM_OPT_SYNC_CHECK).
 * Errors: INVALID_ARG (dt <= 0 or not finite, n_iter < 1 or > 1000), NOT_SPD,
 * NONFINITE (only with NPFEM_OPT_SYNC_CHECK), HIP, OOM. */
int npfem_step(npfem_batch b, const void* ext_forces, double dt, int32_t n_iter);

/* n_steps calls of npfem_step (same forces, dt and n_iter) as ONE launch: the
 * uneven batch's whole run, every step with its branch per mesh class, is
 * captured into one graph at the first call with these arguments (forces
 * pointer, n_iter, n_steps) and replayed afterwards; results are bitwise
 * those of the step-by-step calls. For runs of solid steps with no exchange
 * in between: the solid's own time steps between two fluid-solid exchanges
 * (the time discretisation is per solver, Implementation and architecture)
 * and the cell-packing application's thousands of solid-only steps
 * (Applications, cell packing). With NPFEM_OPT_NO_GRAPH or
 * NPFEM_OPT_KERNEL_TIMING the steps are launched one by one.
 * Errors: as npfem_step; INVALID_ARG for n_steps < 1 or > 1000. */
int npfem_run(npfem_batch b, const void* ext_forces, double dt, int32_t n_iter, int32_t n_steps);

/* Replaces the per-cell weights (host [n_cells][4]: stretch, area, bend,
 * volume; NULL = each class's nominal material). The class operators stay
 * those of the nominal material; cells whose weights differ are solved with
 * correction sweeps against their own matrix (the sweep count follows from
 * the largest deviation). Synchronises; the next step re-captures its graph.
 * Errors: INVALID_ARG (non-finite or negative weights, or weights too far
 * from nominal for the sweeps to converge), HIP. */
int npfem_set_weights(npfem_batch b, const double* cell_weights);

/* Viscous damping of mesh class cls (-1: every class): a damping force
 * -C v with C = alpha m I + beta ((w_s + w_a) L_tri + w_b L_bend), mass- and
 * stiffness-proportional (the material's viscosity parameters Calpha and
 * Cbeta; the elastodynamics equation with a viscous term, Introduction),
 * taken implicitly at the end-of-step velocity: the step minimises its
 * objective plus (1/2h)(q - x)^T C (q - x), so the global system becomes
 * A + C/h and the first iterate (s + alpha h x)/(1 + alpha h). L_tri and
 * L_bend are the cell's strain/area and bending Laplacians (with its own
 * weights), so C has no net force and does not resist rigid translation.
 * 0, 0 (the default) is the undamped step. The next step refactors and
 * re-captures (slow); a stiffness-proportional term allocates one column
 * buffer at the first call that sets it. npfem_rollout_adjoint does not
 * cover damping (INVALID_ARG), and the energy of NPFEM_OPT_ENERGY omits the
 * damping term. Synchronises. Errors: INVALID_ARG (class out of range,
 * negative or non-finite coefficients), HIP, OOM. */
int npfem_set_damping(npfem_batch b, int32_t cls, double alpha, double beta);

/* Solver of the implicit step. history < 0 (the default): classic PD, n_iter
 * local/global iterations. history >= 0: the quasi-Newton step of the
 * redesigned PD the solver follows (Implementation and architecture, after
 * Liu et al.): n_iter L-BFGS iterations on the step's objective
 *   g(q) = (m/2h^2)|q - s|^2 + sum_i (w_i/2) dist^2(S_i q, C_i)
 * (gradient A q - b(q), the PD global step's residual) from q^0 = s, with
 * the PD matrix as initial Hessian (one product with the class operator per
 * iteration), the last `history` (<= 16) pairs of iterate and gradient
 * changes (two-loop recursion; a pair with non-positive curvature is kept
 * inert), and a backtracking line search: alpha = 1, halved while the
 * objective fails the Armijo test (c = 1e-4; FP32 batches allow an increase
 * of 2^-20 of the objective, the rounding of an FP32 state's objective), at
 * most line_search rounds (1..8), the last trial taken if none passes. Each round is one local step
 * for the cells still searching. history 0 with line_search 1 is PD.
 * FP64 and FP32 batches only; not with damping or contacts (npfem_step then
 * fails), nor with npfem_rollout. The first call allocates (4 + 2 history)
 * column sets and per-cell scalars. Synchronises. Errors: INVALID_ARG, HIP,
 * OOM. */
int npfem_set_quasi_newton(npfem_batch b, int32_t history, int32_t line_search);

/* Contact (collision) potentials of every cell against its colliding
 * neighbours, which the caller supplies (the fluid side exchanges them,
 * Implementation and architecture; their strength is the collision weight,
 * section "RBC collision at an obstacle"). Cell c's neighbourhood is the list
 * of contact points y_k, k in [cell_offsets[c], cell_offsets[c + 1]), on
 * the other surfaces (neighbouring cells, obstacles), each with the unit
 * outward normal n_k of that surface, in c's cell-local coordinates. Every
 * vertex carries the potential (weight/2) dist^2(q_v, C_v), C_v the
 * half-space (p - y_k) . n_k >= 0 of the contact point nearest to q_v
 * (first on ties): vertices outside it feel nothing, vertices inside are
 * pulled to its tangent plane. Since every vertex carries it, the system
 * matrix gains weight * I and stays constant.
 *   weight        > 0 enables, 0 disables (the arrays may then be NULL)
 *   points, normals  device SoA [3][n_points], element type as pos
 *   cell_offsets  device int32 [n_cells + 1], non-decreasing
 * The arrays are caller-owned and read at every step: their contents may
 * change between steps (move the contacts), their addresses may not without
 * a new call. A changed weight refactors at the next step; any call
 * re-captures. Each vertex scans its cell's list (cost ~ points per cell).
 * npfem_rollout_adjoint does not cover contacts (INVALID_ARG). Synchronises.
 * Errors: INVALID_ARG (negative or non-finite weight, NULL arrays with a
 * positive weight), HIP. */
int npfem_set_contacts(npfem_batch b, double weight, const void* points, const void* normals,
                       const int32_t* cell_offsets, int64_t n_points);

/* Immersed-boundary transfer between a periodic Cartesian fluid grid and the
 * vertices (the coupling on either side of the solid step: the IBM computes
 * the body force of eqs. 1 and 2, and the data exchange between the grid and
 * the surface meshes goes through interpolation kernels, Introduction), with
 * Peskin's 4-point regularised delta function
 *   delta_h(x) = phi(x/dx) phi(y/dx) phi(z/dx) / dx^3,
 *   phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4r^2))/8       for |r| <= 1,
 *            (5 - 2|r| - sqrt(-7 + 12|r| - 4r^2))/8      for 1 <= |r| <= 2.
 * Grid node (i, j, k) sits at grid_origin + dx (i, j, k) (host [3]); indices
 * wrap periodically over dims (host [3], each >= 4). Grid fields are device
 * SoA [3][nx ny nz], flat index i + nx (j + ny k), element type as pos. A
 * vertex's global position is cell_origins[c] (device FP64 [n_cells][3]) plus
 * its cell-local position (the batch's current pos).
 * npfem_ibm_interpolate: out_u (device SoA [3][sum_N]) = sum over the 64 nodes
 *   around each vertex of u_g phi phi phi (the fluid velocity at the vertex).
 * npfem_ibm_spread: grid_f = sum_v F_v delta_h(x_g - X_v) (a force density;
 *   sum_g grid_f dx^3 = sum_v F_v), bitwise reproducible: contributions are
 *   added as 64-bit fixed-point integers scaled from max |F| (~40 bits below
 *   the largest possible contribution), then converted. The first call for a
 *   grid larger than any before allocates the accumulators (3 x 8 bytes per
 *   node); otherwise nothing is allocated. Non-finite forces set the flag of
 *   npfem_sync_status.
 * Both enqueue on the batch stream and return without synchronising. Errors:
 * INVALID_ARG (NULL arrays, dims < 4 or > 2e9 nodes, dx <= 0), HIP, OOM. */
int npfem_ibm_interpolate(npfem_batch b, const double* cell_origins, const void* grid_u,
                          const int32_t dims[3], double dx, const double grid_origin[3],
                          void* out_u);
int npfem_ibm_spread(npfem_batch b, const double* cell_origins, const void* vertex_f,
                     const int32_t dims[3], double dx, const double grid_origin[3], void* grid_f);

/* Differentiable rollout: n_steps calls of npfem_step under constant forces,
 * storing (positions, velocities) before every ckpt_every-th step as
 * checkpoints for npfem_rollout_adjoint (the time-step loop the adjoint
 * reverses). Positions and velocities hold the final state on return.
 * Errors: as npfem_step; INVALID_ARG for n_steps < 1 or ckpt_every outside
 * [1, n_steps]; OOM. */
int npfem_rollout(npfem_batch b, const void* ext_forces, double dt, int32_t n_iter,
                  int32_t n_steps, int32_t ckpt_every);

/* Reverse-mode gradient of a scalar loss L(x_T, v_T) of the last rollout.
 * Each checkpointed segment is recomputed storing every PD iterate, then the
 * iterations and steps are reversed: per iteration one solve with the
 * (symmetric) system matrix and one projection-VJP kernel.
 *   dL_dx, dL_dv   device SoA [3][sum_N] (element type as pos), dL_dv may be NULL
 *   dL_dw          device FP64 [n_cells][4]: dL/d(stretch, area, bend, volume)
 *                  weights of each cell (may be NULL)
 *   dL_df          device SoA [3][sum_N]: dL/d(ext_forces), constant forces
 *                  (may be NULL)
 *   dL_dx0, dL_dv0 device SoA [3][sum_N]: gradients w.r.t. the initial state
 *                  (may be NULL)
 * Synchronises. Positions and velocities are not modified. Not available for
 * NPFEM_FP16_REFINE (INVALID_ARG). Errors: INVALID_ARG (no rollout, or dt or
 * weights changed since), NONFINITE, HIP, OOM. */
int npfem_rollout_adjoint(npfem_batch b, const void* dL_dx, const void* dL_dv, void* dL_dw,
                          void* dL_df, void* dL_dx0, void* dL_dv0);

/* Synchronises the batch stream, returns NPFEM_ERR_NONFINITE if any kernel
 * saw a NaN/Inf (in state, forces, or a per-cell FP64 reduction) since the
 * previous call, and clears the flag. */
int npfem_sync_status(npfem_batch b);

/* Synchronises and copies to host the per-cell FP64 energy E(q^k) of the PD
 * iterates k = 0 .. n_iter-1 of the last step, layout [n_iter][n_cells].
 * Requires NPFEM_OPT_ENERGY. capacity = number of doubles host_out holds. */
int npfem_get_energy(npfem_batch b, double* host_out, int32_t capacity, int32_t* n_iter_out);

/* Synchronises and writes the FP64 enclosed volume of every cell's current
 * positions into host [n_cells]. */
int npfem_get_volume(npfem_batch b, double* host_out);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): npfem_get_volume
 * with the per-cell staging buffer in a static device array of 65536
 * doubles (one copy per device, held until the process ends) instead of the
 * batch's own buffer. Allocates nothing. Writes the FP64 enclosed volume of
 * every cell's current positions into host [n_cells]; synchronises the batch
 * stream. Every call on one device shares that array: calls that overlap on
 * one device (other host threads, other batches' streams) race and must be
 * serialised by the caller. Errors: INVALID_ARG (NULL output, or more than
 * 65536 cells), HIP. */
int npfem_get_volume_noalloc(npfem_batch b, double* host_out);

/* Launch configuration chosen for mesh class cls (after the first step, which
 * runs the autotuner when NPFEM_OPT_AUTOTUNE is set): out[0] local-step
 * workgroup size, out[1] / out[2] global-step GEMM tile rows / columns
 * (rows 0: the column-stationary kernel, out[2] columns per workgroup, whole
 * operator per workgroup), out[3] correction sweeps per global solve. Host
 * only. */
int npfem_batch_config(npfem_batch b, int32_t cls, int32_t out[4]);

/* Pins the launch configuration of class cls (same layout as
 * npfem_batch_config; in[3] < 0 keeps the automatic sweep count), e.g. to
 * replay a configuration tuned earlier. The next step re-captures its graph.
 * Workgroup sizes: 128, 256, 512, and 1024 for FP32 state and meshes of at
 * most 3072 vertices. Errors: INVALID_ARG for an unsupported workgroup size
 * or tile shape. */
int npfem_set_batch_config(npfem_batch b, int32_t cls, const int32_t in[4]);

/* Requires NPFEM_OPT_KERNEL_TIMING. Synchronises, converts every event pair
 * recorded since the last call into elapsed milliseconds and adds them to
 * running totals per kernel kind; writes the totals (host [NPFEM_KERNEL_KINDS]
 * ms and launch counts, either may be NULL). reset != 0 clears the totals
 * after reading. */
int npfem_kernel_times(npfem_batch b, double* ms_out, int64_t* launches_out, int32_t reset);

/* Releases a mesh or a batch (the handle type is recorded in the object);
 * NULL is accepted. A mesh may be freed once the batches built on it are
 * created (they copy what they need). */
int npfem_free(void* handle);

/* Message of the last error on the calling thread ("" if none). */
const char* npfem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NPFEM_H */
