"""Python objects over the C ABI: meshes, batches and time stepping.

PyTorch provides device memory and the stream; every step of the solver runs
in the HIP library (libnpfem.so). There is no fallback path: if the library or
a GPU is missing, construction raises.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib

_PREC = {"fp64": _lib.FP64, "fp32": _lib.FP32, "bf16": _lib.BF16_REFINE, "fp16": _lib.FP16_REFINE}


def precision_code(p) -> int:
    if isinstance(p, int):
        return p
    return _PREC[p]


def state_dtype(precision) -> torch.dtype:
    return torch.float64 if precision_code(precision) == _lib.FP64 else torch.float32


class Mesh:
    """One mesh class: rest shape, triangles and nominal material (host only)."""

    def __init__(self, rest_xyz, tris, weights=(1.0, 1.0, 0.01, 10.0), vertex_mass=1e-3):
        lib = _lib.load()
        x = np.ascontiguousarray(rest_xyz, dtype=np.float64)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        if x.ndim != 2 or x.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 3:
            raise ValueError("rest_xyz must be [N, 3] and tris [F, 3]")
        mat = _lib.Material(*(float(w) for w in weights), float(vertex_mass))
        h = ctypes.c_void_p()
        _lib.check(lib.npfem_create_mesh(x.ctypes.data, x.shape[0], t.ctypes.data, t.shape[0],
                                         ctypes.byref(mat), ctypes.byref(h)))
        self.handle = h
        self.weights = tuple(float(w) for w in weights)
        self.vertex_mass = float(vertex_mass)
        self.n_verts = int(x.shape[0])

    def info(self):
        n, f, e = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        v = ctypes.c_double()
        _lib.check(_lib.load().npfem_mesh_info(self.handle, ctypes.byref(n), ctypes.byref(f),
                                               ctypes.byref(e), ctypes.byref(v)))
        return n.value, f.value, e.value, v.value

    def system_matrix(self, dt, weights=None) -> np.ndarray:
        A = np.empty((self.n_verts, self.n_verts), dtype=np.float64)
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
        _lib.check(_lib.load().npfem_mesh_system_matrix(
            self.handle, None if w is None else w.ctypes.data, float(dt), A.ctypes.data))
        return A

    def close(self):
        if self.handle:
            _lib.load().npfem_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Cells of several mesh classes stepped together on one GPU.

    pos, vel: CUDA tensors [3, sum_N] (float64 for precision 'fp64', else
    float32), cell-local coordinates, updated in place by step().
    """

    def __init__(self, meshes, cell_mesh, pos: torch.Tensor, vel: torch.Tensor, cell_weights=None,
                 precision="fp32", n_refine=-1, max_vol_iter=0, energy=False, graph=True,
                 sync_check=False, kernel_timing=False, autotune=False, stream=None):
        lib = _lib.load()
        code = precision_code(precision)
        dt_ = state_dtype(code)
        for name, t in (("pos", pos), ("vel", vel)):
            if not (t.is_cuda and t.dtype == dt_ and t.is_contiguous() and t.dim() == 2
                    and t.shape[0] == 3):
                raise ValueError(f"{name} must be a contiguous CUDA {dt_} tensor [3, sum_N]")
        self.pos, self.vel = pos, vel
        self.meshes = list(meshes)
        cm = np.ascontiguousarray(cell_mesh, dtype=np.int32)
        self.n_cells = int(cm.shape[0])
        sum_n = int(sum(self.meshes[k].n_verts for k in cm))
        if pos.shape[1] != sum_n or vel.shape[1] != sum_n:
            raise ValueError(f"state has {pos.shape[1]} vertices, cells need {sum_n}")
        w = None if cell_weights is None else np.ascontiguousarray(cell_weights, dtype=np.float64)
        if w is not None and w.shape != (self.n_cells, 4):
            raise ValueError("cell_weights must be [n_cells, 4]")
        flags = 0
        if energy:
            flags |= _lib.OPT_ENERGY
        if not graph:
            flags |= _lib.OPT_NO_GRAPH
        if sync_check:
            flags |= _lib.OPT_SYNC_CHECK
        if kernel_timing:
            flags |= _lib.OPT_KERNEL_TIMING
        if autotune:
            flags |= _lib.OPT_AUTOTUNE
        if stream is None:
            stream = torch.cuda.current_stream(pos.device)
        self.stream = stream
        opt = _lib.Options(code, int(n_refine), int(max_vol_iter), flags,
                           ctypes.c_void_p(stream.cuda_stream))
        handles = (ctypes.c_void_p * len(self.meshes))(*[m.handle.value for m in self.meshes])
        h = ctypes.c_void_p()
        with torch.cuda.device(pos.device):
            _lib.check(lib.npfem_create_batch(
                handles, len(self.meshes), cm.ctypes.data, self.n_cells,
                None if w is None else w.ctypes.data, pos.data_ptr(), vel.data_ptr(),
                ctypes.byref(opt), ctypes.byref(h)))
        self.handle = h
        self.precision = code
        self.dtype = dt_
        self._forces = None
        self.rollout_generation = 0  # counts rollouts (the library keeps the last one's record)

    def step(self, forces: torch.Tensor, dt: float, n_iter: int):
        if not (forces.is_cuda and forces.dtype == self.dtype and forces.is_contiguous()
                and tuple(forces.shape) == tuple(self.pos.shape)):
            raise ValueError("forces must match pos (contiguous CUDA, same dtype and shape)")
        self._forces = forces  # keep alive while the graph may reference it
        _lib.check(_lib.load().npfem_step(self.handle, forces.data_ptr(), float(dt), int(n_iter)))

    def run(self, forces: torch.Tensor, dt: float, n_iter: int, n_steps: int):
        """n_steps steps as one graph launch (npfem_run)."""
        if not (forces.is_cuda and forces.dtype == self.dtype and forces.is_contiguous()
                and tuple(forces.shape) == tuple(self.pos.shape)):
            raise ValueError("forces must match pos (contiguous CUDA, same dtype and shape)")
        self._forces = forces
        _lib.check(_lib.load().npfem_run(self.handle, forces.data_ptr(), float(dt), int(n_iter),
                                         int(n_steps)))

    def sync_status(self):
        _lib.check(_lib.load().npfem_sync_status(self.handle))

    def set_weights(self, cell_weights):
        """Per-cell (stretch, area, bend, volume) weights [n_cells, 4]; None = nominal."""
        w = None if cell_weights is None else np.ascontiguousarray(cell_weights, dtype=np.float64)
        if w is not None and w.shape != (self.n_cells, 4):
            raise ValueError("cell_weights must be [n_cells, 4]")
        _lib.check(_lib.load().npfem_set_weights(self.handle, None if w is None else w.ctypes.data))

    def set_damping(self, cls: int, alpha: float, beta: float):
        """Viscous damping C = alpha m I + beta K_d of class cls (-1: all)."""
        _lib.check(_lib.load().npfem_set_damping(self.handle, int(cls), float(alpha), float(beta)))

    def set_quasi_newton(self, history: int = 5, line_search: int = 3):
        """L-BFGS implicit step (history >= 0) or classic PD (history < 0)."""
        _lib.check(_lib.load().npfem_set_quasi_newton(self.handle, int(history), int(line_search)))

    def set_contacts(self, weight: float, points=None, normals=None, cell_offsets=None):
        """Contact potentials: points / normals device SoA [3][P] (pos dtype),
        cell_offsets device int32 [n_cells + 1]; weight 0 disables. The
        tensors must stay alive (and at their addresses) while stepping."""
        if weight and not (points is not None and normals is not None and cell_offsets is not None):
            raise ValueError("contact arrays are required with a positive weight")
        if weight:
            for t, name in ((points, "points"), (normals, "normals")):
                if not (t.is_cuda and t.dtype == self.dtype and t.is_contiguous() and t.dim() == 2
                        and t.shape[0] == 3):
                    raise ValueError(f"{name} must be a contiguous CUDA [3, P] tensor of the state dtype")
            if not (cell_offsets.is_cuda and cell_offsets.dtype == torch.int32
                    and tuple(cell_offsets.shape) == (self.n_cells + 1,)):
                raise ValueError("cell_offsets must be a CUDA int32 tensor [n_cells + 1]")
            self._contacts = (points, normals, cell_offsets)
            np_ = points.shape[1]
            _lib.check(_lib.load().npfem_set_contacts(self.handle, float(weight), points.data_ptr(),
                                                      normals.data_ptr(), cell_offsets.data_ptr(),
                                                      int(np_)))
        else:
            self._contacts = None
            _lib.check(_lib.load().npfem_set_contacts(self.handle, 0.0, None, None, None, 0))

    def _grid_args(self, grid, dims, origin):
        dims = np.ascontiguousarray(dims, dtype=np.int32)
        origin = np.ascontiguousarray(origin, dtype=np.float64)
        if dims.shape != (3,) or origin.shape != (3,):
            raise ValueError("dims and origin must have 3 entries")
        n = int(np.prod(dims.astype(np.int64)))
        if not (grid.is_cuda and grid.dtype == self.dtype and grid.is_contiguous()
                and tuple(grid.shape) == (3, n)):
            raise ValueError("grid field must be a contiguous CUDA [3, nx*ny*nz] tensor of the state dtype")
        return dims, origin

    def _origins(self, cell_origins):
        if not (cell_origins.is_cuda and cell_origins.dtype == torch.float64
                and cell_origins.is_contiguous() and tuple(cell_origins.shape) == (self.n_cells, 3)):
            raise ValueError("cell_origins must be a contiguous CUDA float64 [n_cells, 3] tensor")

    def ibm_interpolate(self, cell_origins, grid_u, dims, dx, origin, out=None):
        """Fluid velocity at the vertices (Peskin 4-point kernel, periodic grid)."""
        self._origins(cell_origins)
        dims, origin = self._grid_args(grid_u, dims, origin)
        out = torch.empty_like(self.pos) if out is None else out
        self._check_field(out, "out")
        _lib.check(_lib.load().npfem_ibm_interpolate(self.handle, cell_origins.data_ptr(),
                                                     grid_u.data_ptr(), dims.ctypes.data, float(dx),
                                                     origin.ctypes.data, out.data_ptr()))
        return out

    def ibm_spread(self, cell_origins, vertex_f, dims, dx, origin, out=None):
        """Force density on the grid from the vertex forces (bitwise reproducible)."""
        self._origins(cell_origins)
        self._check_field(vertex_f, "vertex_f")
        n = int(np.prod(np.asarray(dims, dtype=np.int64)))
        out = torch.empty((3, n), dtype=self.dtype, device=self.pos.device) if out is None else out
        dims, origin = self._grid_args(out, dims, origin)
        _lib.check(_lib.load().npfem_ibm_spread(self.handle, cell_origins.data_ptr(),
                                                vertex_f.data_ptr(), dims.ctypes.data, float(dx),
                                                origin.ctypes.data, out.data_ptr()))
        return out

    def rollout(self, forces: torch.Tensor, dt: float, n_iter: int, n_steps: int, ckpt_every: int):
        """n_steps steps under constant forces, checkpointing every ckpt_every steps."""
        self._check_field(forces, "forces")
        self._forces = forces
        self.rollout_generation += 1
        _lib.check(_lib.load().npfem_rollout(self.handle, forces.data_ptr(), float(dt), int(n_iter),
                                             int(n_steps), int(ckpt_every)))

    def rollout_adjoint(self, dL_dx: torch.Tensor, dL_dv: torch.Tensor = None):
        """Gradients of L(x_T, v_T) of the last rollout:
        (dL/dw [n_cells, 4] float64, dL/dforces, dL/dx0, dL/dv0)."""
        self._check_field(dL_dx, "dL_dx")
        if dL_dv is not None:
            self._check_field(dL_dv, "dL_dv")
        dw = torch.zeros((self.n_cells, 4), dtype=torch.float64, device=self.pos.device)
        df = torch.empty_like(self.pos)
        dx0 = torch.empty_like(self.pos)
        dv0 = torch.empty_like(self.pos)
        _lib.check(_lib.load().npfem_rollout_adjoint(
            self.handle, dL_dx.data_ptr(), None if dL_dv is None else dL_dv.data_ptr(),
            dw.data_ptr(), df.data_ptr(), dx0.data_ptr(), dv0.data_ptr()))
        return dw, df, dx0, dv0

    def _check_field(self, t, name):
        if not (t.is_cuda and t.dtype == self.dtype and t.is_contiguous()
                and tuple(t.shape) == tuple(self.pos.shape)):
            raise ValueError(f"{name} must match pos (contiguous CUDA, same dtype and shape)")

    def energy(self) -> np.ndarray:
        n_it = ctypes.c_int32()
        cap = 1000 * self.n_cells
        buf = np.empty(cap, dtype=np.float64)
        _lib.check(_lib.load().npfem_get_energy(self.handle, buf.ctypes.data, cap,
                                                ctypes.byref(n_it)))
        return buf[: n_it.value * self.n_cells].reshape(n_it.value, self.n_cells).copy()

    def volume(self) -> np.ndarray:
        out = np.empty(self.n_cells, dtype=np.float64)
        _lib.check(_lib.load().npfem_get_volume(self.handle, out.ctypes.data))
        return out

    def config(self, cls=0):
        """(local workgroup size, GEMM tile rows, GEMM tile cols, correction sweeps)."""
        out = np.zeros(4, dtype=np.int32)
        _lib.check(_lib.load().npfem_batch_config(self.handle, int(cls), out.ctypes.data))
        return tuple(int(v) for v in out)

    def set_config(self, cls, cfg):
        """Pin (local workgroup size, GEMM tile rows, GEMM tile cols, sweeps or -1)."""
        arr = np.ascontiguousarray(cfg, dtype=np.int32)
        _lib.check(_lib.load().npfem_set_batch_config(self.handle, int(cls), arr.ctypes.data))

    def kernel_times(self, reset=False):
        """{kind: (total ms, launches)} accumulated from per-kernel HIP events."""
        ms = np.zeros(len(_lib.KERNEL_KINDS), dtype=np.float64)
        n = np.zeros(len(_lib.KERNEL_KINDS), dtype=np.int64)
        _lib.check(_lib.load().npfem_kernel_times(self.handle, ms.ctypes.data, n.ctypes.data,
                                                  1 if reset else 0))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(_lib.KERNEL_KINDS)}

    def close(self):
        if getattr(self, "handle", None):
            _lib.load().npfem_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def meshes_for(susp):
    """Mesh objects for the classes of a workload suspension."""
    return [Mesh(c.rest, c.tris, c.weights, c.mass) for c in susp.classes]


def batch_from_suspension(susp, precision="fp32", device="cuda", per_cell_weights=None, **kw):
    """Uploads a workload suspension; returns (batch, pos, vel, forces, meshes).

    per_cell_weights: None = pass the suspension's weights only when they differ
    from each class's nominal material."""
    dt_ = state_dtype(precision)
    pos = torch.tensor(susp.x0, dtype=dt_, device=device).contiguous()
    vel = torch.tensor(susp.v0, dtype=dt_, device=device).contiguous()
    f = torch.tensor(susp.forces, dtype=dt_, device=device).contiguous()
    meshes = meshes_for(susp)
    if per_cell_weights is None:
        per_cell_weights = not susp.uniform_weights()
    w = susp.weights if per_cell_weights else None
    b = Batch(meshes, susp.cell_class, pos, vel, cell_weights=w, precision=precision, **kw)
    for k, c in enumerate(susp.classes):
        alpha, beta = getattr(c, "damping", (0.0, 0.0))
        if alpha or beta:
            b.set_damping(k, alpha, beta)
    wc = float(susp.extra.get("contact_weight", 0.0))
    if wc and susp.extra.get("contacts") is not None:
        pts, nrm, off = susp.extra["contacts"]
        b.set_contacts(wc, torch.tensor(pts.T, dtype=dt_, device=device).contiguous(),
                       torch.tensor(nrm.T, dtype=dt_, device=device).contiguous(),
                       torch.tensor(off, dtype=torch.int32, device=device).contiguous())
    return b, pos, vel, f, meshes
