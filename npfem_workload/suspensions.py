"""Seeded synthetic cell suspensions (the inputs of every test and benchmark).

A suspension is a batch of cells, each an instance of a mesh class, with an
initial state, external nodal forces standing in for the fluid/IBM coupling,
and per-cell constraint weights. Nothing here computes any projective-dynamics
quantity: the oracle and the HIP library both receive these arrays as inputs.

Layout conventions (shared with the C ABI):

* cells are ordered class-major, then cell-major;
* per-vertex arrays are SoA ``[3][sum_N]`` (all x, then all y, then all z);
* positions are *cell-local*: relative to a per-cell origin kept here in FP64
  (``origins``).  The step is translation-equivariant, so the solver never needs
  the origin; keeping it out of the FP32 coordinates preserves precision.

Workloads follow the benchmark configurations of the solver:

* ``single_rbc``    1 RBC (level-2 Evans-Fung, 162 vertices), FP64 run.
* ``rbc_lattice``   4096 RBCs (642 vertices) on a 16^3 lattice of 10 um,
                    random rotations, shear + noise forces.
* ``uneven``        3000 RBC + 600 platelets (162) + 64 large cells (2562),
                    per-cell weights drawn +-20 %.
* ``adjoint``       1024 RBCs, forces N(0, 0.05^2), stretched target shape.
* ``precision``     16384 RBC + 1638 platelets.

Every workload takes ``n_cells`` overrides so tests can use small samples.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import meshes

NOMINAL_WEIGHTS = (1.0, 1.0, 0.01, 10.0)  # stretch, area, bending, volume
VERTEX_MASS = 1e-3
DT = 1e-4


@dataclass
class MeshClass:
    name: str
    rest: np.ndarray  # [N, 3] float64
    tris: np.ndarray  # [F, 3] int32
    weights: tuple = NOMINAL_WEIGHTS
    mass: float = VERTEX_MASS
    damping: tuple = (0.0, 0.0)  # (alpha, beta) viscous damping coefficients

    @property
    def n_verts(self) -> int:
        return int(self.rest.shape[0])


@dataclass
class Suspension:
    classes: list
    cell_class: np.ndarray  # [C] int32, non-decreasing (class-major)
    origins: np.ndarray  # [C, 3] float64
    x0: np.ndarray  # [3, sum_N] float64, cell-local
    v0: np.ndarray  # [3, sum_N] float64
    forces: np.ndarray  # [3, sum_N] float64, held constant over steps
    weights: np.ndarray  # [C, 4] float64 (stretch, area, bend, volume)
    dt: float = DT
    n_iter: int = 10
    n_steps: int = 100
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.cell_class.shape[0])

    def cell_offsets(self) -> np.ndarray:
        n = np.array([self.classes[k].n_verts for k in self.cell_class], dtype=np.int64)
        return np.concatenate([[0], np.cumsum(n)])

    def cell_slice(self, c: int) -> slice:
        off = self.cell_offsets()
        return slice(int(off[c]), int(off[c + 1]))

    def cell_arrays(self, c: int):
        """(mesh class, x0 [N,3], v0 [N,3], f [N,3], weights[4]) of one cell."""
        s = self.cell_slice(c)
        k = int(self.cell_class[c])
        return (self.classes[k], self.x0[:, s].T.copy(), self.v0[:, s].T.copy(),
                self.forces[:, s].T.copy(), self.weights[c].copy())

    def uniform_weights(self) -> bool:
        for c in range(self.n_cells):
            if not np.array_equal(self.weights[c], np.asarray(self.classes[self.cell_class[c]].weights)):
                return False
        return True

    def subset(self, cells) -> "Suspension":
        """A suspension made of the listed cells (kept in class-major order)."""
        cells = np.sort(np.asarray(cells, dtype=np.int64))
        sl = [self.cell_slice(int(c)) for c in cells]
        cat = lambda a: np.concatenate([a[:, s] for s in sl], axis=1)
        return Suspension(self.classes, self.cell_class[cells].copy(), self.origins[cells].copy(),
                          cat(self.x0), cat(self.v0), cat(self.forces), self.weights[cells].copy(),
                          self.dt, self.n_iter, self.n_steps, self.name + "-subset",
                          dict(self.extra))


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-uniform rotations from the QR factorisation of Gaussian matrices."""
    a = rng.standard_normal((n, 3, 3))
    q, r = np.linalg.qr(a)
    d = np.sign(np.diagonal(r, axis1=1, axis2=2))
    d[d == 0] = 1.0
    q = q * d[:, None, :]
    det = np.linalg.det(q)
    q[det < 0, :, 0] *= -1.0
    return q


def rbc_class(level=3):
    x, f = meshes.rbc_mesh(level)
    return MeshClass(f"rbc{x.shape[0]}", x, f)


def platelet_class(level=2):
    x, f = meshes.platelet_mesh(level)
    return MeshClass(f"plt{x.shape[0]}", x, f)


def large_class(level=4):
    x, f = meshes.sphere_mesh(level)
    return MeshClass(f"large{x.shape[0]}", x, f)


def _assemble(classes, counts, rng, force_fn, weight_jitter=0.0, rotate=True, spacing=10.0):
    """Place cells on a cubic lattice with random rotations; build SoA arrays."""
    cell_class = np.concatenate([np.full(n, k, dtype=np.int32) for k, n in enumerate(counts)])
    n_cells = int(cell_class.shape[0])
    side = int(np.ceil(n_cells ** (1.0 / 3.0) - 1e-9))
    idx = np.arange(n_cells)
    lattice = np.stack([idx % side, (idx // side) % side, idx // (side * side)], axis=1)
    origins = lattice.astype(np.float64) * spacing
    rots = random_rotations(rng, n_cells) if rotate else np.repeat(np.eye(3)[None], n_cells, 0)
    xs, fs = [], []
    for c in range(n_cells):
        mc = classes[cell_class[c]]
        x = mc.rest @ rots[c].T
        xs.append(x)
        fs.append(force_fn(c, x, origins[c]))
    x0 = np.concatenate(xs, axis=0).T.copy()
    forces = np.concatenate(fs, axis=0).T.copy()
    w = np.array([classes[k].weights for k in cell_class], dtype=np.float64)
    if weight_jitter > 0.0:
        w = w * rng.uniform(1.0 - weight_jitter, 1.0 + weight_jitter, size=w.shape)
    return cell_class, origins, x0, np.zeros_like(x0), forces, w


def single_rbc(seed=0, n_steps=100, n_iter=20, dt=DT):
    """One level-2 RBC at its rest shape, forces N(0, 0.05^2) held fixed."""
    rng = np.random.default_rng(seed)
    cls = [rbc_class(2)]
    fn = lambda c, x, o: rng.normal(0.0, 0.05, size=x.shape)
    cc, org, x0, v0, f, w = _assemble(cls, [1], rng, fn, rotate=False)
    return Suspension(cls, cc, org, x0, v0, f, w, dt, n_iter, n_steps, "single_rbc")


def rbc_lattice(n_cells=4096, seed=0, n_steps=200, n_iter=10, dt=DT, shear_rate=100.0,
                drag=1e-4, noise=0.02):
    """RBCs on a 10 um lattice with random rotations.

    Force: a uniform shear about each cell's centroid, f_x = drag * rate *
    (y - y_centroid), plus N(0, noise^2) per component, held constant.
    """
    rng = np.random.default_rng(seed)
    cls = [rbc_class(3)]

    def fn(c, x, o):
        f = rng.normal(0.0, noise, size=x.shape)
        f[:, 0] += drag * shear_rate * (x[:, 1] - x[:, 1].mean())
        return f

    cc, org, x0, v0, f, w = _assemble(cls, [n_cells], rng, fn)
    return Suspension(cls, cc, org, x0, v0, f, w, dt, n_iter, n_steps, "rbc_lattice",
                      {"shear_rate": shear_rate, "drag": drag, "noise": noise})


def uneven(n_rbc=3000, n_plt=600, n_large=64, seed=0, n_steps=100, n_iter=10, dt=DT):
    """Mixed RBC / platelet / large-cell batch with weights jittered +-20 %."""
    rng = np.random.default_rng(seed)
    cls = [rbc_class(3), platelet_class(2), large_class(4)]
    fn = lambda c, x, o: rng.normal(0.0, 0.05, size=x.shape)
    cc, org, x0, v0, f, w = _assemble(cls, [n_rbc, n_plt, n_large], rng, fn,
                                      weight_jitter=0.2, spacing=14.0)
    return Suspension(cls, cc, org, x0, v0, f, w, dt, n_iter, n_steps, "uneven")


def adjoint_rbcs(n_cells=1024, seed=0, n_steps=50, n_iter=10, dt=DT, stretch=1.15):
    """RBCs for gradient checks; ``extra['target']`` is the stretched target.

    Target of cell c = centroid(x0_c) + diag(stretch, 1, 1) (X_rest - centroid(X_rest)),
    i.e. the rest shape stretched along x, unrotated, at the cell's initial centroid.
    """
    rng = np.random.default_rng(seed)
    cls = [rbc_class(3)]
    fn = lambda c, x, o: rng.normal(0.0, 0.05, size=x.shape)
    cc, org, x0, v0, f, w = _assemble(cls, [n_cells], rng, fn)
    rest = cls[0].rest
    rc = rest - rest.mean(axis=0)
    tgt = []
    n = cls[0].n_verts
    for c in range(n_cells):
        cen = x0[:, c * n:(c + 1) * n].mean(axis=1)
        tgt.append(cen[None, :] + rc * np.array([stretch, 1.0, 1.0]))
    target = np.concatenate(tgt, axis=0).T.copy()
    return Suspension(cls, cc, org, x0, v0, f, w, dt, n_iter, n_steps, "adjoint",
                      {"target": target, "ckpt_every": 10})


def precision_sweep(n_rbc=16384, n_plt=1638, seed=0, n_steps=100, n_iter=10, dt=DT):
    """Large RBC + platelet suspension for the precision sweep."""
    rng = np.random.default_rng(seed)
    cls = [rbc_class(3), platelet_class(2)]
    fn = lambda c, x, o: rng.normal(0.0, 0.05, size=x.shape)
    cc, org, x0, v0, f, w = _assemble(cls, [n_rbc, n_plt], rng, fn)
    return Suspension(cls, cc, org, x0, v0, f, w, dt, n_iter, n_steps, "precision")


def stiff(s: Suspension, dt=1e-2, n_steps=None) -> Suspension:
    """Stiff twin: larger time step so elastic terms matter (m/h^2 = 10)."""
    return Suspension(s.classes, s.cell_class, s.origins, s.x0, s.v0, s.forces, s.weights,
                      dt, s.n_iter, s.n_steps if n_steps is None else n_steps,
                      s.name + "-stiff", dict(s.extra))


def sample_cells(s: Suspension, n_per_class, seed=0):
    """Seeded sample of cell indices, up to ``n_per_class[k]`` of each class."""
    rng = np.random.default_rng(seed + 12345)
    out = []
    for k, n in enumerate(n_per_class):
        ids = np.nonzero(s.cell_class == k)[0]
        if len(ids) == 0:
            continue
        out.append(np.sort(rng.choice(ids, size=min(n, len(ids)), replace=False)))
    return np.concatenate(out) if out else np.zeros(0, dtype=np.int64)


def wall_contacts(s: Suspension, depth=0.3, n_grid=9, weight=10.0) -> Suspension:
    """Contact lists of a plane wall under every cell (an obstacle, as in the
    single-RBC obstacle case): the wall's surface cuts `depth` um above the
    cell's lowest vertex; contact points on an n_grid x n_grid grid over the
    cell's footprint, outward normals +z (out of the wall), cell-local
    coordinates. Sets extra['contacts'] = (points [P,3], normals [P,3],
    offsets [C+1]) and extra['contact_weight']."""
    pts, nrm, off = [], [], [0]
    for c in range(s.n_cells):
        x = s.x0[:, s.cell_slice(c)].T
        zmin = x[:, 2].min()
        r = np.abs(x[:, :2]).max()
        g = np.linspace(-r, r, n_grid)
        p2 = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
        pts.append(np.c_[p2, np.full(len(p2), zmin + depth)])
        nrm.append(np.tile([0.0, 0.0, 1.0], (len(p2), 1)))
        off.append(off[-1] + len(p2))
    s.extra["contacts"] = (np.concatenate(pts), np.concatenate(nrm), np.asarray(off, np.int64))
    s.extra["contact_weight"] = float(weight)
    return s


def sphere_contacts(s: Suspension, radius=2.0, overlap=0.3, level=2, weight=10.0) -> Suspension:
    """Contact lists of a spherical obstacle beside every cell: centre on the
    cell's +x side so that the sphere reaches `overlap` um into the cell's
    extent along x; contact points are the vertices of an icosphere of that
    radius with their radial (outward) normals, cell-local coordinates."""
    u, _ = meshes.icosphere(level)
    u = u / np.linalg.norm(u, axis=1, keepdims=True)
    pts, nrm, off = [], [], [0]
    for c in range(s.n_cells):
        x = s.x0[:, s.cell_slice(c)].T
        ctr = np.array([x[:, 0].max() + radius - overlap, x[:, 1].mean(), x[:, 2].mean()])
        pts.append(ctr + radius * u)
        nrm.append(u.copy())
        off.append(off[-1] + len(u))
    s.extra["contacts"] = (np.concatenate(pts), np.concatenate(nrm), np.asarray(off, np.int64))
    s.extra["contact_weight"] = float(weight)
    return s
