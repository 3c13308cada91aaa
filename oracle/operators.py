"""Rest-shape operators and the global system matrix (FP64, plain numpy).

Test infrastructure only (see the package docstring).

Per triangle t = (a, b, c) (mass-lumped linear FE on a triangulated surface,
Introduction):
    e1 = X_b - X_a, e2 = X_c - X_a, n = e1 x e2, area A_t = |n| / 2,
    u = e1/|e1|, w = n_hat x u, D = [[u.e1, u.e2], [w.e1, w.e2]],
    G_t = [[-1,-1],[1,0],[0,1]] D^-1          (3 x 2)
so that the deformation gradient is F_t(q) = sum_r q_{t_r} (x) G_t[r, :]
(3 x 2) and F_t(X_rest) = [u w] has orthonormal columns.

Per hinge e = (i, j, k, l) (edge i-j shared by triangles (i, j, k), where the
edge runs i->j, and (j, i, l)): the cotangent bending stencil
    K_e = [c03 + c04, c01 + c02, -(c01 + c03), -(c02 + c04)]
with c01 = cot angle_i(ijk), c02 = cot angle_i(ijl), c03 = cot angle_j(ijk),
c04 = cot angle_j(ijl), weight c_e = 3 / (A_ijk + A_ijl) and rest magnitude
r_e = |sum_r K_e[r] X_r|.

System matrix (projective-dynamics global step, same for x, y and z):
    A = (m/h^2) I + sum_t (w_s + w_a) A_t G_t G_t^T + sum_e w_b c_e K_e K_e^T
        + w_v I.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg


class MeshError(ValueError):
    pass


def check_closed_manifold(tris: np.ndarray, n_verts: int) -> None:
    """Every undirected edge in exactly two triangles with opposite directions,
    every vertex used, and Euler characteristic V - E + F = 2."""
    tris = np.asarray(tris)
    if tris.ndim != 2 or tris.shape[1] != 3:
        raise MeshError("triangles must be [F, 3]")
    if tris.min() < 0 or tris.max() >= n_verts:
        raise MeshError("vertex index out of range")
    directed = {}
    for t, (a, b, c) in enumerate(tris):
        if a == b or b == c or a == c:
            raise MeshError(f"triangle {t} repeats a vertex")
        for u, v in ((a, b), (b, c), (c, a)):
            if (u, v) in directed:
                raise MeshError(f"directed edge {u}->{v} used twice (non-manifold or flipped)")
            directed[(u, v)] = t
    for (u, v) in directed:
        if (v, u) not in directed:
            raise MeshError(f"edge {u}-{v} has one triangle (open mesh)")
    used = np.zeros(n_verts, dtype=bool)
    used[tris.ravel()] = True
    if not used.all():
        raise MeshError("unreferenced vertex")
    n_edges = len(directed) // 2
    if n_verts - n_edges + len(tris) != 2:
        raise MeshError("Euler characteristic is not 2")


def hinges(tris: np.ndarray) -> np.ndarray:
    """[E, 4] hinges (i, j, k, l), one per undirected edge, with i < j.

    k is the third vertex of the triangle in which the edge runs i -> j, l the
    third vertex of the triangle in which it runs j -> i."""
    third = {}
    for a, b, c in np.asarray(tris):
        third[(a, b)] = c
        third[(b, c)] = a
        third[(c, a)] = b
    out = []
    for (u, v), k in third.items():
        if u < v:
            out.append((u, v, k, third[(v, u)]))
    out.sort()
    return np.asarray(out, dtype=np.int64)


def triangle_operators(X: np.ndarray, tris: np.ndarray):
    """(G [F, 3, 2], rest areas [F])."""
    a, b, c = X[tris[:, 0]], X[tris[:, 1]], X[tris[:, 2]]
    e1, e2 = b - a, c - a
    n = np.cross(e1, e2)
    nn = np.linalg.norm(n, axis=1)
    area = 0.5 * nn
    if np.any(area <= 0.0):
        raise MeshError("degenerate rest triangle")
    u = e1 / np.linalg.norm(e1, axis=1, keepdims=True)
    w = np.cross(n / nn[:, None], u)
    D = np.empty((len(tris), 2, 2))
    D[:, 0, 0] = np.einsum("ij,ij->i", u, e1)
    D[:, 0, 1] = np.einsum("ij,ij->i", u, e2)
    D[:, 1, 0] = np.einsum("ij,ij->i", w, e1)
    D[:, 1, 1] = np.einsum("ij,ij->i", w, e2)
    S = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    G = S[None, :, :] @ np.linalg.inv(D)
    return G, area


def deformation_gradients(q: np.ndarray, tris: np.ndarray, G: np.ndarray) -> np.ndarray:
    """F_t(q) = sum_r q_{t_r} (x) G_t[r, :] -> [F, 3, 2]."""
    Q = q[tris]  # [F, 3 vertices, 3 xyz]
    return np.einsum("frd,frk->fdk", Q, G)


def _cot(p, a, b):
    """Cotangent of the angle at p between p->a and p->b."""
    u, v = a - p, b - p
    return np.einsum("ij,ij->i", u, v) / np.linalg.norm(np.cross(u, v), axis=1)


def hinge_operators(X: np.ndarray, H: np.ndarray):
    """(K [E, 4], c [E], rest magnitude r [E])."""
    xi, xj, xk, xl = (X[H[:, r]] for r in range(4))
    c01 = _cot(xi, xj, xk)
    c02 = _cot(xi, xj, xl)
    c03 = _cot(xj, xi, xk)
    c04 = _cot(xj, xi, xl)
    K = np.stack([c03 + c04, c01 + c02, -(c01 + c03), -(c02 + c04)], axis=1)
    a1 = 0.5 * np.linalg.norm(np.cross(xj - xi, xk - xi), axis=1)
    a2 = 0.5 * np.linalg.norm(np.cross(xj - xi, xl - xi), axis=1)
    c = 3.0 / (a1 + a2)
    y = np.einsum("er,erd->ed", K, X[H])
    r = np.linalg.norm(y, axis=1)
    return K, c, r


def volume(q: np.ndarray, tris: np.ndarray) -> float:
    """Enclosed volume (1/6) sum_t q_a . (q_b x q_c)."""
    a, b, c = q[tris[:, 0]], q[tris[:, 1]], q[tris[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def volume_gradient(q: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """dV/dq_v = (1/6) sum over incident triangles of (q_b x q_c), (v, b, c) cyclic."""
    a, b, c = q[tris[:, 0]], q[tris[:, 1]], q[tris[:, 2]]
    g = np.zeros_like(q)
    np.add.at(g, tris[:, 0], np.cross(b, c))
    np.add.at(g, tris[:, 1], np.cross(c, a))
    np.add.at(g, tris[:, 2], np.cross(a, b))
    return g / 6.0


def surface_area(q: np.ndarray, tris: np.ndarray) -> float:
    a, b, c = q[tris[:, 0]], q[tris[:, 1]], q[tris[:, 2]]
    return float(0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1).sum())


@dataclass
class CellOperators:
    """Everything the oracle precomputes for one mesh class."""
    X: np.ndarray
    tris: np.ndarray
    G: np.ndarray
    area: np.ndarray
    H: np.ndarray
    K: np.ndarray
    c: np.ndarray
    r: np.ndarray
    vol_rest: float
    radius: float  # max distance of a rest vertex from the rest centroid

    @property
    def n_verts(self) -> int:
        return self.X.shape[0]


def build_operators(X: np.ndarray, tris: np.ndarray) -> CellOperators:
    X = np.asarray(X, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    check_closed_manifold(tris, X.shape[0])
    G, area = triangle_operators(X, tris)
    H = hinges(tris)
    K, c, r = hinge_operators(X, H)
    rad = float(np.linalg.norm(X - X.mean(axis=0), axis=1).max())
    return CellOperators(X, tris, G, area, H, K, c, r, volume(X, tris), rad)


def laplacians(ops: CellOperators):
    """(L_tri = sum_t A_t G_t G_t^T, L_bend = sum_e c_e K_e K_e^T) as dense N x N."""
    n = ops.n_verts
    Lt = np.zeros((n, n))
    blocks = ops.area[:, None, None] * np.einsum("frk,fsk->frs", ops.G, ops.G)
    for r in range(3):
        for s in range(3):
            np.add.at(Lt, (ops.tris[:, r], ops.tris[:, s]), blocks[:, r, s])
    Lb = np.zeros((n, n))
    kb = ops.c[:, None, None] * ops.K[:, :, None] * ops.K[:, None, :]
    for r in range(4):
        for s in range(4):
            np.add.at(Lb, (ops.H[:, r], ops.H[:, s]), kb[:, r, s])
    return Lt, Lb


def system_matrix(ops: CellOperators, weights, mass: float, dt: float) -> np.ndarray:
    """A = (m/h^2 + w_v) I + (w_s + w_a) L_tri + w_b L_bend (lumped, uniform
    vertex mass; the volume constraint's selection matrix is the identity,
    unscaled: readings that match the right-hand side)."""
    ws, wa, wb, wv = (float(w) for w in weights)
    Lt, Lb = laplacians(ops)
    n = ops.n_verts
    return (mass / dt ** 2 + wv) * np.eye(n) + (ws + wa) * Lt + wb * Lb


def factor(A: np.ndarray):
    """Cholesky factor (raises numpy.linalg.LinAlgError if A is not SPD)."""
    return scipy.linalg.cho_factor(A, lower=True)
