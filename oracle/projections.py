"""Local step of projective dynamics: exact closest-point projections (FP64).

Test infrastructure only (see the package docstring).

Each elemental potential is (w/2) dist^2(S_i q, C_i); the local step replaces
S_i q by its closest point in the constraint set C_i:

* strain  C = {3x2 matrices with orthonormal columns}: the polar factor U V^T
  of F = U diag(s1, s2) V^T (thin SVD);
* area    C = {3x2 matrices with s1 * s2 = 1}: U diag(t, 1/t) V^T where t > 0
  minimises (t - s1)^2 + (1/t - s2)^2, i.e. a positive real root of
  t^4 - s1 t^3 + s2 t - 1 = 0 (smallest objective, then smallest t);
* bending C = {y : |y| = r_e} for the stencil vector y = sum_r K_e[r] q_r:
  r_e y / |y| (y itself when |y| = 0);
* volume  C = {p : V(p) = V_rest} on the whole cell: closest point reached by
  repeatedly projecting q on the constraint linearised at the current iterate,
  p <- q + lam grad V(p), lam = (V_rest - V(p) - grad V(p).(q - p)) / |grad V(p)|^2.
"""
from __future__ import annotations

import numpy as np

from . import operators as ops_mod

DEGENERATE_RATIO = 1e-12


class DegenerateElement(FloatingPointError):
    pass


def thin_svd(F: np.ndarray):
    """Batched thin SVD of [n, 3, 2] matrices (sigma descending)."""
    U, s, Vt = np.linalg.svd(F, full_matrices=False)
    if np.any(s[:, 1] < DEGENERATE_RATIO * s[:, 0]):
        raise DegenerateElement("degenerate (collapsed) triangle in the local step")
    return U, s, Vt


def project_strain(U, s, Vt):
    """Strain target: the polar factor U V^T of F = U diag(s) V^T, the
    nearest 3x2 matrix with orthonormal columns (reading: exact projection,
    as in classic projective dynamics; the paper prints no formula)."""
    return U @ Vt


def area_root(s1: np.ndarray, s2: np.ndarray) -> np.ndarray:
    """Positive real root t of t^4 - s1 t^3 + s2 t - 1 minimising
    (t - s1)^2 + (1/t - s2)^2 (ties: smaller t). Reading: the area target is
    the nearest matrix with singular values (t, 1/t), i.e. with unit area
    ratio; the quartic is the stationarity condition of that distance.

    Roots are the eigenvalues of the quartic's companion matrix (what
    ``numpy.roots`` computes), batched; each real root gets one Newton polish.
    """
    n = s1.shape[0]
    C = np.zeros((n, 4, 4))
    # monic t^4 + a3 t^3 + a2 t^2 + a1 t + a0 with a3 = -s1, a2 = 0, a1 = s2, a0 = -1
    C[:, 0, 0] = s1
    C[:, 0, 1] = 0.0
    C[:, 0, 2] = -s2
    C[:, 0, 3] = 1.0
    C[:, 1, 0] = 1.0
    C[:, 2, 1] = 1.0
    C[:, 3, 2] = 1.0
    lam = np.linalg.eigvals(C)
    re, im = lam.real, lam.imag
    ok = (np.abs(im) <= 1e-7 * np.maximum(1.0, np.abs(re))) & (re > 0.0)
    t = np.where(ok, re, np.nan)
    p = t ** 4 - s1[:, None] * t ** 3 + s2[:, None] * t - 1.0
    dp = 4.0 * t ** 3 - 3.0 * s1[:, None] * t ** 2 + s2[:, None]
    with np.errstate(invalid="ignore", divide="ignore"):
        tp = t - p / dp
    t = np.where(np.isfinite(tp) & (tp > 0.0), tp, t)
    obj = (t - s1[:, None]) ** 2 + (1.0 / t - s2[:, None]) ** 2
    obj = np.where(ok, obj, np.inf)
    best = np.full(n, np.inf)
    tbest = np.full(n, np.nan)
    for j in np.argsort(np.where(ok, t, np.inf), axis=1).T:  # ascending t
        oj = obj[np.arange(n), j]
        tj = t[np.arange(n), j]
        better = oj < best * (1.0 - 1e-14) - 1e-300
        best = np.where(better, oj, best)
        tbest = np.where(better, tj, tbest)
    if np.any(~np.isfinite(tbest)):
        raise DegenerateElement("no positive root for the area projection")
    return tbest


def project_area(U, s, Vt):
    """Area target U diag(t, 1/t) V^T with t from area_root."""
    t = area_root(s[:, 0], s[:, 1])
    d = np.stack([t, 1.0 / t], axis=1)
    return U @ (d[:, :, None] * Vt)


def bending_vectors(q: np.ndarray, H: np.ndarray, K: np.ndarray) -> np.ndarray:
    """y_e = sum_r K_e[r] q_{H_e[r]} -> [E, 3]."""
    return np.einsum("er,erd->ed", K, q[H])


def project_bending(y: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Bending target: y rescaled to its rest magnitude r (reading: the
    hinge keeps the rest length of its cotangent stencil vector; y itself
    where |y| = 0, where every direction is equally near)."""
    n = np.linalg.norm(y, axis=1)
    out = y.copy()
    nz = n > 0.0
    out[nz] = (r[nz] / n[nz])[:, None] * y[nz]
    return out


def project_volume(q: np.ndarray, tris: np.ndarray, vol_rest: float, radius: float,
                   max_iter: int = 100, vol_tol: float = 1e-13, step_tol: float = 1e-15):
    """Closest point to q on {V(p) = vol_rest}; returns (p, iterations used).

    Reading: the volume constraint acts on the whole cell and its target is
    the exact closest point (the KKT point p = q + lam grad V(p)), reached by
    iterating that fixed-point map from p = q until the volume matches to
    vol_tol and the iterate has settled to step_tol of the cell radius."""
    p = q.copy()
    for it in range(1, max_iter + 1):
        g = ops_mod.volume_gradient(p, tris)
        V = ops_mod.volume(p, tris)
        lam = (vol_rest - V - np.sum(g * (q - p))) / np.sum(g * g)
        p_new = q + lam * g
        dp = np.max(np.abs(p_new - p))
        p = p_new
        if abs(ops_mod.volume(p, tris) - vol_rest) <= vol_tol * abs(vol_rest) and dp <= step_tol * radius:
            return p, it
    return p, max_iter


def local_step(q: np.ndarray, o: "ops_mod.CellOperators"):
    """All projections for one cell at iterate q [N, 3]."""
    F = ops_mod.deformation_gradients(q, o.tris, o.G)
    U, s, Vt = thin_svd(F)
    Ps = project_strain(U, s, Vt)
    Pa = project_area(U, s, Vt)
    y = bending_vectors(q, o.H, o.K)
    Pb = project_bending(y, o.r)
    Pv, nv = project_volume(q, o.tris, o.vol_rest, o.radius)
    return {"F": F, "Ps": Ps, "Pa": Pa, "y": y, "Pb": Pb, "Pv": Pv, "n_vol": nv}
