"""Synthetic closed triangulated membranes used as cell rest shapes.

This module only builds geometry (vertex coordinates and triangle lists). It
holds none of the projective-dynamics arithmetic: operators, projections and
solves live separately in the oracle and in the HIP library.

The paper's own RBC/PLT template meshes (258 and 66 vertices, section
"Setting up new materials") are not available; the stand-ins are icospheres of
subdivision level L (10*4^L + 2 vertices, 20*4^L triangles) mapped to

* an Evans-Fung biconcave red blood cell (the paper generates RBC surfaces
  from analytic formulas, section "Rhino-Grasshopper environment"),
* an oblate ellipsoid platelet,
* a sphere (the "large cell" class).

All triangle lists are consistently oriented, counter-clockwise seen from
outside, so that the signed volume is positive.
"""
from __future__ import annotations

import numpy as np

# Evans-Fung shape coefficients (RBC thickness profile) and the RBC radius in um.
EVANS_FUNG_C = (0.207161, 2.002558, -1.122762)
RBC_RADIUS_UM = 3.91


def icosahedron():
    """Regular icosahedron on the unit sphere, outward CCW triangles."""
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array(
        [
            [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
            [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
            [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1],
        ],
        dtype=np.float64,
    )
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(
        [
            [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
            [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
            [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
            [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
        ],
        dtype=np.int32,
    )
    return v, f


def icosphere(level: int):
    """Unit icosphere by repeated 4-to-1 midpoint subdivision."""
    v, f = icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def midpoint(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                m = (np.asarray(verts[a]) + np.asarray(verts[b])) * 0.5
                m /= np.linalg.norm(m)
                verts.append(tuple(m))
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        nf = []
        for a, b, c in f:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = np.asarray(nf, dtype=np.int32)
    return np.asarray(verts, dtype=np.float64), f


def evans_fung(unit_xyz: np.ndarray, radius: float = RBC_RADIUS_UM) -> np.ndarray:
    """Map unit-sphere points onto the Evans-Fung biconcave disc.

    x, y scale by the radius; z = sign(z) * (R/2) * sqrt(1 - rho^2) *
    (c0 + c1 rho^2 + c2 rho^4) with rho^2 = x^2 + y^2 on the unit sphere.
    """
    x, y, z = unit_xyz[:, 0], unit_xyz[:, 1], unit_xyz[:, 2]
    rho2 = np.clip(x * x + y * y, 0.0, 1.0)
    c0, c1, c2 = EVANS_FUNG_C
    h = 0.5 * radius * np.sqrt(1.0 - rho2) * (c0 + c1 * rho2 + c2 * rho2 * rho2)
    return np.stack([radius * x, radius * y, np.sign(z) * h], axis=1)


def rbc_mesh(level: int = 3):
    """Biconcave RBC: level-2 -> 162 vertices, level-3 -> 642."""
    u, f = icosphere(level)
    return evans_fung(u), f


def platelet_mesh(level: int = 2, semi_axes=(1.8, 1.8, 0.5)):
    """Oblate ellipsoid platelet (semi-axes in um)."""
    u, f = icosphere(level)
    return u * np.asarray(semi_axes, dtype=np.float64)[None, :], f


def sphere_mesh(level: int = 4, radius: float = 6.0):
    """Spherical large cell (level-4 -> 2562 vertices)."""
    u, f = icosphere(level)
    return u * radius, f
