"""Immersed-boundary transfer between the fluid grid and the membrane
vertices (FP64).

Test infrastructure only (see the package docstring).

The fluid and the solids exchange data through the interpolation kernels of
the immersed boundary method (Introduction: the IBM computes the body force b
of eqs. 1 and 2, and the data exchange between the grid and the surface
meshes goes through interpolation kernels). Reading: Peskin's 4-point
regularised delta function on a periodic Cartesian grid,

    phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4 r^2)) / 8,   |r| <= 1
           = (5 - 2|r| - sqrt(-7 + 12|r| - 4 r^2)) / 8, 1 <= |r| <= 2
           = 0 otherwise,
    delta_h(x) = phi(x/dx) phi(y/dx) phi(z/dx) / dx^3,

velocity interpolation U(X) = sum_g u_g delta_h(x_g - X) dx^3 and force
spreading f_g = sum_v F_v delta_h(x_g - X_v) (a force density on the grid).
Grid node (i, j, k) sits at origin + dx (i, j, k), indices periodic in
n = (nx, ny, nz); fields are [3, nx, ny, nz] (x fastest in the GPU's flat
layout i + nx (j + ny k)). Vertex positions are global: the cell's origin plus
its cell-local coordinates.
"""
from __future__ import annotations

import numpy as np


def phi(r: np.ndarray) -> np.ndarray:
    """Peskin's 4-point kernel."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a <= 2.0)
    out[m1] = (3.0 - 2.0 * a[m1] + np.sqrt(1.0 + 4.0 * a[m1] - 4.0 * a[m1] ** 2)) / 8.0
    out[m2] = (5.0 - 2.0 * a[m2] - np.sqrt(np.maximum(-7.0 + 12.0 * a[m2] - 4.0 * a[m2] ** 2, 0.0))) / 8.0
    return out


def _support(X: np.ndarray, origin, dx):
    """Per vertex: the 4 node indices per axis around it and their weights."""
    s = (X - np.asarray(origin)[None, :]) / dx  # [V, 3] in grid units
    i0 = np.floor(s).astype(np.int64) - 1  # nodes i0 .. i0 + 3
    idx = i0[:, :, None] + np.arange(4)[None, None, :]  # [V, 3, 4]
    w = phi(s[:, :, None] - idx)  # [V, 3, 4]
    return idx, w


def interpolate(u: np.ndarray, X: np.ndarray, origin, dx) -> np.ndarray:
    """U(X_v) = sum over the 4^3 nodes around X_v of u_g phi phi phi; u [3, nx, ny, nz]."""
    n = u.shape[1:]
    idx, w = _support(X, origin, dx)
    out = np.zeros((X.shape[0], 3))
    for a in range(4):
        for b in range(4):
            for c in range(4):
                wt = w[:, 0, a] * w[:, 1, b] * w[:, 2, c]
                ii = idx[:, 0, a] % n[0]
                jj = idx[:, 1, b] % n[1]
                kk = idx[:, 2, c] % n[2]
                out += wt[:, None] * u[:, ii, jj, kk].T
    return out


def spread(F: np.ndarray, X: np.ndarray, shape, origin, dx) -> np.ndarray:
    """f_g = sum_v F_v phi phi phi / dx^3 on the periodic grid -> [3, nx, ny, nz]."""
    f = np.zeros((3,) + tuple(shape))
    idx, w = _support(X, origin, dx)
    for a in range(4):
        for b in range(4):
            for c in range(4):
                wt = w[:, 0, a] * w[:, 1, b] * w[:, 2, c] / dx ** 3
                ii = idx[:, 0, a] % shape[0]
                jj = idx[:, 1, b] % shape[1]
                kk = idx[:, 2, c] % shape[2]
                for d in range(3):
                    np.add.at(f[d], (ii, jj, kk), wt * F[:, d])
    return f


def interpolate_direct(u: np.ndarray, X: np.ndarray, origin, dx) -> np.ndarray:
    """The same sum over every grid node (no support bookkeeping), with the
    minimum-image periodic distance; for tiny grids."""
    n = np.array(u.shape[1:])
    g = np.stack(np.meshgrid(*[np.arange(k) for k in n], indexing="ij"), -1).reshape(-1, 3)
    xg = np.asarray(origin)[None, :] + dx * g
    L = dx * n
    out = np.zeros((X.shape[0], 3))
    uf = u.reshape(3, -1)
    for v in range(X.shape[0]):
        d = X[v][None, :] - xg
        d -= L * np.round(d / L)
        wt = np.prod(phi(d / dx), axis=1)
        out[v] = uf @ wt
    return out
