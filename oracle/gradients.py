"""Finite-difference gradients of rollout losses through the FP64 oracle.

Test infrastructure only (see the package docstring).

For calibrating membrane moduli the quantity of interest is the gradient of
a loss of the final positions, L = sum_v |x_T,v - target_v|^2, with respect
to a cell's constraint weights (w_stretch, w_area, w_bend, w_volume) and the
constant external nodal forces. Central differences of the oracle's rollout
are the plain definition of those derivatives; each cell is independent, so
one cell is rolled out at a time.
"""
from __future__ import annotations

import numpy as np

from . import solver as S


def rollout(mesh_class, weights, mass, dt, x0, v0, f, n_iter, n_steps):
    o = S.operators_for(mesh_class)
    cs = S.CellSolver(o, S.Params(tuple(float(w) for w in weights), mass, dt))
    return cs.rollout(x0, v0, f, n_iter, n_steps)


def loss(mesh_class, weights, mass, dt, x0, v0, f, target, n_iter, n_steps):
    x, _ = rollout(mesh_class, weights, mass, dt, x0, v0, f, n_iter, n_steps)
    return float(np.sum((x - target) ** 2))


def fd_weight_grad(mesh_class, weights, mass, dt, x0, v0, f, target, n_iter, n_steps,
                   h=1e-3, which=(0, 1, 2, 3)):
    """Central differences dL/dw_i with the step h |w_i| relative to each
    weight (h itself for a zero weight): the weights span three decades
    (bending 0.01, volume 10), and an absolute step of 1e-3 would be 10 % of
    the bending weight."""
    w = np.asarray(weights, dtype=np.float64)
    g = np.zeros(4)
    for i in which:
        hi = h * abs(w[i]) if w[i] != 0.0 else h
        wp, wm = w.copy(), w.copy()
        wp[i] += hi
        wm[i] -= hi
        lp = loss(mesh_class, wp, mass, dt, x0, v0, f, target, n_iter, n_steps)
        lm = loss(mesh_class, wm, mass, dt, x0, v0, f, target, n_iter, n_steps)
        g[i] = (lp - lm) / (2.0 * hi)
    return g


def fd_force_grad(mesh_class, weights, mass, dt, x0, v0, f, target, n_iter, n_steps, comps,
                  h=1e-3):
    """Central differences dL/df for the listed (vertex, axis) components."""
    out = []
    for v, d in comps:
        fp, fm = f.copy(), f.copy()
        fp[v, d] += h
        fm[v, d] -= h
        lp = loss(mesh_class, weights, mass, dt, x0, v0, fp, target, n_iter, n_steps)
        lm = loss(mesh_class, weights, mass, dt, x0, v0, fm, target, n_iter, n_steps)
        out.append((lp - lm) / (2.0 * h))
    return np.asarray(out)
