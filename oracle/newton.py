"""Brute-force minimiser of the implicit-step objective (pins PD convergence).

Test infrastructure only (see the package docstring).

The solver is meant to deliver a converged implicit step rather than an
approximation of it (Implementation and architecture). The converged step
minimises

    E_true(q) = (m/2h^2)|q - s|^2 + sum_i (w_i/2) dist^2(S_i q, C_i),

whose gradient, by the envelope theorem, is

    (m/h^2)(q - s) + sum_t w_s A_t G_t (F_t - Ps_t)^T + w_a A_t G_t (F_t - Pa_t)^T
                   + sum_e w_b c_e K_e (x) (y_e - Pb_e) + w_v (q - Pv).

This module evaluates that gradient element by element (it does not use the
assembled system matrix), builds a Hessian from central differences of it and
runs damped Newton. A projective-dynamics rollout with enough iterations must
land on the same minimiser.
"""
from __future__ import annotations

import numpy as np

from . import projections as proj


def objective(o, q, s, prm) -> float:
    ws, wa, wb, wv = prm.weights
    P = proj.local_step(q, o)
    e = 0.5 * prm.mass / prm.dt ** 2 * np.sum((q - s) ** 2)
    e += np.sum(0.5 * o.area * (ws * np.sum((P["F"] - P["Ps"]) ** 2, axis=(1, 2))
                                + wa * np.sum((P["F"] - P["Pa"]) ** 2, axis=(1, 2))))
    e += np.sum(0.5 * wb * o.c * np.sum((P["y"] - P["Pb"]) ** 2, axis=1))
    e += 0.5 * wv * np.sum((q - P["Pv"]) ** 2)
    return float(e)


def gradient(o, q, s, prm) -> np.ndarray:
    ws, wa, wb, wv = prm.weights
    P = proj.local_step(q, o)
    g = (prm.mass / prm.dt ** 2) * (q - s)
    R = o.area[:, None, None] * (ws * (P["F"] - P["Ps"]) + wa * (P["F"] - P["Pa"]))
    for t in range(o.tris.shape[0]):
        for r in range(3):
            g[o.tris[t, r]] += R[t] @ o.G[t, r]
    dy = P["y"] - P["Pb"]
    for e in range(o.H.shape[0]):
        for r in range(4):
            g[o.H[e, r]] += wb * o.c[e] * o.K[e, r] * dy[e]
    g += wv * (q - P["Pv"])
    return g


def minimise(o, s, prm, q0=None, tol=1e-12, max_iter=50, fd_step=1e-6):
    """Newton with a finite-difference Hessian; returns (q, |grad|_inf)."""
    q = s.copy() if q0 is None else q0.copy()
    n = q.size
    for _ in range(max_iter):
        g = gradient(o, q, s, prm).ravel()
        gn = np.max(np.abs(g))
        if gn <= tol:
            return q, gn
        Hm = np.empty((n, n))
        for i in range(n):
            dq = np.zeros(n)
            dq[i] = fd_step
            gp = gradient(o, q + dq.reshape(q.shape), s, prm).ravel()
            gm = gradient(o, q - dq.reshape(q.shape), s, prm).ravel()
            Hm[:, i] = (gp - gm) / (2.0 * fd_step)
        Hm = 0.5 * (Hm + Hm.T)
        step = np.linalg.solve(Hm, -g)
        e0 = objective(o, q, s, prm)
        alpha = 1.0
        while alpha > 1e-8:
            qn = q + alpha * step.reshape(q.shape)
            if objective(o, qn, s, prm) <= e0 + 1e-14 * abs(e0):
                break
            alpha *= 0.5
        q = qn
    g = gradient(o, q, s, prm).ravel()
    return q, float(np.max(np.abs(g)))
