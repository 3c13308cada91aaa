"""Quasi-Newton projective dynamics: L-BFGS on the implicit step's objective
with the PD system matrix as initial Hessian (FP64).

Test infrastructure only (see the package docstring).

The solver delivers converged implicit steps rather than a fixed number of
projective-dynamics sweeps: its kernel follows the redesigned PD of Liu et
al., which treats the step as the minimisation of

    g(q) = (m/2h^2)|q - s|^2 + sum_i (w_i/2) dist^2(S_i q, C_i)

by a quasi-Newton method (Implementation and architecture). By the envelope
theorem grad g(q) = A q - b(q), with A the constant PD matrix and b(q) =
(m/h^2) s + sum_i w_i S_i^T P_i(q) the right-hand side of the PD global step
at the projections of q; one PD iteration is the step q - A^-1 grad g(q).
L-BFGS keeps the last `history` pairs (s_k = q_{k+1} - q_k,
y_k = grad_{k+1} - grad_k) and applies the inverse-Hessian estimate by the
standard two-loop recursion with A^-1 in the middle (Nocedal and Wright,
Algorithm 7.4). The step length comes from backtracking on g: alpha = 1, then
halved while g(q + alpha d) > g(q) + c alpha grad^T d (Armijo, c = 1e-4), at
most `max_ls` trials, the last trial taken if none passes. Every iteration
stores its pair in a ring of `history` slots; a pair with y^T s <= 0 gets
rho = 0, which makes it inert in the recursion (reading: the slot is used
all the same, so that every cell's history advances in step). With history 0
and full steps this is plain PD.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import projections as proj
from . import solver as S

ARMIJO_C = 1e-4


def objective_and_gradient(cs: "S.CellSolver", q, s):
    """(g(q), grad g(q)) at iterate q of a step with inertial prediction s."""
    P = proj.local_step(q, cs.o)
    E = S.energy(cs.o, q, s, P, cs.prm)
    return E, cs.A @ q - S.rhs(cs.o, P, s, cs.prm)


def step(cs: "S.CellSolver", x, v, f, n_iter, history=5, max_ls=3, record=False):
    """One implicit step by n_iter L-BFGS iterations from q^0 = s; returns
    (x_new, v_new, objective values of q^0..q^n_iter if record)."""
    if cs.C is not None or cs.wc != 0.0:
        raise ValueError("the quasi-Newton step covers the undamped, contact-free objective")
    h, m = cs.prm.dt, cs.prm.mass
    s = x + h * v + (h * h / m) * f
    q = s.copy()
    E, g = objective_and_gradient(cs, q, s)
    hist = []  # (s_k, y_k, rho_k), oldest first
    trace = [E]
    for _ in range(n_iter):
        # two-loop recursion: d = -H grad
        r = g.copy()
        alphas = []
        for sk, yk, rk in reversed(hist):
            a = rk * np.sum(sk * r)
            alphas.append(a)
            r = r - a * yk
        z = scipy.linalg.cho_solve(cs.chol, r)
        for (sk, yk, rk), a in zip(hist, reversed(alphas)):
            bta = rk * np.sum(yk * z)
            z = z + (a - bta) * sk
        d = -z
        gd = float(np.sum(g * d))
        alpha = 1.0
        for t in range(max_ls):
            qn = q + alpha * d
            En, gn = objective_and_gradient(cs, qn, s)
            if En <= E + ARMIJO_C * alpha * gd or t == max_ls - 1:
                break
            alpha *= 0.5
        sk, yk = qn - q, gn - g
        sy = float(np.sum(sk * yk))
        if history > 0:
            hist.append((sk, yk, 1.0 / sy if sy > 0.0 else 0.0))
            if len(hist) > history:
                hist.pop(0)
        q, E, g = qn, En, gn
        trace.append(E)
    return q, (q - x) / h, (trace if record else None)


def rollout(cs: "S.CellSolver", x0, v0, f, n_iter, n_steps, history=5, max_ls=3):
    x, v = x0.copy(), v0.copy()
    for _ in range(n_steps):
        x, v, _ = step(cs, x, v, f, n_iter, history, max_ls)
    return x, v
