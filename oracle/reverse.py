"""Reverse-mode FP64 gradient of a rollout loss through the oracle's step.

Test infrastructure only (see the package docstring).

For calibrating membrane moduli (section "Setting up new materials": the body
energy is a weighted sum of elemental potentials whose weights are fitted)
the quantity of interest is the gradient of a loss of the final positions,
L = sum_v |x_T,v - target_v|^2, with respect to a cell's constraint weights
(w_stretch, w_area, w_bend, w_volume), the constant external nodal forces and
the initial state. Here that gradient is taken by reverse-mode automatic
differentiation (PyTorch autograd on the CPU, float64) of a transcription of
the oracle's time step (``solver.CellSolver.step``), in the same order:

    s = x + h v + (h^2/m) f,  q = s
    repeat n_iter: P = projections(q); q = A(w)^-1 ((m/h^2) s + sum_i w_i S_i^T P_i)
    x' = q,  v' = (q - x)/h

Only the projections are written in forms whose derivatives exist where the
singular values of a triangle coincide (at and near rest, where the SVD's
singular vectors are not differentiable):

* strain  Ps = U V^T = F (F^T F)^{-1/2}, with the 2x2 matrix square root of an
  SPD matrix S in closed form (Cayley-Hamilton): sqrt(S) = (S + sqrt(det S) I)
  / sqrt(tr S + 2 sqrt(det S));
* area    Pa = U diag(d) V^T = F V diag(d/s) V^T. The stationarity conditions
  of |d - s|^2/2 - mu (d1 d2 - 1) give d_i = (s_i + mu s_j)/(1 - mu^2), so
  d_i/s_i = (1 + mu J/s_i^2)/(1 - mu^2) with J = s1 s2, and
  V diag(1/s_i^2) V^T = S^-1: Pa = F (I + mu J S^-1)/(1 - mu^2). The
  multiplier's value is the one the oracle's projection selects,
  mu = t (t - s1) with t from ``projections.area_root``; its derivative
  follows from the constraint g(mu) = (1 - mu^2)^2 - J (1 + mu^2) - mu I1 = 0
  (I1 = tr S) by the implicit function theorem, realised as one Newton step
  from the detached root (value unchanged, derivative -g_theta / g_mu);
* bending Pb = r y/|y| (differentiable for |y| > 0);
* volume  the oracle's fixed-point iteration p <- q + lam grad V(p),
  transcribed and differentiated as iterated (its derivative converges with
  the iterates to that of the exact closest point).

Memory: the time loop is differentiated step by step (the forward stores the
state before every step; the reverse re-runs one step with autograd and pulls
the adjoint of its output back), so only one step's graph is alive.
"""
from __future__ import annotations

import numpy as np
import torch

from . import operators as ops_mod
from . import projections as proj

DT = torch.float64


def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=DT)


class TorchCell:
    """The oracle's rest operators of one mesh class as float64 tensors."""

    def __init__(self, o: ops_mod.CellOperators):
        self.o = o
        self.n = o.n_verts
        self.tris = torch.as_tensor(o.tris, dtype=torch.long)
        self.G = _t(o.G)
        self.area = _t(o.area)
        self.H = torch.as_tensor(o.H, dtype=torch.long)
        self.K = _t(o.K)
        self.c = _t(o.c)
        self.r = _t(o.r)
        self.vol_rest = float(o.vol_rest)
        self.radius = float(o.radius)
        Lt, Lb = ops_mod.laplacians(o)
        self.Lt = _t(Lt)
        self.Lb = _t(Lb)


def deformation_gradients(q, ct: TorchCell):
    """F_t = sum_r q_{t_r} (x) G_t[r, :] -> [F, 3, 2]."""
    return torch.einsum("frd,frk->fdk", q[ct.tris], ct.G)


def _sym2_inverse(S):
    det = S[:, 0, 0] * S[:, 1, 1] - S[:, 0, 1] * S[:, 1, 0]
    inv = torch.stack([torch.stack([S[:, 1, 1], -S[:, 0, 1]], -1),
                       torch.stack([-S[:, 1, 0], S[:, 0, 0]], -1)], -2)
    return inv / det[:, None, None]


def strain_targets(F):
    """Ps = F (F^T F)^{-1/2} (the polar factor U V^T)."""
    S = F.transpose(1, 2) @ F
    J = torch.sqrt(S[:, 0, 0] * S[:, 1, 1] - S[:, 0, 1] * S[:, 1, 0])
    I1 = S[:, 0, 0] + S[:, 1, 1]
    eye = torch.eye(2, dtype=DT).expand_as(S)
    sqrtS = (S + J[:, None, None] * eye) / torch.sqrt(I1 + 2.0 * J)[:, None, None]
    return F @ _sym2_inverse(sqrtS)


def area_targets(F):
    """Pa = F (I + mu J S^-1)/(1 - mu^2), mu the oracle projection's multiplier."""
    S = F.transpose(1, 2) @ F
    J = torch.sqrt(S[:, 0, 0] * S[:, 1, 1] - S[:, 0, 1] * S[:, 1, 0])
    I1 = S[:, 0, 0] + S[:, 1, 1]
    with torch.no_grad():
        _, s, _ = proj.thin_svd(F.detach().numpy())
        t = proj.area_root(s[:, 0], s[:, 1])
        mu0 = _t(t * (t - s[:, 0]))
    u = 1.0 - mu0 * mu0
    g = u * u - J * (1.0 + mu0 * mu0) - mu0 * I1
    dg = -4.0 * mu0 * u - 2.0 * J * mu0 - I1
    mu = mu0 - g / dg
    eye = torch.eye(2, dtype=DT).expand_as(S)
    M = (eye + (mu * J)[:, None, None] * _sym2_inverse(S)) / (1.0 - mu * mu)[:, None, None]
    return F @ M


def bending_vectors(q, ct: TorchCell):
    return torch.einsum("er,erd->ed", ct.K, q[ct.H])


def bending_targets(y, ct: TorchCell):
    """r y/|y| (y itself where |y| = 0)."""
    n = torch.linalg.norm(y, dim=1)
    scale = torch.where(n > 0.0, ct.r / torch.where(n > 0.0, n, torch.ones_like(n)),
                        torch.ones_like(n))
    return scale[:, None] * y


def volume(q, ct: TorchCell):
    a, b, c = q[ct.tris[:, 0]], q[ct.tris[:, 1]], q[ct.tris[:, 2]]
    return (a * torch.linalg.cross(b, c)).sum() / 6.0


def volume_gradient(q, ct: TorchCell):
    a, b, c = q[ct.tris[:, 0]], q[ct.tris[:, 1]], q[ct.tris[:, 2]]
    g = torch.zeros_like(q)
    g = g.index_add(0, ct.tris[:, 0], torch.linalg.cross(b, c))
    g = g.index_add(0, ct.tris[:, 1], torch.linalg.cross(c, a))
    g = g.index_add(0, ct.tris[:, 2], torch.linalg.cross(a, b))
    return g / 6.0


def volume_target(q, ct: TorchCell, max_iter=100, vol_tol=1e-13, step_tol=1e-15):
    """The oracle's closest-point iteration on V(p) = V_rest, same stopping rule."""
    p = q
    for _ in range(max_iter):
        g = volume_gradient(p, ct)
        V = volume(p, ct)
        lam = (ct.vol_rest - V - (g * (q - p)).sum()) / (g * g).sum()
        p_new = q + lam * g
        dp = float((p_new - p).detach().abs().max())
        p = p_new
        if (abs(float(volume(p, ct).detach()) - ct.vol_rest) <= vol_tol * abs(ct.vol_rest)
                and dp <= step_tol * ct.radius):
            break
    return p


def rhs(q, s, ct: TorchCell, w, m, h):
    """(m/h^2) s + sum_t A_t G_t (w_s Ps^T + w_a Pa^T) + sum_e w_b c_e K_e (x) Pb_e + w_v Pv."""
    F = deformation_gradients(q, ct)
    Wt = ct.area[:, None, None] * (w[0] * strain_targets(F) + w[1] * area_targets(F))
    contrib = torch.einsum("frk,fdk->frd", ct.G, Wt)
    b = (m / h ** 2) * s
    for r in range(3):
        b = b.index_add(0, ct.tris[:, r], contrib[:, r, :])
    Pb = bending_targets(bending_vectors(q, ct), ct)
    hb = (w[2] * ct.c)[:, None, None] * ct.K[:, :, None] * Pb[:, None, :]
    for r in range(4):
        b = b.index_add(0, ct.H[:, r], hb[:, r, :])
    return b + w[3] * volume_target(q, ct)


def system_factor(ct: TorchCell, w, m, h):
    n = ct.n
    A = (m / h ** 2 + w[3]) * torch.eye(n, dtype=DT) + (w[0] + w[1]) * ct.Lt + w[2] * ct.Lb
    return torch.linalg.cholesky(A)


def step(ct: TorchCell, x, v, f, w, m, h, n_iter, chol=None):
    """One PD time step, differentiable in (x, v, f, w)."""
    if chol is None:
        chol = system_factor(ct, w, m, h)
    s = x + h * v + (h * h / m) * f
    q = s
    for _ in range(n_iter):
        q = torch.cholesky_solve(rhs(q, s, ct, w, m, h), chol)
    return q, (q - x) / h


def _step_vjp_along_iterates(ct: TorchCell, xn, vn, fn, wn, m, h, q_given, gx, gv):
    """Vector-Jacobian product of one step whose iterates q^1 .. q^K are given
    (q_given, K = n_iter; q^0 = s): every iteration q^{k+1} = A(w)^-1 rhs(q^k)
    is differentiated at the given q^k, and the adjoints are chained by hand
    from the last iterate back to s. Returns (dx, dv, dw, df)."""
    xn = xn.clone().requires_grad_(True)
    vn = vn.clone().requires_grad_(True)
    wn = wn.clone().requires_grad_(True)
    fn = fn.clone().requires_grad_(True)
    chol = system_factor(ct, wn, m, h)
    s = xn + h * vn + (h * h / m) * fn
    K = len(q_given)
    # x' = q^K, v' = (q^K - x)/h
    g = gx + gv / h
    gw = torch.zeros_like(wn)
    gs = torch.zeros_like(s)
    for k in range(K - 1, -1, -1):
        if k == 0:
            phi = torch.cholesky_solve(rhs(s, s, ct, wn, m, h), chol)
            ds, dw = torch.autograd.grad(phi, (s, wn), g, retain_graph=True)
            gs = gs + ds
        else:
            qk = q_given[k - 1].clone().requires_grad_(True)
            phi = torch.cholesky_solve(rhs(qk, s, ct, wn, m, h), chol)
            dq, ds, dw = torch.autograd.grad(phi, (qk, s, wn), g, retain_graph=True)
            g = dq
            gs = gs + ds
        gw = gw + dw
    dx, dv, df = torch.autograd.grad(s, (xn, vn, fn), gs)
    return dx - gv / h, dv, gw, df


def rollout_grad(o: ops_mod.CellOperators, weights, mass, dt, x0, v0, f, target, n_iter,
                 n_steps, round_state=None, states=None, x_final=None, iterates=None):
    """L = sum |x_T - target|^2 and its gradients.

    Returns (L, dL/dw [4], dL/df [N,3], dL/dx0 [N,3], dL/dv0 [N,3]), float64
    numpy, for constant forces f over the n_steps steps.

    round_state (e.g. torch.float32): round positions and velocities to that
    type after every step and differentiate each step at the rounded state,
    i.e. the exact gradient along the trajectory of a solver that stores its
    state in that type (the step itself stays FP64). The difference from the
    unrounded gradient measures how much the storage rounding alone moves the
    gradient.

    states, x_final: differentiate along a given trajectory instead of the
    oracle's own: states[n] = (x_n, v_n) at the start of step n (n_steps of
    them) and x_final the positions after the last step, e.g. the states a
    reduced-precision solver went through. Each step's derivative is taken
    at the given state (FP64), so the result is the exact gradient of the
    composed step maps along that trajectory.

    iterates (with states): iterates[n] = [q^1, ..., q^n_iter] of step n as
    the other solver formed them; every PD iteration is then differentiated at
    the given iterate instead of at the oracle's own (x_final defaults to the
    last step's last iterate). With the oracle's own iterates this is the
    same gradient."""
    ct = TorchCell(o)
    m, h = float(mass), float(dt)
    w_val = _t(np.asarray(weights, dtype=np.float64))
    f_val = _t(f)
    if iterates is not None:
        assert states is not None and len(iterates) == n_steps
        iterates = [[_t(q) for q in its] for its in iterates]
        assert all(len(its) == n_iter for its in iterates)
        if x_final is None:
            x_final = iterates[-1][-1].numpy()
    if states is not None:
        assert len(states) == n_steps and x_final is not None
        states = [(_t(a), _t(b)) for a, b in states]
        x = _t(x_final)
    else:
        states = []
        x, v = _t(x0), _t(v0)
        with torch.no_grad():
            chol = system_factor(ct, w_val, m, h)
            for _ in range(n_steps):
                states.append((x, v))
                x, v = step(ct, x, v, f_val, w_val, m, h, n_iter, chol)
                if round_state is not None:
                    x, v = x.to(round_state).to(DT), v.to(round_state).to(DT)
    loss = float(((x - _t(target)) ** 2).sum())
    gx = 2.0 * (x - _t(target))
    gv = torch.zeros_like(gx)
    gw = torch.zeros(4, dtype=DT)
    gf = torch.zeros_like(f_val)
    for n in range(n_steps - 1, -1, -1):
        if iterates is not None:
            dx, dv, dw, df = _step_vjp_along_iterates(ct, states[n][0], states[n][1], f_val,
                                                      w_val, m, h, iterates[n], gx, gv)
            gx, gv = dx, dv
            gw += dw
            gf += df
            continue
        xn = states[n][0].clone().requires_grad_(True)
        vn = states[n][1].clone().requires_grad_(True)
        wn = w_val.clone().requires_grad_(True)
        fn = f_val.clone().requires_grad_(True)
        x1, v1 = step(ct, xn, vn, fn, wn, m, h, n_iter)
        dx, dv, dw, df = torch.autograd.grad((x1, v1), (xn, vn, wn, fn), (gx, gv))
        gx, gv = dx, dv
        gw += dw
        gf += df
    return loss, gw.numpy(), gf.numpy(), gx.numpy(), gv.numpy()


def cell_rollout_grad(susp, c: int, target, n_steps=None, n_iter=None, dt=None,
                      round_state=None):
    """rollout_grad for cell c of a suspension (its class, weights, state, forces)."""
    from . import solver as S
    mc, x0, v0, f, w = susp.cell_arrays(int(c))
    return rollout_grad(S.operators_for(mc), w, mc.mass, susp.dt if dt is None else dt,
                        x0, v0, f, target, susp.n_iter if n_iter is None else n_iter,
                        susp.n_steps if n_steps is None else n_steps, round_state)
