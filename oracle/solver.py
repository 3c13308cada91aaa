"""Projective-dynamics time stepping for one cell and for a suspension (FP64).

Test infrastructure only (see the package docstring).

One implicit step from (x_n, v_n) under external nodal forces f_n (the
elastodynamics equation, eq. 2, with lumped vertex mass m and body force
standing in for the fluid coupling, Introduction; forces in, positions and
velocities out as in the fluid-solid exchange, Implementation and
architecture):

    s = x_n + h v_n + (h^2/m) f_n,   q = s
    repeat n_iter times:
        local step:  projections P(q) (``projections.local_step``)
        global step: A q = (m/h^2) s + sum_t A_t G_t (w_s Ps_t^T + w_a Pa_t^T)
                           + sum_e w_b c_e K_e (x) Pb_e + w_v Pv
    x_{n+1} = q,   v_{n+1} = (q - x_n) / h

The diagnostic energy at iterate q (with P = P(q)) is
    E(q) = (m/2h^2)|q - s|^2 + sum_t (A_t/2)[w_s |F - Ps|^2 + w_a |F - Pa|^2]
           + sum_e (w_b c_e/2)|y - Pb|^2 + (w_v/2)|q - Pv|^2,
which the alternation never increases.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg

from . import contacts as contacts_mod
from . import operators as ops_mod
from . import projections as proj


@dataclass
class Params:
    weights: tuple  # (w_stretch, w_area, w_bend, w_volume)
    mass: float
    dt: float
    damping: tuple = (0.0, 0.0)  # (alpha, beta): Rayleigh-type viscous damping


def damping_stiffness(o: ops_mod.CellOperators, weights) -> np.ndarray:
    """K_d = (w_s + w_a) L_tri + w_b L_bend: the constraint stiffness without
    the volume term's identity (it vanishes on rigid translations, which the
    stiffness-proportional damping must not resist)."""
    ws, wa, wb, _ = (float(w) for w in weights)
    Lt, Lb = ops_mod.laplacians(o)
    return (ws + wa) * Lt + wb * Lb


def rhs(o: ops_mod.CellOperators, P: dict, s: np.ndarray, prm: Params) -> np.ndarray:
    """Right-hand side (m/h^2) s + sum of the constraints' weighted targets.
    Reading of the weights: strain and area scaled by the rest triangle area,
    bending by c_e = 3 / (A1 + A2), volume per vertex unscaled."""
    ws, wa, wb, wv = prm.weights
    b = (prm.mass / prm.dt ** 2) * s
    # triangles: rows of A_t G_t (w_s Ps^T + w_a Pa^T) go to the triangle's vertices
    Wt = o.area[:, None, None] * (ws * P["Ps"] + wa * P["Pa"])  # [F, 3xyz, 2]
    contrib = np.einsum("frk,fdk->frd", o.G, Wt)  # [F, 3 vertices, 3 xyz]
    for r in range(3):
        np.add.at(b, o.tris[:, r], contrib[:, r, :])
    # hinges: w_b c_e K_e[r] Pb_e to vertex H_e[r]
    hb = (wb * o.c)[:, None, None] * o.K[:, :, None] * P["Pb"][:, None, :]  # [E, 4, 3]
    for r in range(4):
        np.add.at(b, o.H[:, r], hb[:, r, :])
    b += wv * P["Pv"]
    return b


def energy(o: ops_mod.CellOperators, q: np.ndarray, s: np.ndarray, P: dict, prm: Params,
           x=None, C=None) -> float:
    """The step's objective at q (with the projections P = P(q)); with a
    damping matrix C and the step's start x, plus (1/2h)(q - x)^T C (q - x)."""
    ws, wa, wb, wv = prm.weights
    e = 0.5 * prm.mass / prm.dt ** 2 * np.sum((q - s) ** 2)
    if C is not None:
        e += 0.5 / prm.dt * float(np.sum((q - x) * (C @ (q - x))))
    dF_s = np.sum((P["F"] - P["Ps"]) ** 2, axis=(1, 2))
    dF_a = np.sum((P["F"] - P["Pa"]) ** 2, axis=(1, 2))
    e += np.sum(0.5 * o.area * (ws * dF_s + wa * dF_a))
    e += np.sum(0.5 * wb * o.c * np.sum((P["y"] - P["Pb"]) ** 2, axis=1))
    e += 0.5 * wv * np.sum((q - P["Pv"]) ** 2)
    return float(e)


class CellSolver:
    """Factorised system for one (mesh class, weights, mass, dt, damping).

    Viscoelastic reading (the elastodynamics equation with a viscous term,
    Introduction; the viscosity parameters Calpha and Cbeta of the material,
    sections "RBC collision at an obstacle" and "Setting up new materials"):
    a damping force -C v with C = alpha m I + beta K_d (mass- and
    stiffness-proportional, K_d = damping_stiffness), taken implicitly at
    v_{n+1} = (q - x_n)/h. It adds (1/2h)(q - x_n)^T C (q - x_n) to the
    step's objective, so the system matrix becomes A + C/h and the
    right-hand side gains C x_n / h; the local step is unchanged. The first
    iterate minimises the inertia and mass-damping terms alone,
    q^0 = (s + alpha h x_n)/(1 + alpha h) (s itself without damping), which
    keeps the momentum balance exact at every iteration count."""

    def __init__(self, o: ops_mod.CellOperators, prm: Params, contact_weight: float = 0.0):
        self.o = o
        self.prm = prm
        self.wc = float(contact_weight)
        self.A = ops_mod.system_matrix(o, prm.weights, prm.mass, prm.dt)
        if self.wc != 0.0:
            # every vertex carries the contact potential (oracle.contacts)
            self.A = self.A + self.wc * np.eye(o.n_verts)
        alpha, beta = prm.damping
        self.C = None
        if alpha != 0.0 or beta != 0.0:
            self.C = alpha * prm.mass * np.eye(o.n_verts) + beta * damping_stiffness(o, prm.weights)
            self.A = self.A + self.C / prm.dt
        self.chol = ops_mod.factor(self.A)

    def step(self, x, v, f, n_iter, record_energy=False, contacts=None):
        """One time step; returns (x_new, v_new, energies) with energies
        E(q^0..q^n_iter) when requested. Readings: a fixed count of n_iter
        local/global iterations from q^0 = s (the inertial prediction),
        v = (q - x) / h, no damping. contacts = (points [K,3], normals [K,3])
        of the cell's neighbourhood (oracle.contacts), with the weight given
        at construction."""
        h, m = self.prm.dt, self.prm.mass
        s = x + h * v + (h * h / m) * f
        alpha = self.prm.damping[0]
        q = s.copy() if alpha == 0.0 else (s + alpha * h * x) / (1.0 + alpha * h)
        energies = []
        cx = None if self.C is None else (self.C @ x) / h
        use_c = contacts is not None and self.wc != 0.0
        for _ in range(n_iter):
            P = proj.local_step(q, self.o)
            if use_c:
                Pc = contacts_mod.project_contacts(q, contacts[0], contacts[1])
            if record_energy:
                e = energy(self.o, q, s, P, self.prm, x, self.C)
                if use_c:
                    e += 0.5 * self.wc * float(np.sum((q - Pc) ** 2))
                energies.append(e)
            b = rhs(self.o, P, s, self.prm)
            if cx is not None:
                b = b + cx
            if use_c:
                b = b + self.wc * Pc
            q = scipy.linalg.cho_solve(self.chol, b)
        if record_energy:
            P = proj.local_step(q, self.o)
            e = energy(self.o, q, s, P, self.prm, x, self.C)
            if use_c:
                Pc = contacts_mod.project_contacts(q, contacts[0], contacts[1])
                e += 0.5 * self.wc * float(np.sum((q - Pc) ** 2))
            energies.append(e)
        return q, (q - x) / h, energies

    def rollout(self, x0, v0, f, n_iter, n_steps, forces_per_step=None, contacts=None):
        x, v = x0.copy(), v0.copy()
        for n in range(n_steps):
            fn = f if forces_per_step is None else forces_per_step[n]
            x, v, _ = self.step(x, v, fn, n_iter, contacts=contacts)
        return x, v


_OPS_CACHE: dict = {}


def operators_for(mesh_class) -> ops_mod.CellOperators:
    key = id(mesh_class)
    o = _OPS_CACHE.get(key)
    if o is None or o.X is not mesh_class.rest:
        o = ops_mod.build_operators(mesh_class.rest, mesh_class.tris)
        _OPS_CACHE[key] = o
    return o


def cell_contacts(susp, c: int):
    """(contact weight, (points, normals) or None) of cell c of a suspension."""
    wc = float(susp.extra.get("contact_weight", 0.0))
    ct = susp.extra.get("contacts")
    if ct is None or wc == 0.0:
        return wc, None
    pts, nrm, off = ct
    return wc, (pts[off[c]:off[c + 1]], nrm[off[c]:off[c + 1]])


def run_cell(susp, c: int, n_steps=None, n_iter=None, dt=None):
    """Roll out one cell of a suspension; returns (x [N,3], v [N,3]) local coords."""
    mc, x0, v0, f, w = susp.cell_arrays(c)
    o = operators_for(mc)
    prm = Params(tuple(w), mc.mass, susp.dt if dt is None else dt,
                 tuple(getattr(mc, "damping", (0.0, 0.0))))
    wc, ct = cell_contacts(susp, c)
    solver = CellSolver(o, prm, wc)
    return solver.rollout(x0, v0, f, susp.n_iter if n_iter is None else n_iter,
                          susp.n_steps if n_steps is None else n_steps, contacts=ct)


def run_cells(susp, cells, n_steps=None, n_iter=None):
    """Roll out the listed cells; returns {cell: (x, v)}."""
    return {int(c): run_cell(susp, int(c), n_steps, n_iter) for c in cells}


def rel_position_error(x: np.ndarray, x_ref: np.ndarray) -> float:
    """max_v |x - x_ref| / R with R = max_v |x_ref_v - centroid(x_ref)|."""
    R = np.linalg.norm(x_ref - x_ref.mean(axis=0), axis=1).max()
    return float(np.linalg.norm(x - x_ref, axis=1).max() / R)
