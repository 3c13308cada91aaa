"""Pins of the oracle's quasi-Newton step (L-BFGS with the PD matrix as the
initial Hessian and Armijo backtracking).

* Without history and with full steps it is the PD iteration itself.
* The objective never increases (Armijo), and the gradient it uses is the
  gradient of the objective (central differences).
* It converges to the minimiser that PD converges to and that Newton's method
  finds on the 12-vertex icosahedron (stiff twin), and it gets there in far
  fewer iterations than PD on a stiff RBC.
"""
import numpy as np

from npfem_workload import meshes, suspensions as W
from oracle import newton
from oracle import operators as ops_mod
from oracle import quasi_newton as Q
from oracle import solver as S


def _rbc(dt=1e-2, level=2, seed=0, amp=0.05):
    x, t = meshes.rbc_mesh(level)
    o = ops_mod.build_operators(x, t)
    cs = S.CellSolver(o, S.Params((1.0, 1.0, 0.01, 10.0), 1e-3, dt))
    rng = np.random.default_rng(seed)
    x0 = o.X + amp * rng.standard_normal(o.X.shape)
    f = 0.05 * rng.standard_normal(o.X.shape)
    return o, cs, x0, np.zeros_like(x0), f


def test_no_history_full_step_is_pd():
    o, cs, x0, v0, f = _rbc()
    xq, _, _ = Q.step(cs, x0, v0, f, 6, history=0, max_ls=1)
    xp, _, _ = cs.step(x0, v0, f, 6)
    assert np.abs(xq - xp).max() <= 1e-12 * o.radius


def test_gradient_is_the_objective_gradient():
    o, cs, x0, v0, f = _rbc()
    h, m = cs.prm.dt, cs.prm.mass
    s = x0 + h * v0 + (h * h / m) * f
    q = s + 0.01 * np.random.default_rng(9).standard_normal(s.shape)
    E, g = Q.objective_and_gradient(cs, q, s)
    rng = np.random.default_rng(10)
    for _ in range(3):
        dq = rng.standard_normal(q.shape)
        eps = 1e-6
        Ep, _ = Q.objective_and_gradient(cs, q + eps * dq, s)
        Em, _ = Q.objective_and_gradient(cs, q - eps * dq, s)
        assert abs((Ep - Em) / (2 * eps) - np.sum(g * dq)) <= 1e-6 * np.abs(g).sum()


def test_objective_monotone_and_same_minimiser_as_pd():
    o, cs, x0, v0, f = _rbc()
    xq, _, Eq = Q.step(cs, x0, v0, f, 60, record=True)
    Eq = np.asarray(Eq)
    assert np.all(np.diff(Eq) <= 1e-13 * abs(Eq[0]))
    xp, _, _ = cs.step(x0, v0, f, 3000)
    assert np.abs(xq - xp).max() <= 1e-10 * o.radius


def test_matches_newton_on_icosahedron():
    x, t = meshes.icosahedron()
    o = ops_mod.build_operators(x, t)
    prm = S.Params((1.0, 1.0, 0.01, 10.0), 1e-3, 1e-2)
    cs = S.CellSolver(o, prm)
    rng = np.random.default_rng(2)
    x0 = o.X + 1e-2 * rng.standard_normal(o.X.shape)
    v0 = np.zeros_like(x0)
    f = 0.05 * rng.standard_normal(o.X.shape)
    xq, _, _ = Q.step(cs, x0, v0, f, 80)
    s = x0 + prm.dt * v0 + prm.dt ** 2 / prm.mass * f
    qn, gn = newton.minimise(o, s, prm)
    assert gn <= 1e-10
    assert np.abs(xq - qn).max() <= 1e-10


def test_fewer_iterations_than_pd():
    """Stiff RBC (m/h^2 ~ 1.1, weights 1/1/0.01/10): L-BFGS reaches 1e-9 of
    the radius from the converged step in k iterations; PD has not after 3k."""
    o, cs, x0, v0, f = _rbc(dt=3e-2, amp=0.1)
    x_ref, _, _ = Q.step(cs, x0, v0, f, 300)
    tol = 1e-9 * o.radius
    k_qn = next(k for k in range(1, 300)
                if np.abs(Q.step(cs, x0, v0, f, k)[0] - x_ref).max() <= tol)
    err_pd = np.abs(cs.step(x0, v0, f, 3 * k_qn)[0] - x_ref).max()
    assert err_pd > tol, (k_qn, err_pd)
