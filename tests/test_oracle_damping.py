"""Pins of the oracle's viscous (Rayleigh-type) damping, C = alpha m I +
beta K_d taken implicitly at the end-of-step velocity.

* Free flight (all weights zero, so K_d = 0) with mass damping: the velocity
  obeys v_{n+1} (1 + alpha h) = v_n + (h/m) f, a linear recursion with the
  closed form v_n = v_inf + (v_0 - v_inf) r^n, r = 1/(1 + alpha h),
  v_inf = f/(alpha m).
* Momentum: the elastic forces and K_d have no net force on a closed cell,
  so (1 + alpha h) sum m v_{n+1} = sum m v_n + h sum f for any weights.
* Stiffness damping does not act on a rigid translation (K_d 1 = 0): a
  cell at its rest shape moving uniformly keeps moving uniformly.
* The PD iteration still never increases the step's objective (the damping
  term is quadratic and enters the exact global minimisation).
* A damped free vibration ends with less mechanical energy than the undamped
  one, and alpha = beta = 0 is the undamped step exactly.
"""
import numpy as np
import pytest

from npfem_workload import meshes, suspensions as W
from oracle import operators as ops_mod
from oracle import projections as proj
from oracle import solver as S


def _solver(weights, damping, dt=1e-2, mass=1e-3, level=2):
    x, t = meshes.rbc_mesh(level)
    o = ops_mod.build_operators(x, t)
    return o, S.CellSolver(o, S.Params(tuple(weights), mass, dt, tuple(damping)))


def test_free_flight_mass_damping_closed_form():
    alpha, h, m = 30.0, 1e-2, 1e-3
    o, cs = _solver((0, 0, 0, 0), (alpha, 0.7))
    rng = np.random.default_rng(0)
    x0 = o.X.copy()
    v0 = 0.1 * rng.standard_normal(x0.shape)
    f = 0.05 * rng.standard_normal(x0.shape)
    n = 6
    x, v = cs.rollout(x0, v0, f, 3, n)
    r = 1.0 / (1.0 + alpha * h)
    vinf = f / (alpha * m)
    vn = vinf + (v0 - vinf) * r ** n
    xn = x0 + h * (n * vinf + (v0 - vinf) * r * (1.0 - r ** n) / (1.0 - r))
    assert np.allclose(v, vn, rtol=1e-11, atol=1e-13)
    assert np.allclose(x, xn, rtol=1e-12, atol=1e-13)


def test_momentum_balance_with_damping():
    alpha, h, m = 20.0, 1e-2, 1e-3
    o, cs = _solver((1.0, 1.0, 0.01, 10.0), (alpha, 0.05))
    rng = np.random.default_rng(1)
    x = o.X + 0.02 * rng.standard_normal(o.X.shape)
    v = 0.05 * rng.standard_normal(o.X.shape)
    f = 0.05 * rng.standard_normal(o.X.shape)
    for _ in range(3):
        x1, v1, _ = cs.step(x, v, f, 5)
        lhs = (1.0 + alpha * h) * m * v1.sum(axis=0)
        rhs = m * v.sum(axis=0) + h * f.sum(axis=0)
        assert np.allclose(lhs, rhs, rtol=0, atol=1e-12 * max(1.0, np.abs(rhs).max()))
        x, v = x1, v1


def test_stiffness_damping_spares_rigid_translation():
    o, cs = _solver((1.0, 1.0, 0.01, 10.0), (0.0, 0.5))
    u = np.array([0.3, -0.2, 0.1])
    x, v = o.X.copy(), np.tile(u, (o.n_verts, 1))
    f = np.zeros_like(x)
    for k in range(1, 5):
        x, v, _ = cs.step(x, v, f, 5)
        assert np.abs(x - (o.X + k * 1e-2 * u)).max() <= 1e-12 * o.radius
        assert np.abs(v - u).max() <= 1e-10


@pytest.mark.parametrize("damping", [(10.0, 0.0), (0.0, 0.02), (10.0, 0.02)])
def test_objective_monotone_with_damping(damping):
    o, cs = _solver((1.0, 1.0, 0.01, 10.0), damping)
    rng = np.random.default_rng(2)
    x = o.X + 0.05 * rng.standard_normal(o.X.shape)
    v = 0.1 * rng.standard_normal(o.X.shape)
    f = 0.05 * rng.standard_normal(o.X.shape)
    _, _, E = cs.step(x, v, f, 20, record_energy=True)
    E = np.asarray(E)
    assert np.all(np.diff(E) <= 1e-12 * abs(E[0])) and E[-1] < E[0]


def _mechanical_energy(o, prm, x, v):
    """Kinetic energy plus the elastic potential sum_i (w_i/2) dist^2(S_i x, C_i)."""
    ws, wa, wb, wv = prm.weights
    P = proj.local_step(x, o)
    e = 0.5 * prm.mass * np.sum(v * v)
    e += np.sum(0.5 * o.area * (ws * np.sum((P["F"] - P["Ps"]) ** 2, axis=(1, 2))
                                + wa * np.sum((P["F"] - P["Pa"]) ** 2, axis=(1, 2))))
    e += np.sum(0.5 * wb * o.c * np.sum((P["y"] - P["Pb"]) ** 2, axis=1))
    e += 0.5 * wv * np.sum((x - P["Pv"]) ** 2)
    return float(e)


def test_damping_dissipates_and_reduces_to_undamped():
    w = (1.0, 1.0, 0.01, 10.0)
    rng = np.random.default_rng(3)
    x, t = meshes.rbc_mesh(2)
    o = ops_mod.build_operators(x, t)
    x0 = o.X + 0.05 * rng.standard_normal(o.X.shape)
    v0 = np.zeros_like(x0)
    f = np.zeros_like(x0)
    out = {}
    for damping in ((0.0, 0.0), (20.0, 0.0), (0.0, 0.02)):
        prm = S.Params(w, 1e-3, 1e-2, damping)
        xs, vs = S.CellSolver(o, prm).rollout(x0, v0, f, 10, 20)
        out[damping] = (_mechanical_energy(o, prm, xs, vs), xs)
    e0 = out[(0.0, 0.0)][0]
    assert out[(20.0, 0.0)][0] < e0 and out[(0.0, 0.02)][0] < e0
    # zero damping is the undamped solver itself
    xs, _ = S.CellSolver(o, S.Params(w, 1e-3, 1e-2)).rollout(x0, v0, f, 10, 20)
    assert np.array_equal(xs, out[(0.0, 0.0)][1])


def test_damped_matrix_is_scaled_system_matrix():
    """A + C/h equals the system matrix with mass m (1 + alpha h) and
    stretch/area/bend weights (1 + beta/h) w (volume weight unchanged)."""
    alpha, beta, h, m = 7.0, 0.03, 1e-2, 1e-3
    w = (1.0, 0.8, 0.01, 10.0)
    o, cs = _solver(w, (alpha, beta), dt=h, mass=m)
    k = 1.0 + beta / h
    A2 = ops_mod.system_matrix(o, (k * w[0], k * w[1], k * w[2], w[3]), m * (1.0 + alpha * h), h)
    assert np.allclose(cs.A, A2, rtol=1e-14, atol=1e-12)
