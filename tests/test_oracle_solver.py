"""Full oracle step pinned to closed forms, invariants and a Newton minimiser."""
import numpy as np
import pytest

from npfem_workload import meshes, suspensions
from oracle import newton
from oracle import operators as O
from oracle import solver as S

NOMINAL = (1.0, 1.0, 0.01, 10.0)


@pytest.fixture(scope="module")
def rbc2():
    x, f = meshes.rbc_mesh(2)
    return O.build_operators(x, f)


@pytest.fixture(scope="module")
def ico():
    v, f = meshes.icosahedron()
    return O.build_operators(v, f)


def test_free_flight_closed_form(rbc2):
    """All weights zero: x_n = x0 + n h v0 + h^2 n(n+1)/2 f/m."""
    rng = np.random.default_rng(0)
    prm = S.Params((0.0, 0.0, 0.0, 0.0), 2e-3, 1e-3)
    cs = S.CellSolver(rbc2, prm)
    x0 = rbc2.X.copy()
    v0 = rng.standard_normal(x0.shape)
    f = rng.standard_normal(x0.shape)
    n = 7
    x, v = cs.rollout(x0, v0, f, n_iter=3, n_steps=n)
    h, m = prm.dt, prm.mass
    assert np.allclose(x, x0 + n * h * v0 + h * h * n * (n + 1) / 2 * f / m, atol=1e-13)
    assert np.allclose(v, v0 + n * h * f / m, atol=1e-10)


def test_rest_state_stays_or_translates(rbc2):
    cs = S.CellSolver(rbc2, S.Params(NOMINAL, 1e-3, 1e-4))
    z = np.zeros_like(rbc2.X)
    x, v = cs.rollout(rbc2.X, z, z, n_iter=5, n_steps=5)
    assert np.abs(x - rbc2.X).max() < 1e-12 and np.abs(v).max() < 1e-8
    u = np.array([0.3, -0.2, 0.1])
    x, v = cs.rollout(rbc2.X, z + u, z, n_iter=5, n_steps=5)
    assert np.abs(x - (rbc2.X + 5 * 1e-4 * u)).max() < 1e-12


def test_rigid_motion_equivariance(rbc2):
    rng = np.random.default_rng(1)
    cs = S.CellSolver(rbc2, S.Params(NOMINAL, 1e-3, 1e-2))
    x0 = rbc2.X + 0.02 * rng.standard_normal(rbc2.X.shape)
    v0 = 0.1 * rng.standard_normal(x0.shape)
    f = 0.05 * rng.standard_normal(x0.shape)
    R = suspensions.random_rotations(rng, 1)[0]
    t = np.array([100.0, -40.0, 7.0])
    xa, va = cs.rollout(x0, v0, f, 5, 3)
    xb, vb = cs.rollout(x0 @ R.T + t, v0 @ R.T, f @ R.T, 5, 3)
    assert np.abs(xb - (xa @ R.T + t)).max() < 1e-11
    assert np.abs(vb - va @ R.T).max() < 1e-8


def test_momentum_balance(rbc2):
    """Sum m v_{n+1} = sum m v_n + h sum f, for any number of PD iterations."""
    rng = np.random.default_rng(2)
    for dt in (1e-4, 1e-2):
        cs = S.CellSolver(rbc2, S.Params(NOMINAL, 1e-3, dt))
        x0 = rbc2.X + 0.05 * rng.standard_normal(rbc2.X.shape)
        v0 = rng.standard_normal(x0.shape)
        f = rng.standard_normal(x0.shape)
        for n_iter in (1, 3):
            _, v1, _ = cs.step(x0, v0, f, n_iter)
            lhs = 1e-3 * v1.sum(axis=0)
            rhs = 1e-3 * v0.sum(axis=0) + dt * f.sum(axis=0)
            assert np.allclose(lhs, rhs, rtol=0, atol=1e-11 * max(1.0, np.abs(rhs).max()))


def test_energy_monotone_stiff(rbc2):
    rng = np.random.default_rng(3)
    cs = S.CellSolver(rbc2, S.Params(NOMINAL, 1e-3, 1e-2))
    x0 = rbc2.X + 0.05 * rng.standard_normal(rbc2.X.shape)
    f = 0.05 * rng.standard_normal(x0.shape)
    _, _, E = cs.step(x0, np.zeros_like(x0), f, 25, record_energy=True)
    E = np.asarray(E)
    assert E[0] > E[-1] > 0
    assert np.all(np.diff(E) <= 1e-12 * abs(E[0]))


def test_energy_zero_at_rest(rbc2):
    from oracle import projections as P
    prm = S.Params(NOMINAL, 1e-3, 1e-4)
    proj = P.local_step(rbc2.X, rbc2)
    assert S.energy(rbc2, rbc2.X, rbc2.X, proj, prm) < 1e-20


def test_pd_converges_to_newton_minimiser(ico):
    """2000 PD iterations on the 12-vertex icosahedron equal the Newton minimiser."""
    rng = np.random.default_rng(0)
    prm = S.Params(NOMINAL, 1e-3, 1e-2)
    cs = S.CellSolver(ico, prm)
    x0 = ico.X + 1e-2 * rng.standard_normal(ico.X.shape)
    v0 = np.zeros_like(x0)
    f = 0.05 * rng.standard_normal(x0.shape)
    q_pd, _, _ = cs.step(x0, v0, f, 2000)
    s = x0 + prm.dt * v0 + prm.dt ** 2 / prm.mass * f
    q_nt, gnorm = newton.minimise(ico, s, prm)
    assert gnorm <= 1e-12
    assert np.abs(q_pd - q_nt).max() <= 1e-10


def test_newton_gradient_matches_objective(ico):
    rng = np.random.default_rng(5)
    prm = S.Params(NOMINAL, 1e-3, 1e-2)
    s = ico.X + 0.02 * rng.standard_normal(ico.X.shape)
    q = s + 0.01 * rng.standard_normal(s.shape)
    g = newton.gradient(ico, q, s, prm)
    d = rng.standard_normal(q.shape)
    eps = 1e-6
    fd = (newton.objective(ico, q + eps * d, s, prm) - newton.objective(ico, q - eps * d, s, prm)) / (2 * eps)
    assert abs(fd - np.sum(g * d)) < 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("dt", [1e-2, 1e-1])
def test_large_time_steps_stay_bounded(rbc2, dt):
    rng = np.random.default_rng(6)
    cs = S.CellSolver(rbc2, S.Params(NOMINAL, 1e-3, dt))
    x0 = rbc2.X + 0.3 * rng.standard_normal(rbc2.X.shape)  # badly distorted start
    x, v = cs.rollout(x0, np.zeros_like(x0), np.zeros_like(x0), 10, 10)
    assert np.all(np.isfinite(x)) and np.all(np.isfinite(v))
    Vr = O.volume(rbc2.X, rbc2.tris)
    assert abs(O.volume(x, rbc2.tris) - Vr) < 0.2 * Vr
