"""Local-step projections pinned to library routines, brute force and symmetry."""
import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

from npfem_workload import meshes, suspensions
from oracle import operators as O
from oracle import projections as P


def random_F(rng, n, spread=0.3):
    R = suspensions.random_rotations(rng, n)[:, :, :2]
    S = np.eye(2)[None] + spread * rng.standard_normal((n, 2, 2))
    return R @ S


def test_strain_projection_is_polar_factor():
    rng = np.random.default_rng(0)
    F = random_F(rng, 50)
    Ps = P.project_strain(*P.thin_svd(F))
    for i in range(50):
        u, _ = scipy.linalg.polar(F[i], side="right")
        assert np.allclose(Ps[i], u, atol=1e-12)
    # F = R diag(s) has polar factor R
    R = suspensions.random_rotations(rng, 5)[:, :, :2]
    F2 = R * np.array([1.7, 0.6])[None, None, :]
    assert np.allclose(P.project_strain(*P.thin_svd(F2)), R, atol=1e-13)


def brute_area(s1, s2):
    f = lambda t: (t - s1) ** 2 + (1.0 / t - s2) ** 2
    grid = np.exp(np.linspace(np.log(1e-3), np.log(1e3), 200001))
    t0 = grid[np.argmin(f(grid))]
    res = scipy.optimize.minimize_scalar(f, bracket=(t0 * 0.999, t0, t0 * 1.001), tol=1e-14)
    return res.x


def test_area_root_matches_brute_force():
    rng = np.random.default_rng(1)
    s1 = 0.3 + 2.0 * rng.random(40)
    s2 = s1 * rng.random(40)
    t = P.area_root(s1, s2)
    for i in range(40):
        assert abs(t[i] - brute_area(s1[i], s2[i])) < 1e-6 * t[i]
        # stationarity: the quartic vanishes at the root
        assert abs(t[i] ** 4 - s1[i] * t[i] ** 3 + s2[i] * t[i] - 1.0) < 1e-12


def test_area_special_cases():
    # already on the constraint set: identity
    s1 = np.array([2.0, 1.25, 1.0])
    assert np.allclose(P.area_root(s1, 1.0 / s1), s1, atol=1e-13)
    # equal singular values below 2 project to (1, 1)
    assert np.allclose(P.area_root(np.array([0.5, 1.3, 1.9]), np.array([0.5, 1.3, 1.9])), 1.0, atol=1e-13)


def test_area_projection_is_closest_point_on_set():
    rng = np.random.default_rng(2)
    F = random_F(rng, 10)
    Pa = P.project_area(*P.thin_svd(F))
    for i in range(10):
        s = np.linalg.svd(Pa[i], compute_uv=False)
        assert abs(s[0] * s[1] - 1.0) < 1e-12
        d0 = np.linalg.norm(F[i] - Pa[i])
        for _ in range(200):
            X = Pa[i] + 0.05 * rng.standard_normal((3, 2))
            u, sx, vt = np.linalg.svd(X, full_matrices=False)
            sx = sx / np.sqrt(sx[0] * sx[1])
            X = u @ np.diag(sx) @ vt
            assert np.linalg.norm(F[i] - X) >= d0 - 1e-12


def test_bending_projection_at_rest_and_zero():
    x, f = meshes.rbc_mesh(2)
    o = O.build_operators(x, f)
    y = P.bending_vectors(o.X, o.H, o.K)
    assert np.allclose(P.project_bending(y, o.r), y, atol=1e-13)
    z = np.zeros((2, 3))
    assert np.all(P.project_bending(z, np.array([1.0, 2.0])) == 0.0)
    yy = np.array([[3.0, 4.0, 0.0]])
    assert np.allclose(P.project_bending(yy, np.array([10.0])), [[6.0, 8.0, 0.0]])


def test_volume_projection_of_scaled_icosahedron_is_exact():
    v, f = meshes.icosahedron()
    Vr = O.volume(v, f)
    for alpha in (0.9, 1.05, 1.3):
        p, it = P.project_volume(alpha * v, f, Vr, 1.0)
        assert np.allclose(p, v, atol=1e-14), (alpha, it)


def test_volume_projection_fixed_point_and_closest_point():
    v, f = meshes.icosahedron()
    Vr = O.volume(v, f)
    p, _ = P.project_volume(v, f, Vr, 1.0)
    assert np.array_equal(p, v)
    rng = np.random.default_rng(4)
    q = v + 0.05 * rng.standard_normal(v.shape)
    p, it = P.project_volume(q, f, Vr, 1.0)
    assert abs(O.volume(p, f) - Vr) < 1e-13 * Vr and it < 100
    assert np.allclose((p - q).sum(axis=0), 0.0, atol=1e-14)
    cons = {"type": "eq", "fun": lambda z: O.volume(z.reshape(-1, 3), f) - Vr}
    res = scipy.optimize.minimize(lambda z: np.sum((z - q.ravel()) ** 2), q.ravel(),
                                  constraints=[cons], method="SLSQP",
                                  options={"ftol": 1e-16, "maxiter": 500})
    assert np.allclose(res.x.reshape(-1, 3), p, atol=1e-7)


def test_degenerate_triangle_raises():
    F = np.zeros((1, 3, 2))
    F[0, 0, 0] = 1.0
    with pytest.raises(P.DegenerateElement):
        P.thin_svd(F)
