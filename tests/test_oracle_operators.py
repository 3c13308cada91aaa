"""Oracle operators pinned to closed forms and textbook identities."""
import numpy as np
import pytest

from npfem_workload import meshes, suspensions
from oracle import operators as O


@pytest.fixture(scope="module")
def rbc():
    x, f = meshes.rbc_mesh(2)
    return O.build_operators(x, f)


def test_rest_deformation_gradient_is_orthonormal(rbc):
    F = O.deformation_gradients(rbc.X, rbc.tris, rbc.G)
    FtF = np.einsum("fdk,fdl->fkl", F, F)
    assert np.allclose(FtF, np.eye(2)[None], atol=1e-13)
    # rows of G sum to zero: F is blind to translations
    assert np.allclose(rbc.G.sum(axis=1), 0.0, atol=1e-13)


def test_deformation_gradient_rotates_with_the_body(rbc):
    R = suspensions.random_rotations(np.random.default_rng(1), 1)[0]
    F0 = O.deformation_gradients(rbc.X, rbc.tris, rbc.G)
    F1 = O.deformation_gradients(rbc.X @ R.T + np.array([3.0, -2.0, 7.0]), rbc.tris, rbc.G)
    assert np.allclose(F1, np.einsum("de,fek->fdk", R, F0), atol=1e-12)


def _cot(p, a, b):
    u, v = a - p, b - p
    return np.dot(u, v) / np.linalg.norm(np.cross(u, v))


def test_triangle_laplacian_is_cotangent_laplacian(rbc):
    """sum_t A_t G_t G_t^T is the P1 finite-element stiffness matrix:
    off-diagonal (i, j) = -(cot alpha + cot beta) / 2 over the two angles
    opposite the edge, rows summing to zero."""
    Lt, _ = O.laplacians(rbc)
    X = rbc.X
    for i, j, k, l in rbc.H[:40]:
        expect = -0.5 * (_cot(X[k], X[i], X[j]) + _cot(X[l], X[i], X[j]))
        assert abs(Lt[i, j] - expect) < 1e-12 and abs(Lt[j, i] - expect) < 1e-12
    assert np.allclose(Lt.sum(axis=1), 0.0, atol=1e-12)
    nonedge = np.ones_like(Lt, dtype=bool)
    nonedge[rbc.H[:, 0], rbc.H[:, 1]] = nonedge[rbc.H[:, 1], rbc.H[:, 0]] = False
    np.fill_diagonal(nonedge, False)
    assert np.all(Lt[nonedge] == 0.0)


def test_hinge_topology(rbc):
    H = rbc.H
    tri_set = {tuple(sorted(t)) for t in rbc.tris.tolist()}
    for i, j, k, l in H:
        assert i < j and k != l
        assert tuple(sorted((i, j, k))) in tri_set and tuple(sorted((i, j, l))) in tri_set
    # k sits in the triangle where the edge runs i -> j
    directed = {}
    for a, b, c in rbc.tris.tolist():
        directed[(a, b)] = c
        directed[(b, c)] = a
        directed[(c, a)] = b
    assert all(directed[(i, j)] == k and directed[(j, i)] == l for i, j, k, l in H.tolist())


def test_bending_stencil_flat_hinge_and_invariance():
    rng = np.random.default_rng(3)
    for _ in range(20):
        # a random planar hinge: i, j on the x axis, k above, l below
        X = np.array([[0.0, 0, 0], [1.0 + rng.random(), 0, 0],
                      [rng.random(), 0.3 + rng.random(), 0], [rng.random(), -0.3 - rng.random(), 0]])
        H = np.array([[0, 1, 2, 3]])
        K, c, r = O.hinge_operators(X, H)
        assert abs(K.sum()) < 1e-13
        assert r[0] < 1e-13  # flat hinge: zero stencil vector
        Y = X.copy()
        Y[3, 2] = 0.4  # fold it
        K2, _, r2 = O.hinge_operators(Y, H)
        R = suspensions.random_rotations(rng, 1)[0]
        Z = Y @ R.T + rng.standard_normal(3)
        y2 = K2[0] @ Y
        y3 = K2[0] @ Z
        assert r2[0] > 1e-3 and abs(np.linalg.norm(y3) - np.linalg.norm(y2)) < 1e-12


def test_system_matrix_spd_and_translation_nullspace(rbc):
    w = (1.0, 1.0, 0.01, 10.0)
    A = O.system_matrix(rbc, w, 1e-3, 1e-2)
    assert np.allclose(A, A.T, atol=0)
    assert np.linalg.eigvalsh(A).min() > 0
    # elastic part annihilates constants; only inertia and volume act on a translation
    ones = np.ones(rbc.n_verts)
    assert np.allclose(A @ ones, (1e-3 / 1e-4 + 10.0) * ones, atol=1e-10)
    # the two factorisations agree
    b = np.random.default_rng(0).standard_normal((rbc.n_verts, 3))
    import scipy.linalg
    assert np.allclose(scipy.linalg.cho_solve(O.factor(A), b), np.linalg.solve(A, b), atol=1e-12)


def test_mesh_errors():
    v, f = meshes.icosahedron()
    with pytest.raises(O.MeshError):
        O.check_closed_manifold(f[:-1], 12)  # open
    g = f.copy()
    g[0] = g[0][::-1]
    with pytest.raises(O.MeshError):
        O.check_closed_manifold(g, 12)  # one flipped triangle
    with pytest.raises(O.MeshError):
        O.triangle_operators(np.zeros((3, 3)), np.array([[0, 1, 2]]))
