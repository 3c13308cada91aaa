"""Synthetic meshes: counts, topology and closed-form geometry."""
import math

import numpy as np
import pytest

from npfem_workload import meshes, suspensions
from oracle import operators as O


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_icosphere_counts_and_topology(level):
    v, f = meshes.icosphere(level)
    assert v.shape[0] == 10 * 4 ** level + 2
    assert f.shape[0] == 20 * 4 ** level
    O.check_closed_manifold(f, v.shape[0])  # includes Euler characteristic 2
    assert O.hinges(f).shape[0] == 30 * 4 ** level
    assert O.volume(v, f) > 0.0  # outward orientation


def test_regular_icosahedron_closed_forms():
    # unit circumradius: edge a = 4 / sqrt(10 + 2 sqrt 5), V = (5/12)(3 + sqrt5) a^3, area = 5 sqrt3 a^2
    v, f = meshes.icosahedron()
    a = 4.0 / math.sqrt(10.0 + 2.0 * math.sqrt(5.0))
    edges = np.linalg.norm(v[f[:, 1]] - v[f[:, 0]], axis=1)
    assert np.allclose(edges, a, rtol=0, atol=1e-14)
    assert abs(a - 1.0514622242382672) < 1e-15
    assert abs(O.volume(v, f) - 5.0 / 12.0 * (3.0 + math.sqrt(5.0)) * a ** 3) < 1e-14
    assert abs(O.surface_area(v, f) - 5.0 * math.sqrt(3.0) * a * a) < 1e-13


def evans_fung_volume(R=meshes.RBC_RADIUS_UM):
    # V = 2 pi R^3 int_0^1 sqrt(1-rho^2)(c0 + c1 rho^2 + c2 rho^4) rho drho
    #   = pi R^3 (2 c0 / 3 + 4 c1 / 15 + 16 c2 / 105)
    c0, c1, c2 = meshes.EVANS_FUNG_C
    return math.pi * R ** 3 * (2 * c0 / 3 + 4 * c1 / 15 + 16 * c2 / 105)


def test_evans_fung_shape():
    x, f = meshes.rbc_mesh(3)
    R = meshes.RBC_RADIUS_UM
    # centre thickness R * c0 (the poles of the sphere map to the disc centre)
    top = x[np.argmax(x[:, 2] * (np.hypot(x[:, 0], x[:, 1]) < 1e-9))]
    assert abs(2 * top[2] - R * meshes.EVANS_FUNG_C[0]) < 1e-12
    assert abs(np.hypot(x[:, 0], x[:, 1]).max() - R) < 1e-12
    # discrete volume converges to the analytic integral at second order
    exact = evans_fung_volume()
    errs = []
    for level in (2, 3, 4):
        xv, fv = meshes.rbc_mesh(level)
        errs.append(exact - O.volume(xv, fv))
    assert all(e > 0 for e in errs)  # inscribed polyhedra
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5
    assert abs(exact - 94.09) < 0.01


def test_sphere_and_platelet_volumes_converge():
    xs, fs = meshes.sphere_mesh(4, 6.0)
    assert abs(O.volume(xs, fs) / (4 / 3 * math.pi * 216) - 1) < 3e-3
    xp, fp = meshes.platelet_mesh(2)
    exact = 4 / 3 * math.pi * 1.8 * 1.8 * 0.5
    assert 0 < exact - O.volume(xp, fp) < 0.05 * exact


def test_random_rotations_are_proper():
    rng = np.random.default_rng(0)
    R = suspensions.random_rotations(rng, 64)
    assert np.allclose(np.einsum("nij,nkj->nik", R, R), np.eye(3)[None], atol=1e-13)
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-13)


def test_suspension_layout():
    s = suspensions.uneven(n_rbc=3, n_plt=2, n_large=1)
    off = s.cell_offsets()
    assert list(np.diff(off)) == [642, 642, 642, 162, 162, 2562]
    assert s.x0.shape == (3, off[-1])
    mc, x0, v0, f, w = s.cell_arrays(4)
    assert mc.n_verts == 162 and x0.shape == (162, 3)
    # cell-local: rotated rest shape, same edge lengths as the rest mesh
    e0 = np.linalg.norm(mc.rest[mc.tris[:, 1]] - mc.rest[mc.tris[:, 0]], axis=1)
    e1 = np.linalg.norm(x0[mc.tris[:, 1]] - x0[mc.tris[:, 0]], axis=1)
    assert np.allclose(e0, e1, atol=1e-13)
    ratio = w / np.asarray(mc.weights)
    assert np.all((ratio > 0.8) & (ratio < 1.2))
