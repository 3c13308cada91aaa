"""Pins of the oracle's immersed-boundary transfer (Peskin's 4-point kernel).

* The kernel's defining properties (Peskin 2002): sum_j phi(r - j) = 1,
  sum_j (r - j) phi(r - j) = 0, sum_j phi(r - j)^2 = 3/8, and the even and the
  odd nodes each carry 1/2, for any r; phi(0) = 1/2, phi(1) = 1/4, phi(2) = 0.
* Interpolation reproduces constant and linear fields exactly (from the two
  moment conditions), and equals the direct sum over every node of a tiny
  periodic grid.
* Spreading conserves the total force and its first moment (sum_g f_g dx^3 =
  sum_v F_v, sum_g x_g f_g dx^3 = sum_v X_v F_v away from the periodic seam),
  and is the adjoint of interpolation: sum_v U(X_v).F_v = sum_g u_g.f_g dx^3.
"""
import numpy as np

from oracle import ibm


def test_kernel_moments():
    rng = np.random.default_rng(0)
    r = rng.uniform(0.0, 1.0, 200)
    j = np.arange(-3, 5)
    P = ibm.phi(r[:, None] - j[None, :])
    assert np.allclose(P.sum(1), 1.0, atol=1e-15)
    assert np.allclose(((r[:, None] - j[None, :]) * P).sum(1), 0.0, atol=1e-15)
    assert np.allclose((P ** 2).sum(1), 3.0 / 8.0, atol=1e-15)
    assert np.allclose(P[:, (j % 2) == 0].sum(1), 0.5, atol=1e-15)
    assert np.allclose(ibm.phi(np.array([0.0, 1.0, 2.0, 2.5])), [0.5, 0.25, 0.0, 0.0], atol=1e-16)


def _field(shape, rng):
    return rng.standard_normal((3,) + shape)


def test_interpolation_exact_for_linear_fields_and_equals_direct_sum():
    rng = np.random.default_rng(1)
    shape, dx, origin = (16, 12, 10), 0.5, np.array([-1.0, 2.0, 0.25])
    X = origin + dx * rng.uniform(3.0, 7.0, (40, 3))  # well inside: no periodic seam
    g = np.stack(np.meshgrid(*[np.arange(k) for k in shape], indexing="ij"), 0)
    xg = origin[:, None, None, None] + dx * g
    A = rng.standard_normal((3, 3))
    c = rng.standard_normal(3)
    u = np.einsum("de,e...->d...", A, xg) + c[:, None, None, None]
    U = ibm.interpolate(u, X, origin, dx)
    assert np.allclose(U, X @ A.T + c, atol=1e-12)
    # any field, tiny grid, positions anywhere (including across the seam)
    small = (6, 5, 7)
    us = _field(small, rng)
    Xs = origin + dx * rng.uniform(-2.0, 9.0, (25, 3))
    assert np.allclose(ibm.interpolate(us, Xs, origin, dx), ibm.interpolate_direct(us, Xs, origin, dx),
                       atol=1e-13)


def test_spreading_conserves_force_and_moment_and_is_adjoint():
    rng = np.random.default_rng(2)
    shape, dx, origin = (20, 18, 16), 0.4, np.array([0.3, -0.2, 1.0])
    X = origin + dx * rng.uniform(4.0, 12.0, (60, 3))
    F = rng.standard_normal((60, 3))
    f = ibm.spread(F, X, shape, origin, dx)
    g = np.stack(np.meshgrid(*[np.arange(k) for k in shape], indexing="ij"), 0)
    xg = origin[:, None, None, None] + dx * g
    vol = dx ** 3
    assert np.allclose(f.reshape(3, -1).sum(1) * vol, F.sum(0), atol=1e-12)
    mom = np.einsum("aijk,bijk->ab", xg, f) * vol  # sum_g x_g (x) f_g
    assert np.allclose(mom, X.T @ F, atol=1e-11)
    u = _field(shape, rng)
    lhs = np.sum(ibm.interpolate(u, X, origin, dx) * F)
    rhs = np.sum(u * f) * vol
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
