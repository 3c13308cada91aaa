"""Finite-difference gradients of the oracle pinned to a closed form."""
import numpy as np

from npfem_workload import meshes, suspensions as W
from oracle import gradients as Gr


def test_force_gradient_free_flight_closed_form():
    """All weights zero: x_T = x0 + T h v0 + h^2 T(T+1)/2 f/m, so
    dL/df = 2 (x_T - target) h^2 T(T+1) / (2 m), and dL/dw = 0 at w = 0 only
    through the elastic terms (checked against the closed form here)."""
    x, f = meshes.rbc_mesh(2)
    mc = W.MeshClass("rbc162", x, f, weights=(0.0, 0.0, 0.0, 0.0))
    rng = np.random.default_rng(0)
    x0 = x.copy()
    v0 = 0.1 * rng.standard_normal(x.shape)
    fo = 0.05 * rng.standard_normal(x.shape)
    target = x0 * 1.01
    T, h, m = 4, 1e-2, 1e-3
    xT, _ = Gr.rollout(mc, (0, 0, 0, 0), m, h, x0, v0, fo, 3, T)
    closed = 2.0 * (xT - target) * h * h * T * (T + 1) / (2.0 * m)
    comps = [(0, 0), (17, 1), (101, 2)]
    fd = Gr.fd_force_grad(mc, (0, 0, 0, 0), m, h, x0, v0, fo, target, 3, T, comps, h=1e-3)
    assert np.allclose(fd, [closed[v, d] for v, d in comps], rtol=1e-7, atol=1e-12)


def test_weight_gradient_converges_with_step():
    """Central differences at relative steps h and h/3 agree to O(h^2)."""
    s = W.stiff(W.adjoint_rbcs(n_cells=1, n_steps=2, n_iter=3))
    mc, x0, v0, f, w = s.cell_arrays(0)
    target = s.extra["target"].T
    g1 = Gr.fd_weight_grad(mc, w, mc.mass, s.dt, x0, v0, f, target, 3, 2, h=3e-3)
    g2 = Gr.fd_weight_grad(mc, w, mc.mass, s.dt, x0, v0, f, target, 3, 2, h=1e-3)
    assert np.all(np.abs(g1 - g2) <= 1e-4 * np.abs(g2) + 1e-12)
    assert np.all(np.abs(g2) > 0)
