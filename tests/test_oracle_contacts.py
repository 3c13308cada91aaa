"""Pins of the oracle's contact projection and contact potentials.

* The projection: a vertex outside its nearest contact point's half-space is
  unchanged, one inside lands on the tangent plane (its penetration removed
  exactly); the nearest point decides, the first on ties; with a single
  plane it is the textbook half-space projection.
* Inactive contacts (every vertex outside): the contact term adds w_c q to
  both sides, so the converged step equals the step without contacts.
* A plane wall: the contact set of every vertex is the same half-space, the
  local step minimises exactly, so the PD objective (with the contact term)
  never increases over the iterations; the wall reduces the penetration.
"""
import numpy as np

from npfem_workload import meshes, suspensions as W
from oracle import contacts as C
from oracle import operators as ops_mod
from oracle import solver as S


def test_projection_half_space():
    pts = np.array([[0.0, 0.0, 0.0], [5.0, 0.0, 0.0]])
    nrm = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    q = np.array([[0.1, 0.2, 0.5], [0.3, -0.1, -0.4], [4.0, 0.0, 0.0], [2.5, 0.0, -1.0]])
    p = C.project_contacts(q, pts, nrm)
    assert np.array_equal(p[0], q[0])                       # outside the plane z >= 0
    assert np.allclose(p[1], [0.3, -0.1, 0.0], atol=0)      # pulled onto it
    assert np.allclose(p[2], [5.0, 0.0, 0.0], atol=1e-15)   # nearest is the second point
    # equidistant (2.5 from both? no: |(2.5,0,-1)-(0,0,0)| = |(2.5,0,-1)-(5,0,0)|): first wins
    assert np.allclose(p[3], [2.5, 0.0, 0.0], atol=0)
    # a random plane: the textbook projection onto {(p - y) . n >= 0}
    rng = np.random.default_rng(0)
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    y = rng.standard_normal(3)
    qs = rng.standard_normal((50, 3))
    got = C.project_contacts(qs, y[None], n[None])
    sd = (qs - y) @ n
    want = qs - np.minimum(sd, 0.0)[:, None] * n
    assert np.allclose(got, want, atol=1e-15)
    assert np.all((got - y) @ n >= -1e-14)


def _cell(contacts=None, wc=10.0, dt=1e-2):
    x, t = meshes.rbc_mesh(2)
    o = ops_mod.build_operators(x, t)
    prm = S.Params((1.0, 1.0, 0.01, 10.0), 1e-3, dt)
    return o, S.CellSolver(o, prm, wc if contacts is not None else 0.0)


def test_inactive_contacts_leave_the_converged_step():
    x, t = meshes.rbc_mesh(2)
    o = ops_mod.build_operators(x, t)
    prm = S.Params((1.0, 1.0, 0.01, 10.0), 1e-3, 1e-2)
    rng = np.random.default_rng(1)
    x0 = o.X + 0.02 * rng.standard_normal(o.X.shape)
    f = 0.05 * rng.standard_normal(o.X.shape)
    far = (np.array([[0.0, 0.0, -50.0]]), np.array([[0.0, 0.0, 1.0]]))  # everything outside
    a, _, _ = S.CellSolver(o, prm).step(x0, np.zeros_like(x0), f, 300)
    b, _, _ = S.CellSolver(o, prm, 10.0).step(x0, np.zeros_like(x0), f, 300, contacts=far)
    assert np.abs(a - b).max() <= 1e-10 * o.radius


def test_wall_objective_monotone_and_penetration_reduced():
    s = W.wall_contacts(W.stiff(W.rbc_lattice(n_cells=1, n_steps=1)), depth=0.4, weight=10.0)
    mc, x0, v0, f, w = s.cell_arrays(0)
    o = S.operators_for(mc)
    wc, ct = S.cell_contacts(s, 0)
    cs = S.CellSolver(o, S.Params(tuple(w), mc.mass, s.dt), wc)
    _, _, E = cs.step(x0, v0, f, 30, record_energy=True, contacts=ct)
    E = np.asarray(E)
    assert np.all(np.diff(E) <= 1e-12 * abs(E[0])) and E[-1] < E[0]
    plane = ct[0][0, 2]
    xc, _ = cs.rollout(x0, v0, f, 10, 3, contacts=ct)
    xn, _ = S.CellSolver(o, S.Params(tuple(w), mc.mass, s.dt)).rollout(x0, v0, f, 10, 3)
    pen = lambda x: np.maximum(plane - x[:, 2], 0.0).sum()
    assert pen(xc) < 0.5 * pen(xn) and pen(xn) > 0
