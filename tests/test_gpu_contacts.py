"""Contact potentials on the GPU (npfem_set_contacts) against the FP64 oracle.

Cells pressed onto a plane wall (every nearest contact point gives the same
half-space, so the FP32 nearest-point choice cannot differ from the
oracle's), and cells touching a spherical obstacle sampled by 162 points
(the nearest point decides the half-space; compared in FP64, where both
sides make the same choice). Bounds: FP64 1e-12, FP32 1e-6 of the cell
radius.
"""
import numpy as np
import pytest

from npfem_workload import suspensions as W

from gpu_helpers import as_precision, log, max_error, oracle_cells, run_gpu

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_04332_amd import _lib
    _lib.load()


def _oracle(s, cells, n_iter):
    from oracle import solver as S
    out = {}
    for c in cells:
        mc, x0, v0, f, w = s.cell_arrays(int(c))
        wc, ct = S.cell_contacts(s, int(c))
        cs = S.CellSolver(S.operators_for(mc), S.Params(tuple(w), mc.mass, s.dt), wc)
        out[int(c)] = cs.rollout(x0, v0, f, n_iter, s.n_steps, contacts=ct)
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dt", [1e-2, 1e-4])
def test_wall(prec, dt):
    s = W.wall_contacts(W.stiff(W.rbc_lattice(n_cells=12, n_steps=3), dt=dt), depth=0.4)
    if prec == "fp32":
        s = as_precision(s, np.float32)
    cells = [0, 5, 11]
    log(f"wall contacts {prec} dt {dt}")
    x, _ = run_gpu(s, prec, n_iter=5)
    err = max_error(s, x, _oracle(s, cells, 5))
    log(f"wall contacts {prec} dt {dt} err {err:.3e}")
    assert err <= TOL[prec]


def test_sphere_obstacle_fp64_uneven():
    """Spherical obstacles beside RBCs, platelets and large cells (FP64 takes
    meshes up to 2550 vertices: no large class), per-cell weights."""
    s = W.sphere_contacts(W.stiff(W.uneven(n_rbc=5, n_plt=4, n_large=0, n_steps=3)), overlap=0.4)
    cells = [0, 4, 5, 8]
    log("sphere contacts fp64")
    x, _ = run_gpu(s, "fp64", n_iter=5)
    err = max_error(s, x, _oracle(s, cells, 5))
    log(f"sphere contacts fp64 err {err:.3e}")
    assert err <= TOL["fp64"]


def test_contacts_with_16bit_product_and_refused_adjoint():
    import torch
    from paper_2011_04332_amd import _lib, solver
    s = as_precision(W.wall_contacts(W.stiff(W.rbc_lattice(n_cells=8, n_steps=3)), depth=0.4),
                     np.float32)
    x, _ = run_gpu(s, "fp16", n_iter=4)
    err = max_error(s, x, _oracle(s, [0, 7], 4))
    log(f"wall contacts fp16 err {err:.3e}")
    assert err <= 1e-5
    b, pos, vel, f, _ = solver.batch_from_suspension(s, "fp32")
    b.rollout(f, s.dt, 2, 2, 1)
    with pytest.raises(_lib.NpfemError) as e:
        b.rollout_adjoint(torch.zeros_like(pos))
    assert e.value.code == _lib.ERR_INVALID_ARG
    b.set_contacts(0.0)  # disabling is accepted
    b.close()
