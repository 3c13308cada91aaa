"""Viscous (Rayleigh-type) damping on the GPU (npfem_set_damping) against the
FP64 oracle, cell by cell.

C = alpha m I + beta K_d, K_d = (w_s + w_a) L_tri + w_b L_bend, taken
implicitly at the end-of-step velocity. On the GPU the mass part enters the
first increment and the local step's coefficient of delta, the stiffness
part a sparse product of the two Laplacians per PD iteration, and both the
factorised operator A + C/h. Bounds as in the other parity tests: FP64
1e-12, FP32 1e-6, 16-bit global step with refinement 1e-5 (relative to the
cell radius).
"""
import numpy as np
import pytest

from npfem_workload import suspensions as W

from gpu_helpers import as_precision, log, max_error, oracle_cells, run_gpu

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16": 1e-5, "fp16": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_04332_amd import _lib
    _lib.load()


def damped(s, alpha, beta):
    for mc in s.classes:
        mc.damping = (float(alpha), float(beta))
    return s


# (dt, alpha, beta): alpha h = 0.2 and beta/h = 1 on the stiff twin, alpha h =
# 0.02 and beta/h = 1 at the workloads' own time step
CASES = {"stiff": (1e-2, 20.0, 1e-2), "nominal": (1e-4, 200.0, 1e-4),
         "mass_only": (1e-2, 20.0, 0.0), "stiffness_only": (1e-2, 0.0, 1e-2)}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(CASES))
def test_damped_lattice(prec, case):
    dt, alpha, beta = CASES[case]
    s = W.rbc_lattice(n_cells=24, n_steps=4)
    s = damped(W.stiff(s, dt=dt), alpha, beta)
    if prec == "fp32":
        s = as_precision(s, np.float32)
    cells = [0, 11, 23]
    log(f"damped lattice {case} {prec}")
    x, _ = run_gpu(s, prec, n_iter=5)
    err = max_error(s, x, oracle_cells(s, cells, n_iter=5))
    log(f"damped lattice {case} {prec} err {err:.3e}")
    assert err <= TOL[prec], (case, prec, err)


def test_damped_uneven_per_cell_weights():
    """Per-cell weights (+-20 %) with damping on the three mesh classes: the
    correction sweeps solve each cell's own damped system."""
    s = W.uneven(n_rbc=6, n_plt=4, n_large=2, n_steps=3)
    # (beta/h = 0.2: with +-20 % weights the shared operator must still
    # contract the correction, which the library checks)
    s = as_precision(damped(W.stiff(s), 20.0, 2e-3), np.float32)
    cells = [0, 5, 6, 9, 10, 11]
    log("damped uneven fp32")
    x, _ = run_gpu(s, "fp32", n_iter=5)
    err = max_error(s, x, oracle_cells(s, cells, n_iter=5))
    log(f"damped uneven err {err:.3e}")
    assert err <= TOL["fp32"]


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_damped_low_precision(prec):
    s = W.precision_sweep(n_rbc=17, n_plt=5, n_steps=3)
    s = as_precision(damped(W.stiff(s), 20.0, 1e-2), np.float32)
    cells = [0, 16, 19]
    log(f"damped {prec}")
    x, _ = run_gpu(s, prec, n_iter=4)
    err = max_error(s, x, oracle_cells(s, cells, n_iter=4))
    log(f"damped {prec} err {err:.3e}")
    assert err <= TOL[prec]


def test_damped_momentum_balance_and_adjoint_refused():
    """(1 + alpha h) sum m v_{n+1} = sum m v_n + h sum f per cell (the
    elastic forces and K_d have no net force), on the GPU; the adjoint
    refuses a damped batch."""
    import torch
    from paper_2011_04332_amd import _lib, solver
    alpha, beta, h, m = 20.0, 1e-2, 1e-2, 1e-3
    s = damped(W.stiff(W.rbc_lattice(n_cells=8, n_steps=1)), alpha, beta)
    b, pos, vel, f, _ = solver.batch_from_suspension(s, "fp64")
    v0 = vel.clone()
    b.step(f, h, 5)
    b.sync_status()
    n = s.classes[0].n_verts
    lhs = (1.0 + alpha * h) * m * vel.reshape(3, 8, n).sum(-1)
    rhs = m * v0.reshape(3, 8, n).sum(-1) + h * f.reshape(3, 8, n).sum(-1)
    assert torch.allclose(lhs, rhs, rtol=0, atol=1e-13)
    b.rollout(f, h, 2, 2, 1)
    with pytest.raises(_lib.NpfemError) as e:
        b.rollout_adjoint(torch.zeros_like(pos))
    assert e.value.code == _lib.ERR_INVALID_ARG
    b.close()
