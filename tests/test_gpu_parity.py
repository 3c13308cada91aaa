"""GPU path (through the C ABI) against the FP64 oracle, element by element.

Error metric: max over checked cells of max_v |x - x_ref| / R_cell with
R_cell = max_v |x_ref_v - centroid|. Bounds: FP64 1e-12, FP32 1e-6,
BF16/FP16 global step with refinement 1e-5. Cells are independent, so a
sampled cell of a large batch is checked exactly against a one-cell oracle run.
"""
import numpy as np
import pytest

from npfem_workload import suspensions as W
from oracle import solver as S

from gpu_helpers import as_precision, cell_error, log, max_error, oracle_cells, run_gpu

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16": 1e-5, "fp16": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_04332_amd import _lib
    _lib.load()  # fails loudly if the HIP library is missing


# FP64 over long runs: the oracle forms v = (q - x_n)/h from two nearly equal
# positions, losing log10(|x| / |q - x|) ~ 7 digits of v each step; the error
# it carries grows ~ n^2 (a velocity offset integrated twice). Two FP64
# evaluations of the same step definition (this one and the delta form
# A (q - x) = b - A x that the GPU uses) already differ by 2.3e-12 after
# 100 steps x 20 iterations of the single-RBC run, so the bound there is
# 1e-11; runs of <= 10 steps keep 1e-12.
FP64_LONG_RUN_TOL = 1e-11


def test_single_rbc_fp64_full_run():
    """1 RBC (162 vertices), FP64, 100 steps x 20 PD iterations, dt 1e-4."""
    s = W.single_rbc()
    log("single_rbc fp64 100x20")
    x, v = run_gpu(s, "fp64")
    ref = oracle_cells(s, [0])
    err = max_error(s, x, ref)
    log(f"single_rbc fp64 err {err:.3e}")
    assert err <= FP64_LONG_RUN_TOL
    assert np.abs(v.T - ref[0][1]).max() <= 1e-8 * max(1.0, np.abs(ref[0][1]).max())


def test_single_rbc_fp64_stiff():
    s = W.stiff(W.single_rbc(n_steps=10))
    log("single_rbc fp64 stiff dt 1e-2")
    x, _ = run_gpu(s, "fp64")
    err = max_error(s, x, oracle_cells(s, [0]))
    log(f"stiff fp64 err {err:.3e}")
    assert err <= TOL["fp64"]


@pytest.mark.parametrize("stiff", [False, True])
def test_rbc_lattice_fp32_sample(stiff):
    """64 RBCs (642 vertices): 192 columns span a ragged tile; 4 cells checked."""
    s = W.rbc_lattice(n_cells=64, n_steps=6 if stiff else 10)
    if stiff:
        s = W.stiff(s)
    s = as_precision(s, np.float32)
    log(f"rbc_lattice fp32 64 cells stiff={stiff}")
    x, _ = run_gpu(s, "fp32")
    cells = [0, 17, 42, 63]
    err = max_error(s, x, oracle_cells(s, cells))
    log(f"rbc_lattice fp32 stiff={stiff} err {err:.3e}")
    assert err <= TOL["fp32"]


def test_rbc_lattice_full_size_sampled():
    """The benchmark workload at full size (4096 RBCs), a few steps, 3 sampled cells."""
    s = as_precision(W.rbc_lattice(n_steps=5), np.float32)
    log("rbc_lattice fp32 4096 cells, 5 steps")
    x, _ = run_gpu(s, "fp32")
    cells = W.sample_cells(s, [3])
    err = max_error(s, x, oracle_cells(s, cells))
    log(f"rbc_lattice 4096 err {err:.3e}")
    assert err <= TOL["fp32"]


@pytest.mark.parametrize("n_cells", [1024, 2048])
def test_fp32_product_rows_split_stiff(n_cells):
    """The FP32 default product for few columns: 1024 (2048) RBCs make 64
    (128) column blocks of 48, so the column-stationary kernel splits the row
    pairs over 4 (2) workgroups per block. Stiff twin (the product shapes the
    positions), 3 steps x 2 PD iterations, 3 sampled cells against the oracle."""
    from paper_2011_04332_amd import solver
    import torch
    s = as_precision(W.stiff(W.rbc_lattice(n_cells=n_cells, n_steps=3, n_iter=2)), np.float32)
    log(f"fp32 row-split product, {n_cells} RBCs, stiff")
    b, pos, vel, f, _ = solver.batch_from_suspension(s, precision="fp32")
    for _ in range(s.n_steps):
        b.step(f, s.dt, s.n_iter)
    b.sync_status()
    torch.cuda.synchronize()
    cfg = b.config(0)
    x = pos.double().cpu().numpy()
    b.close()
    assert tuple(cfg[1:3]) == (0, 48), cfg  # the column-stationary kernel by default
    cells = [0, n_cells // 2 + 5, n_cells - 1]
    err = max_error(s, x, oracle_cells(s, cells))
    log(f"row-split product {n_cells} err {err:.3e}")
    assert err <= TOL["fp32"]


@pytest.mark.parametrize("stiff", [False, True])
def test_uneven_batch_per_cell_weights(stiff):
    """RBC + platelet + large-cell classes with per-cell weights (+-20 %)."""
    s = W.uneven(n_rbc=20, n_plt=12, n_large=3, n_steps=3 if stiff else 4)
    if stiff:
        s = W.stiff(s)
    s = as_precision(s, np.float32)
    log(f"uneven fp32 stiff={stiff} (autotuned launch shapes)")
    x, _ = run_gpu(s, "fp32", autotune=True)
    cells = [0, 19, 20, 31, 32, 34]
    err = max_error(s, x, oracle_cells(s, cells))
    log(f"uneven stiff={stiff} err {err:.3e}")
    assert err <= TOL["fp32"]


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_mixed_precision_refined(prec):
    s = as_precision(W.precision_sweep(n_rbc=48, n_plt=16, n_steps=5), np.float32)
    log(f"precision {prec}")
    x, _ = run_gpu(s, prec)
    cells = [0, 47, 48, 63]
    err = max_error(s, x, oracle_cells(s, cells))
    log(f"precision {prec} err {err:.3e}")
    assert err <= TOL[prec]


def test_mixed_precision_sweeps_skipped_on_lattice():
    """16-bit global step with the automatic sweep count on lattice cells
    (uniform weights, dt 1e-4): the a-priori bound on the product's error is
    below the FP32 rounding of the coordinates for every cell, so the sweeps
    are skipped on the device. Results equal a run pinned to 0 sweeps bitwise,
    and the error against the oracle stays at the FP32 run's level."""
    s = as_precision(W.rbc_lattice(n_cells=64, n_steps=5), np.float32)
    cells = [0, 37, 63]
    ref = oracle_cells(s, cells)
    x32, _ = run_gpu(s, "fp32")
    err32 = max_error(s, x32, ref)
    for prec in ("fp16", "bf16"):
        log(f"lattice {prec} automatic sweeps")
        x_auto, _ = run_gpu(s, prec)
        x_none, _ = run_gpu(s, prec, n_refine=0)
        assert np.array_equal(x_auto, x_none)
        err = max_error(s, x_auto, ref)
        log(f"lattice {prec} err {err:.3e} (fp32 {err32:.3e})")
        assert err <= max(2.0 * err32, 2e-7)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_mixed_precision_uneven_adaptive(prec):
    """Per-cell weights (+-20 %) make the shared class operator inexact for
    every cell. At dt 1e-4 the mass term dominates A and the a-priori bound
    lets the device skip the correction; on the stiff twin (dt 1e-2) it must
    not: the sweeps run (the result differs from a run without them). Both
    match the oracle within the reduced-precision bound."""
    cells = [0, 19, 20, 31, 32, 34]
    for stiff in (False, True):
        s = W.uneven(n_rbc=20, n_plt=12, n_large=3, n_steps=3)
        s = as_precision(W.stiff(s) if stiff else s, np.float32)
        log(f"uneven {prec} stiff={stiff} automatic sweeps")
        x_auto, _ = run_gpu(s, prec, autotune=True)
        if stiff:
            x_none, _ = run_gpu(s, prec, n_refine=0)
            assert not np.array_equal(x_auto, x_none)
        err = max_error(s, x_auto, oracle_cells(s, cells))
        log(f"uneven {prec} stiff={stiff} err {err:.3e}")
        assert err <= TOL[prec]


# every global-step kernel shape (14 tiled shapes, then the column-stationary
# kernel, reported with tile rows 0), forced through set_config
GEMM_SHAPES = [(64, 64), (64, 128), (128, 64), (128, 128), (96, 64), (96, 128), (224, 32),
               (224, 64), (96, 96), (224, 96), (224, 128), (64, 96), (128, 96), (64, 32),
               (0, 48)]


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_every_gemm_shape(prec):
    """17 RBCs (51 columns: one full column-stationary workgroup and a ragged
    one of 3 columns; ragged tiles for every tiled shape) plus 5 platelets,
    each kernel shape pinned in turn; 3 steps; 3 cells against the oracle."""
    import torch
    from paper_2011_04332_amd import solver
    s = as_precision(W.precision_sweep(n_rbc=17, n_plt=5, n_steps=3), np.float32)
    cells = [0, 16, 19]
    ref = oracle_cells(s, cells)
    for bm, bn in GEMM_SHAPES:
        b, pos, vel, f, _ = solver.batch_from_suspension(s, precision=prec)
        for k in range(len(s.classes)):
            b.set_config(k, (256, bm, bn, -1))
        log(f"{prec} gemm shape {bm}x{bn}")
        for _ in range(s.n_steps):
            b.step(f, s.dt, s.n_iter)
        b.sync_status()
        torch.cuda.synchronize()
        assert b.config(0)[1:3] == (bm, bn)
        x = pos.double().cpu().numpy()
        b.close()
        err = max_error(s, x, ref)
        log(f"{prec} gemm shape {bm}x{bn} err {err:.3e}")
        assert err <= TOL[prec], (bm, bn, err)


def test_momentum_and_rest_invariants():
    import torch
    from paper_2011_04332_amd import solver
    s = as_precision(W.rbc_lattice(n_cells=16, n_steps=1), np.float32)
    b, pos, vel, f, _ = solver.batch_from_suspension(s, "fp32")
    v0 = vel.double().clone()
    b.step(f, 1e-2, 5)
    b.sync_status()
    # sum m v_{n+1} = sum m v_n + h sum f, per cell
    n = s.classes[0].n_verts
    dv = (vel.double() - v0).reshape(3, 16, n).sum(-1)
    df = 1e-2 / 1e-3 * f.double().reshape(3, 16, n).sum(-1)
    assert torch.allclose(dv, df, rtol=0, atol=1e-4 * df.abs().max().item() + 1e-6)
    b.close()
    # rest state with no forces stays at rest
    z = W.rbc_lattice(n_cells=8, n_steps=1)
    z.forces[:] = 0.0
    b, pos, vel, f, _ = solver.batch_from_suspension(as_precision(z, np.float32), "fp32")
    x0 = pos.clone()
    for _ in range(5):
        b.step(f, 1e-4, 10)
    b.sync_status()
    R = 3.91
    assert (pos - x0).abs().max().item() <= 1e-6 * R
    b.close()


def test_energy_monotone_stiff_fp64():
    from paper_2011_04332_amd import solver
    s = W.stiff(W.single_rbc(n_steps=1))
    s.x0 = s.x0 + 0.05 * np.random.default_rng(0).standard_normal(s.x0.shape)
    b, pos, vel, f, _ = solver.batch_from_suspension(s, "fp64", energy=True)
    b.step(f, s.dt, 25)
    E = b.energy()[:, 0]
    b.close()
    assert np.all(np.diff(E) <= 1e-12 * abs(E[0])) and E[-1] < E[0]
    mc, x0, v0, fo, w = s.cell_arrays(0)
    cs = S.CellSolver(S.operators_for(mc), S.Params(tuple(w), mc.mass, s.dt))
    _, _, Eo = cs.step(x0, v0, fo, 25, record_energy=True)
    assert np.allclose(E, Eo[:25], rtol=1e-10, atol=0)


def test_bitwise_reproducible_and_graph_equals_eager():
    s = as_precision(W.uneven(n_rbc=6, n_plt=4, n_large=1, n_steps=3), np.float32)
    a, _ = run_gpu(s, "fp32")
    b, _ = run_gpu(s, "fp32")
    c, _ = run_gpu(s, "fp32", graph=False)
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_nonfinite_forces_are_reported():
    import torch
    from paper_2011_04332_amd import _lib, solver
    s = W.rbc_lattice(n_cells=2, n_steps=1)
    b, pos, vel, f, _ = solver.batch_from_suspension(s, "fp32")
    f[0, 5] = float("nan")
    b.step(f, 1e-4, 2)
    with pytest.raises(_lib.NpfemError) as e:
        b.sync_status()
    assert e.value.code == _lib.ERR_NONFINITE
    b.sync_status()  # flag cleared
    b.close()


def test_time_step_change_refactors():
    s = as_precision(W.rbc_lattice(n_cells=4, n_steps=2), np.float32)
    import torch
    from paper_2011_04332_amd import solver
    b, pos, vel, f, _ = solver.batch_from_suspension(s, "fp32")
    b.step(f, 1e-4, 5)
    b.step(f, 1e-2, 5)
    b.sync_status()
    x = pos.double().cpu().numpy()
    b.close()
    for c in (0, 3):
        mc, x0, v0, fo, w = s.cell_arrays(c)
        o = S.operators_for(mc)
        xa, va, _ = S.CellSolver(o, S.Params(tuple(w), mc.mass, 1e-4)).step(x0, v0, fo, 5)
        xb, _, _ = S.CellSolver(o, S.Params(tuple(w), mc.mass, 1e-2)).step(xa, va, fo, 5)
        assert cell_error(s, x, c, xb) <= TOL["fp32"]
