"""Edge cases of the GPU step against the oracle: a mesh class with no
cells in the batch, a one-cell batch, a single PD iteration per step, and
meshes beyond the local step's limits refused at batch creation."""
import numpy as np
import pytest

from npfem_workload import meshes, suspensions as W

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


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_mesh_class_without_cells(prec):
    """RBC and platelet classes with cells, the large class with none (its
    operators are built, its launches skipped); stiff twin, 2 steps x 4
    iterations, every cell against the oracle."""
    s = W.stiff(W.uneven(n_rbc=5, n_plt=3, n_large=0, n_steps=2, n_iter=4))
    if prec == "fp32":
        s = as_precision(s, np.float32)
    assert not np.any(s.cell_class == 2) and len(s.classes) == 3
    log(f"empty class {prec}")
    x, _ = run_gpu(s, prec)
    err = max_error(s, x, oracle_cells(s, range(s.n_cells)))
    log(f"empty class {prec} err {err:.3e}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_one_cell_one_iteration(prec):
    """One RBC, 5 stiff steps of a single PD iteration each."""
    s = W.stiff(W.rbc_lattice(n_cells=1, n_steps=5, n_iter=1))
    if prec == "fp32":
        s = as_precision(s, np.float32)
    log(f"one cell one iteration {prec}")
    x, _ = run_gpu(s, prec)
    err = max_error(s, x, oracle_cells(s, [0]))
    log(f"one cell one iteration {prec} err {err:.3e}")
    assert err <= TOL[prec]


def test_mesh_beyond_local_step_refused():
    """A 10242-vertex sphere (level 5) exceeds the widest local-step
    workgroup (512 threads x 11 vertices): refused at creation, FP32 too."""
    from paper_2011_04332_amd import _lib, solver
    s = W.uneven(n_rbc=1, n_plt=1, n_large=1, n_steps=1)
    big = W.large_class(5)
    s = W.Suspension([s.classes[0], s.classes[1], big], s.cell_class, s.origins,
                     *_restate(s, big), s.dt, s.n_iter, s.n_steps, "too-large")
    with pytest.raises(_lib.NpfemError) as e:
        solver.batch_from_suspension(s, precision="fp32")
    assert e.value.code == _lib.ERR_INVALID_ARG and "5632" in str(e.value)


def _restate(s, big):
    """State arrays with the last cell replaced by the big class's rest shape."""
    keep = s.cell_slice(s.n_cells - 1).start
    xb = big.rest.T
    cat = lambda a, b: np.concatenate([a[:, :keep], b], axis=1)
    return (cat(s.x0, xb), cat(s.v0, np.zeros_like(xb)), cat(s.forces, np.zeros_like(xb)),
            s.weights.copy())


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_run_as_one_launch_equals_steps(prec):
    """npfem_run: the uneven batch (three classes, per-cell weights) for 6
    steps as one graph launch gives bitwise the positions and velocities of 6
    npfem_step calls, twice in a row (the captured run replays), and the
    oracle's within the bound (FP32)."""
    import torch
    from paper_2011_04332_amd import solver
    s = W.stiff(W.uneven(n_rbc=6, n_plt=4, n_large=2, n_steps=6, n_iter=3))
    if prec == "fp32":
        s = as_precision(s, np.float32)
    # (fixed launch shapes: two autotuned batches may pick different ones)
    b1, p1, v1, f1, _ = solver.batch_from_suspension(s, precision=prec, autotune=False)
    for _ in range(s.n_steps):
        b1.step(f1, s.dt, s.n_iter)
    b1.sync_status()
    b2, p2, v2, f2, _ = solver.batch_from_suspension(s, precision=prec, autotune=False)
    x0, u0 = p2.clone(), v2.clone()
    log(f"run {prec}: one launch of {s.n_steps} steps")
    for rep in range(2):
        p2.copy_(x0)
        v2.copy_(u0)
        b2.run(f2, s.dt, s.n_iter, s.n_steps)
        b2.sync_status()
        torch.cuda.synchronize()
        assert torch.equal(p1, p2) and torch.equal(v1, v2), rep
    if prec == "fp32":
        err = max_error(s, p2.double().cpu().numpy(), oracle_cells(s, [0, 6, 10]))
        log(f"run fp32 err {err:.3e}")
        assert err <= TOL["fp32"]
    with pytest.raises(Exception):
        b2.run(f2, s.dt, s.n_iter, 0)
    b1.close()
    b2.close()


@pytest.mark.parametrize("stiff", [False, True])
def test_local_block_1024(stiff):
    """1024-thread local steps pinned for every class of an uneven batch
    (RBCs and platelets with two vertices per thread, 2562-vertex cells with
    three, the large mesh's elements in two LDS chunks), FP32, 3 steps x 3
    iterations; cells of every class against the oracle."""
    import torch
    from paper_2011_04332_amd import solver
    s = W.uneven(n_rbc=4, n_plt=3, n_large=2, n_steps=3, n_iter=3)
    if stiff:
        s = W.stiff(s)
    s = as_precision(s, np.float32)
    log(f"local block 1024 stiff={stiff}")
    b, pos, vel, f, _ = solver.batch_from_suspension(s, precision="fp32")
    for k in range(len(s.classes)):
        b.set_config(k, (1024, 64, 64, -1))
    for _ in range(s.n_steps):
        b.step(f, s.dt, s.n_iter)
    b.sync_status()
    torch.cuda.synchronize()
    assert all(b.config(k)[0] == 1024 for k in range(len(s.classes)))
    x = pos.double().cpu().numpy()
    b.close()
    cells = [0, 3, 4, 6, 7, 8]
    err = max_error(s, x, oracle_cells(s, cells))
    log(f"local block 1024 stiff={stiff} err {err:.3e}")
    assert err <= TOL["fp32"]


def test_local_block_1024_refused_for_fp64():
    """The 1024-thread local step exists for FP32 state only."""
    from paper_2011_04332_amd import _lib, solver
    s = W.uneven(n_rbc=2, n_plt=1, n_large=0, n_steps=1)
    b, _, _, _, _ = solver.batch_from_suspension(s, precision="fp64")
    try:
        with pytest.raises(_lib.NpfemError, match="1024"):
            b.set_config(0, (1024, 64, 64, -1))
    finally:
        b.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_whole_step_tuning_restores_state(prec):
    """The autotuner's whole-step trials (several classes, a 2562-vertex
    class) run real steps from the batch's state and restore it: an
    autotuned batch's steps equal, bitwise, those of a fresh batch pinned to
    the configuration the tuner chose."""
    import torch
    from paper_2011_04332_amd import solver
    s = as_precision(W.uneven(n_rbc=6, n_plt=4, n_large=2, n_steps=2, n_iter=3), np.float32)
    log(f"whole-step tuning {prec}")
    b, pos, vel, f, _ = solver.batch_from_suspension(s, precision=prec, autotune=True)
    for _ in range(s.n_steps):
        b.step(f, s.dt, s.n_iter)
    b.sync_status()
    torch.cuda.synchronize()
    cfgs = [b.config(k) for k in range(len(s.classes))]
    x_tuned, v_tuned = pos.clone(), vel.clone()
    b.close()
    b, pos, vel, f, _ = solver.batch_from_suspension(s, precision=prec)
    for k, cfg in enumerate(cfgs):
        b.set_config(k, (cfg[0], cfg[1], cfg[2], -1))  # sweeps: automatic, as tuned
    for _ in range(s.n_steps):
        b.step(f, s.dt, s.n_iter)
    b.sync_status()
    torch.cuda.synchronize()
    log(f"whole-step tuning {prec}: configs {cfgs}")
    assert torch.equal(pos, x_tuned) and torch.equal(vel, v_tuned)
    b.close()
