"""Immersed-boundary transfer on the GPU (npfem_ibm_interpolate /
npfem_ibm_spread) against the oracle (oracle/ibm.py), and the solid step
coupled to a synthetic flow through them.

Cells sit in a periodic 48 x 40 x 44 grid (dx 0.5 um) or 24 x 20 x 22 (dx 1 um), some across the
periodic seam. Bounds: FP64 interpolation 1e-13 and spreading 1e-11 of the
largest value (the spreading's 64-bit fixed point keeps ~40 bits below the
largest possible contribution); FP32 1e-6 (FP32 weights and sums).
"""
import numpy as np
import pytest

from npfem_workload import suspensions as W
from oracle import ibm

from gpu_helpers import as_precision, log

pytestmark = pytest.mark.gpu

DIMS, DX = (48, 40, 44), 0.5
ORIGIN = np.array([-1.0, 0.5, 2.0])


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_04332_amd import _lib
    _lib.load()


def _setup(prec, dims=DIMS, dx=DX, n_rbc=4, n_plt=2):
    """A small RBC + platelet batch placed in the periodic box (the last cell
    straddles the seam)."""
    s = W.precision_sweep(n_rbc=n_rbc, n_plt=n_plt, n_steps=3)
    if prec == "fp32":
        s = as_precision(s, np.float32)
    L = dx * np.array(dims)
    rng = np.random.default_rng(4)
    org = ORIGIN + rng.uniform(0.2, 0.8, (s.n_cells, 3)) * L
    org[-1] = ORIGIN + L - 0.3  # across the seam
    return s, org


def _global(s, x, org):
    """Global positions [sum_N, 3] from cell-local SoA x [3, sum_N]."""
    out = []
    for c in range(s.n_cells):
        out.append(org[c][None, :] + x[:, s.cell_slice(c)].T)
    return np.concatenate(out)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dx", [0.5, 1.0])
def test_interpolate_and_spread(prec, dx):
    """dx 0.5: a cell's support box exceeds the spreading kernel's LDS box
    (global atomics per contribution); dx 1.0: it fits (LDS box, one global
    atomic per node)."""
    import torch
    from paper_2011_04332_amd import solver
    dims = DIMS if dx == 0.5 else (24, 20, 22)
    s, org = _setup(prec, dims, dx)
    b, pos, vel, f, _ = solver.batch_from_suspension(s, precision=prec)
    dt_ = pos.dtype
    rng = np.random.default_rng(5)
    u = rng.standard_normal((3,) + dims)
    ug = torch.tensor(u.reshape(3, -1, order="F"), dtype=dt_, device="cuda").contiguous()
    u_ref = u.astype(np.float32).astype(np.float64) if prec == "fp32" else u
    orgd = torch.tensor(org, dtype=torch.float64, device="cuda").contiguous()
    X = _global(s, pos.double().cpu().numpy(), org)
    log(f"ibm interpolate {prec}")
    U = b.ibm_interpolate(orgd, ug, dims, dx, ORIGIN)
    U_ref = ibm.interpolate(u_ref, X, ORIGIN, dx)
    err = np.abs(U.double().cpu().numpy().T - U_ref).max() / np.abs(U_ref).max()
    log(f"ibm interpolate {prec} rel err {err:.3e}")
    assert err <= (1e-13 if prec == "fp64" else 1e-6)
    F = rng.standard_normal(pos.shape) * 0.05
    Fg = torch.tensor(F, dtype=dt_, device="cuda").contiguous()
    F_ref = Fg.double().cpu().numpy().T
    log(f"ibm spread {prec}")
    g1 = b.ibm_spread(orgd, Fg, dims, dx, ORIGIN)
    g2 = b.ibm_spread(orgd, Fg, dims, dx, ORIGIN)
    b.sync_status()
    assert torch.equal(g1, g2)  # bitwise reproducible
    f_ref = ibm.spread(F_ref, X, dims, ORIGIN, dx).reshape(3, -1, order="F")
    got = g1.double().cpu().numpy()
    err = np.abs(got - f_ref).max() / np.abs(f_ref).max()
    log(f"ibm spread {prec} rel err {err:.3e}")
    assert err <= (1e-11 if prec == "fp64" else 1e-6)
    if prec == "fp64":  # total force conserved
        assert np.allclose(got.sum(1) * dx ** 3, F_ref.sum(0), rtol=0, atol=1e-12)
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_coupled_shear_flow(prec):
    """Three steps of the solid coupled to a shear flow u = (rate (y - y0), 0, 0):
    per step the flow velocity is interpolated at the vertices, the penalty
    force F = kappa (U - v) drives the step, and -F is spread back; GPU
    (interpolation, step, spreading in the library) against the oracle doing
    the same chain, positions at the step bounds (FP64 1e-12, FP32 1e-6 of
    the cell radius) and the last spread force density."""
    import torch
    from oracle import solver as S
    from paper_2011_04332_amd import solver
    s, org = _setup(prec, n_rbc=3, n_plt=1)
    s = W.stiff(s, dt=1e-3)
    kappa, rate = 2e-2, 50.0
    g = np.stack(np.meshgrid(*[np.arange(k) for k in DIMS], indexing="ij"), 0)
    yg = ORIGIN[1] + DX * g[1]
    u = np.zeros((3,) + DIMS)
    u[0] = rate * (yg - yg.mean())
    b, pos, vel, f, _ = solver.batch_from_suspension(s, precision=prec)
    dt_ = pos.dtype
    ug = torch.tensor(u.reshape(3, -1, order="F"), dtype=dt_, device="cuda").contiguous()
    u_ref = u.astype(np.float32).astype(np.float64) if prec == "fp32" else u
    orgd = torch.tensor(org, dtype=torch.float64, device="cuda").contiguous()
    Fb = torch.empty_like(pos)
    for _ in range(3):
        U = b.ibm_interpolate(orgd, ug, DIMS, DX, ORIGIN)
        Fb.copy_(kappa * (U - vel))
        b.step(Fb, s.dt, 5)
        fg = b.ibm_spread(orgd, -Fb, DIMS, DX, ORIGIN)
    b.sync_status()
    x_gpu = pos.double().cpu().numpy()
    fg = fg.double().cpu().numpy()
    b.close()
    # oracle chain (each cell independent given the flow)
    rd = (lambda a: a.astype(np.float32).astype(np.float64)) if prec == "fp32" else (lambda a: a)
    err = 0.0
    xs, Fs = [], []
    for c in range(s.n_cells):
        mc, x, v, _, w = s.cell_arrays(c)
        cs = S.CellSolver(S.operators_for(mc), S.Params(tuple(w), mc.mass, s.dt))
        for _ in range(3):
            Ui = ibm.interpolate(u_ref, org[c] + x, ORIGIN, DX)
            F = rd(kappa * (Ui - v))
            xprev = x
            x, v, _ = cs.step(x, v, F, 5)
        err = max(err, S.rel_position_error(x_gpu[:, s.cell_slice(c)].T, x))
        xs.append(org[c] + xprev)
        Fs.append(F)
    log(f"coupled shear {prec} position err {err:.3e}")
    assert err <= (1e-12 if prec == "fp64" else 1e-6)
    # the last spreading happened at the positions after the last step
    X_last = _global(s, x_gpu, org)
    f_ref = ibm.spread(-np.concatenate(Fs), X_last, DIMS, ORIGIN, DX).reshape(3, -1, order="F")
    e2 = np.abs(fg - f_ref).max() / np.abs(f_ref).max()
    log(f"coupled shear {prec} spread err {e2:.3e}")
    assert e2 <= (1e-9 if prec == "fp64" else 1e-4)
