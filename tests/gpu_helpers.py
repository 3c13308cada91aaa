"""Shared helpers for the GPU parity tests (GPU path via the C ABI, oracle on
the CPU, identical seeded inputs)."""
from __future__ import annotations

import sys

import numpy as np

from oracle import solver as S


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def as_precision(susp, dtype):
    """Copy of a suspension with state, forces and weights rounded to dtype
    (the oracle then starts from exactly what the GPU receives)."""
    from npfem_workload.suspensions import Suspension
    r = lambda a: a.astype(dtype).astype(np.float64)
    return Suspension(susp.classes, susp.cell_class, susp.origins, r(susp.x0), r(susp.v0),
                      r(susp.forces), (susp.weights if susp.uniform_weights() else r(susp.weights)), susp.dt, susp.n_iter, susp.n_steps,
                      susp.name, dict(susp.extra))


def run_gpu(susp, precision="fp32", n_steps=None, n_iter=None, dt=None, **kw):
    """Runs the suspension on cuda:0; returns (x, v) as float64 [3, sum_N]."""
    import torch
    from paper_2011_04332_amd import solver
    b, pos, vel, f, meshes = solver.batch_from_suspension(susp, precision=precision, **kw)
    n_steps = susp.n_steps if n_steps is None else n_steps
    n_iter = susp.n_iter if n_iter is None else n_iter
    dt = susp.dt if dt is None else dt
    for _ in range(n_steps):
        b.step(f, dt, n_iter)
    b.sync_status()
    torch.cuda.synchronize()
    x = pos.double().cpu().numpy()
    v = vel.double().cpu().numpy()
    b.close()
    return x, v


def oracle_cells(susp, cells, n_steps=None, n_iter=None, dt=None):
    """{cell: (x [N,3], v [N,3])} from the FP64 oracle."""
    out = {}
    for c in cells:
        mc, x0, v0, f, w = susp.cell_arrays(int(c))
        o = S.operators_for(mc)
        prm = S.Params(tuple(w), mc.mass, susp.dt if dt is None else dt,
                       tuple(getattr(mc, "damping", (0.0, 0.0))))
        cs = S.CellSolver(o, prm)
        out[int(c)] = cs.rollout(x0, v0, f, susp.n_iter if n_iter is None else n_iter,
                                 susp.n_steps if n_steps is None else n_steps)
    return out


def cell_error(susp, x_gpu, cell, x_ref):
    """Relative position error of one cell (max |dx| / cell radius)."""
    s = susp.cell_slice(int(cell))
    return S.rel_position_error(x_gpu[:, s].T, x_ref)


def max_error(susp, x_gpu, ref):
    return max(cell_error(susp, x_gpu, c, xr) for c, (xr, _) in ref.items())


def reverse_along(args):
    """Worker (spawned process): the oracle's FP64 reverse-mode gradient of
    one cell along the trajectory another solver went through
    (susp, cell, target, step-start states, final positions[, the PD
    iterates of every step])."""
    import os
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import torch
    torch.set_num_threads(1)
    from oracle import reverse as R
    susp, c, tgt, states, x_final = args[:5]
    iterates = args[5] if len(args) > 5 else None
    mc, x0, v0, f, w = susp.cell_arrays(int(c))
    o = S.operators_for(mc)
    _, gw, gf, _, _ = R.rollout_grad(o, w, mc.mass, susp.dt, x0, v0, f, tgt, susp.n_iter,
                                     susp.n_steps, states=states, x_final=x_final,
                                     iterates=iterates)
    return int(c), gw, gf
