"""Writes adjoint_fd_rbc1024.json: central finite differences of the FP64
oracle for the differentiation workload (1024 RBCs of 642 vertices, 50 steps
x 10 PD iterations, dt 1e-4, loss = sum |x_T - target|^2 with the rest shape
stretched 15 % along x as target), on 8 seeded sample cells.

Inputs are the workload's seeded state, forces and weights rounded to FP32
(what an FP32 run receives; an FP64 run is given the same values).
Weight gradients: central difference quotients D(h) at relative steps h =
0.05, 0.1, 0.15 and 0.2 of each weight, fitted by least squares with
D(h) = g + c h^2 (the truncation error of a central difference is even in
h); the value is g, and the fit's largest residual serves as the uncertainty
of the differences themselves. The FP64 rollout of 500 iterations carries
rounding noise of ~1e-9 on L ~ 1e3 that does not vary smoothly with the
weights; at a relative step of 1e-3 it would swamp the bending gradient
(step 2e-5), hence the large steps.
Force gradients: central differences with h = 1e-3 on 3 seeded components.

Only the oracle computes these values. Usage:
    python tests/golden/make_adjoint_fd.py [--procs 8]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

OUT = os.path.join(HERE, "adjoint_fd_rbc1024.json")
N_CELLS, N_STEPS, N_ITER = 1024, 50, 10
STEPS = (0.05, 0.1, 0.15, 0.2)


def workload():
    from npfem_workload import suspensions as W
    from npfem_workload.suspensions import Suspension
    s = W.adjoint_rbcs(n_cells=N_CELLS, n_steps=N_STEPS, n_iter=N_ITER)
    r = lambda a: a.astype(np.float32).astype(np.float64)
    return Suspension(s.classes, s.cell_class, s.origins, r(s.x0), r(s.v0), r(s.forces),
                      s.weights, s.dt, s.n_iter, s.n_steps, s.name, dict(s.extra))


def one_cell(c):
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import gradients as Gr
    s = workload()
    mc, x0, v0, f, w = s.cell_arrays(c)
    tgt = s.extra["target"][:, s.cell_slice(c)].T
    args = (mc, w, mc.mass, s.dt, x0, v0, f, tgt, N_ITER, N_STEPS)
    steps = np.array(STEPS)
    D = np.array([Gr.fd_weight_grad(*args, h=float(h)) for h in steps])  # [len(steps), 4]
    X = np.stack([np.ones_like(steps), steps ** 2], axis=1)
    coef, *_ = np.linalg.lstsq(X, D, rcond=None)
    resid = np.abs(D - X @ coef).max(axis=0)
    rng = np.random.default_rng(1000 + c)
    comps = [(int(rng.integers(mc.n_verts)), int(rng.integers(3))) for _ in range(3)]
    gf = Gr.fd_force_grad(*args, comps, h=1e-3)
    return {"cell": int(c), "dw": coef[0].tolist(), "dw_fit_resid": resid.tolist(),
            "dw_quotients": {f"{h:g}": D[i].tolist() for i, h in enumerate(steps)},
            "force_comps": comps, "df": gf.tolist()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    a = ap.parse_args()
    from npfem_workload import suspensions as W
    s = workload()
    cells = [int(c) for c in W.sample_cells(s, [8])]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(a.procs) as pool:
        rows = pool.map(one_cell, cells)
    doc = {"workload": f"adjoint_rbcs(n_cells={N_CELLS}, n_steps={N_STEPS}, n_iter={N_ITER}), "
                       "state/forces rounded to FP32",
           "dt": s.dt, "loss": "sum |x_T - target|^2", "cells": rows}
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(OUT)


if __name__ == "__main__":
    main()
