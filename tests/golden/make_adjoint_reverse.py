"""Writes adjoint_reverse_rbc1024.json: the FP64 reverse-mode gradient of the
oracle (oracle/reverse.py) for the differentiation workload (1024 RBCs of 642
vertices, 50 steps x 10 PD iterations, dt 1e-4, loss = sum |x_T - target|^2
with the rest shape stretched 15 % along x as target), on the same 8 seeded
cells and FP32-rounded inputs as adjoint_fd_rbc1024.json.

Per cell: the loss, dL/dw (stretch, area, bend, volume), dL/df at the force
components of the finite-difference file ("df_at") and at 64 further seeded
components ("df_sample_comps" / "df_sample"), and dL/dx0 at the same 64.
"dw_fp32_state" / "df_sample_fp32_state": the same gradients along the
trajectory whose positions and velocities are rounded to FP32 after every
step (the FP64 step and its exact gradient otherwise): how far the rounding
of an FP32 state alone moves the gradients.

Only the oracle computes these values. Usage:
    python tests/golden/make_adjoint_reverse.py [--procs 8]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

OUT = os.path.join(HERE, "adjoint_reverse_rbc1024.json")
FD = os.path.join(HERE, "adjoint_fd_rbc1024.json")
N_CELLS, N_STEPS, N_ITER = 1024, 50, 10


def workload():
    from npfem_workload import suspensions as W
    from npfem_workload.suspensions import Suspension
    s = W.adjoint_rbcs(n_cells=N_CELLS, n_steps=N_STEPS, n_iter=N_ITER)
    r = lambda a: a.astype(np.float32).astype(np.float64)
    return Suspension(s.classes, s.cell_class, s.origins, r(s.x0), r(s.v0), r(s.forces),
                      s.weights, s.dt, s.n_iter, s.n_steps, s.name, dict(s.extra))


def one_cell(c):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import torch
    torch.set_num_threads(1)
    from oracle import reverse as R
    s = workload()
    tgt = s.extra["target"][:, s.cell_slice(c)].T
    L, gw, gf, gx, _ = R.cell_rollout_grad(s, c, tgt)
    _, gw32, gf32, _, _ = R.cell_rollout_grad(s, c, tgt, round_state=torch.float32)
    with open(FD) as fh:
        fd = {r["cell"]: r for r in json.load(fh)["cells"]}
    at = {f"{v},{d}": float(gf[v, d]) for v, d in fd[c]["force_comps"]} if c in fd else {}
    n = gf.shape[0]
    rng = np.random.default_rng(2000 + c)
    comps = [(int(rng.integers(n)), int(rng.integers(3))) for _ in range(64)]
    return {"cell": int(c), "loss": L, "dw": gw.tolist(), "df_at": at,
            "df_sample_comps": comps, "df_sample": [float(gf[v, d]) for v, d in comps],
            "dx0_sample": [float(gx[v, d]) for v, d in comps],
            "dw_fp32_state": gw32.tolist(),
            "df_sample_fp32_state": [float(gf32[v, d]) for v, d in comps]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    a = ap.parse_args()
    with open(FD) as fh:
        cells = [r["cell"] for r in json.load(fh)["cells"]]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(a.procs) as pool:
        rows = pool.map(one_cell, cells)
    s = workload()
    doc = {"workload": f"adjoint_rbcs(n_cells={N_CELLS}, n_steps={N_STEPS}, n_iter={N_ITER}), "
                       "state/forces rounded to FP32",
           "dt": s.dt, "loss": "sum |x_T - target|^2", "method": "FP64 reverse mode (oracle/reverse.py)",
           "cells": rows}
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(OUT)


if __name__ == "__main__":
    main()
