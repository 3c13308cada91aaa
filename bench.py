"""Throughput of the batched projective-dynamics step on one MI355X.

One "step" is one implicit time step of every cell: predict, n_iter x (local
step + global GEMM), update. Default workload: 4096 RBCs (642 vertices each,
Evans-Fung shape, random rotations on a 10 um lattice, shear + noise forces),
FP32, 10 PD iterations per step, dt = 1e-4.

Prints ONE JSON line: cell-PD-iterations per second over K timed steps
(inputs resident in HBM, hipGraph replays), the roofline position of the
dominant kernel (per-kernel HIP events in a second, eagerly launched pass over
the same steps), the FP64 oracle timed on host cores on a bounded sample of
cells, and the relative position error of those cells against the oracle.
Beside it: the same workload with the global step in FP16 MFMA plus
correction sweeps (throughput, speedup, error against the same oracle
cells), and the forward + backward time of the differentiation workload
(1024 RBCs, 50 steps x 10 iterations, checkpoints every 10 steps).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rbc_lattice]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "cell-PD-iterations/sec at ≤1e-6 rel err vs FP64; fwd+bwd time; roofline %"
PEAK = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "fp32_matrix_TF": 157.3,
    "fp64_matrix_TF": 78.6,
    "bf16_matrix_TF": 2500.0,
    "fp16_matrix_TF": 2500.0,
    "fp32_vector_TF": 157.3,
}
DTYPE = {"fp32": "f32", "fp64": "f64", "bf16": "bf16+f32", "fp16": "f16+f32"}


def build_workload(name, cells):
    from npfem_workload import suspensions as W
    if name == "rbc_lattice":
        s = W.rbc_lattice(n_cells=cells or 4096)
        desc = f"{s.n_cells} RBC x 642 vertices (Evans-Fung, icosphere L3), 10 um lattice, shear+noise forces"
    elif name == "uneven":
        s = W.uneven()
        desc = "3000 RBC (642 v) + 600 platelets (162 v) + 64 large cells (2562 v), weights +-20%"
    elif name == "precision":
        s = W.precision_sweep()
        desc = "16384 RBC (642 v) + 1638 platelets (162 v)"
    elif name == "single_rbc":
        s = W.single_rbc()
        desc = "1 RBC x 162 vertices"
    else:
        raise SystemExit(f"unknown workload {name}")
    return s, desc


def round_inputs(s, precision):
    from npfem_workload.suspensions import Suspension
    if precision == "fp64":
        return s
    r = lambda a: a.astype(np.float32).astype(np.float64)
    return Suspension(s.classes, s.cell_class, s.origins, r(s.x0), r(s.v0), r(s.forces),
                      (s.weights if s.uniform_weights() else r(s.weights)), s.dt, s.n_iter, s.n_steps, s.name, dict(s.extra))


def _oracle_cell(args):
    """Worker: roll one cell out with the oracle, single-threaded BLAS."""
    susp, c, n_steps = args
    from oracle import solver as S
    t0 = time.perf_counter()
    x, v = S.run_cell(susp, c, n_steps=n_steps)
    return c, x, time.perf_counter() - t0


def cpu_baseline(susp, cells, n_steps):
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(len(cells), initializer=_pin_threads) as pool:
        res = pool.map(_oracle_cell, [(susp, int(c), n_steps) for c in cells])
    wall = time.perf_counter() - t0
    return {c: x for c, x, _ in res}, wall, sum(t for _, _, t in res)


def _pin_threads():
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def class_counts(s):
    for k, mc in enumerate(s.classes):
        n_c = int((s.cell_class == k).sum())
        F = int(mc.tris.shape[0])
        yield n_c, mc.n_verts, F, 3 * F // 2


def gemm_flops(s):
    """Algorithmic FLOPs of one global-step launch: dense 2 N^2 per column,
    3 columns per cell, N the real (unpadded) vertex count."""
    return sum(2.0 * N * N * 3 * n_c for n_c, N, F, E in class_counts(s))


# Algorithmic FLOPs of the local step per element (FMA = 2, add/mul/sqrt/rcp = 1),
# counted from the operations it performs: strain + area projection and
# contribution per triangle, bending per hinge (both against q only: the
# kernel forms the increment right-hand side), one volume pass per vertex
# (36 per triangle for the corner cross products, 33 per vertex), the two
# gathers (12 per triangle corner, 24 per hinge) and the per-vertex inertia
# term and final sum (9 per vertex).
TRI_FLOPS, HINGE_FLOPS = 221, 35
VOL_TRI_FLOPS, VOL_VERT_FLOPS = 36, 33
VOLUME_PASSES = 1  # the minimum: the settling test can stop after the first pass


def local_flops(s):
    total = 0.0
    for n_c, N, F, E in class_counts(s):
        per_cell = (TRI_FLOPS * F + HINGE_FLOPS * E
                    + VOLUME_PASSES * (VOL_TRI_FLOPS * F + VOL_VERT_FLOPS * N) + 6 * N
                    + 12 * 3 * F + 24 * E + 9 * N)
        total += n_c * per_cell
    return total


def local_bytes(s, elem=4):
    """Algorithmic HBM bytes of one local-step launch: read x, delta and the
    inertia term (3 N each), write the right-hand side (3 Npad)."""
    return sum(n_c * elem * (9 * N + 3 * ((N + 15) // 16 * 16)) for n_c, N, F, E in class_counts(s))


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2011_04332_amd", "csrc")
    for name in ("kernels_local.hip", "local_common.h", "projections.h", "kernels_gemm.hip",
                 "device_utils.h", "npfem_internal.h"):
        with open(os.path.join(root, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, if it was taken on the current kernel sources (else None)."""
    import re
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        f"{workload}_{precision}_traffic.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\s*(\{.*?\})\s*```", open(path).read(), re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    return d if d.get("kernel_source_sha256_16") == kernel_source_digest() else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rbc_lattice")
    ap.add_argument("--cells", type=int, default=0)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16", "fp16"])
    ap.add_argument("--n-iter", type=int, default=10)
    ap.add_argument("--cpu-cells", type=int, default=8)
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--pin-config", default="",
                    help="local block,tile m,tile n,sweeps for every class (skips the autotuner); "
                         "profiling runs use it to launch exactly the configuration the timed run chose")
    ap.add_argument("--compare-precision", default="fp16", choices=["none", "bf16", "fp16"],
                    help="also time the workload with this 16-bit global step (FP32 runs only)")
    ap.add_argument("--mixed-sweeps", type=int, default=-1,
                    help="correction sweeps of the 16-bit comparison run (-1: the library's "
                         "automatic count)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the forward + backward timing of the differentiation workload")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (3 times), the "
                         "reference for scaling FETCH_SIZE / WRITE_SIZE counters")
    a = ap.parse_args()
    if a.calibrate_copy_mb:
        import torch
        n = a.calibrate_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4, "copies": 3}), flush=True)
        return
    if a.gpus != 1:
        print("bench.py: this build measures one GPU only (the per-cell step needs no "
              "exchange between GPUs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2011_04332_amd import solver
    from npfem_workload import suspensions as W

    s, desc = build_workload(a.workload, a.cells)
    s = round_inputs(s, a.precision)
    dt, n_iter = s.dt, a.n_iter
    print(f"[bench] workload {a.workload}: {desc}; {a.precision}; steps {a.steps} warmup {a.warmup}",
          file=sys.stderr, flush=True)

    pinned = [int(v) for v in a.pin_config.split(",")] if a.pin_config else None
    b, pos, vel, f, meshes = solver.batch_from_suspension(
        s, precision=a.precision, autotune=not (a.no_autotune or pinned))
    if pinned:
        for k in range(len(s.classes)):
            b.set_config(k, pinned)
    x_init, v_init = pos.clone(), vel.clone()
    for _ in range(max(1, a.warmup)):
        b.step(f, dt, n_iter)
    b.sync_status()
    launch_cfgs = [b.config(k) for k in range(len(s.classes))]
    print(f"[bench] launch configs per class (local block, tile m, tile n, sweeps): {launch_cfgs}",
          file=sys.stderr, flush=True)
    pos.copy_(x_init)
    vel.copy_(v_init)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        b.step(f, dt, n_iter)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    b.sync_status()
    elapsed = t1 - t0
    cell_its = s.n_cells * n_iter * a.steps
    value = cell_its / elapsed
    x_timed = pos.clone()
    print(f"[bench] timed: {elapsed * 1e3:.1f} ms, {value:.4g} cell-it/s", file=sys.stderr, flush=True)

    # second pass over the same steps, launched one by one with HIP events
    roof, kt, snap = None, None, None
    cpu_steps = min(a.cpu_steps, a.steps)
    if not a.no_kernel_timing:
        pos.copy_(x_init)
        vel.copy_(v_init)
        bt = solver.Batch(meshes, s.cell_class, pos, vel,
                          cell_weights=None if s.uniform_weights() else s.weights,
                          precision=a.precision, kernel_timing=True)
        for k, cfg in enumerate(launch_cfgs):
            # pins the launch shapes; the sweep count stays automatic (with
            # 16-bit products, sweeps a cell does not need are skipped)
            bt.set_config(k, (cfg[0], cfg[1], cfg[2], -1))
        for i in range(a.steps):
            bt.step(f, dt, n_iter)
            if i + 1 == cpu_steps:
                snap = pos.double().cpu().numpy()
        kt = bt.kernel_times()
        bt.sync_status()
        bitwise = bool(torch.equal(pos, x_timed))
        bt.close()
        traffic = measured_traffic(a.workload, a.precision)
        entries = {}
        sweeps = launch_cfgs[0][3]
        for kind in ("local", "global"):
            ms, n = kt[kind]
            avg_s = ms / n * 1e-3
            # algorithmic work of all launches of this kind in the timing pass,
            # spread evenly over the launches (classes differ in size)
            if kind == "local":
                total = local_flops(s) * n_iter * a.steps
                peak = PEAK["fp64_matrix_TF"] if a.precision == "fp64" else PEAK["fp32_vector_TF"]
                e = {"bound": "alu", "kernel": "local_kernel (projections + RHS gather)",
                     "algorithmic_flops": total / n,
                     "algorithmic_hbm_bytes": local_bytes(s, 8 if a.precision == "fp64" else 4)
                     * n_iter * a.steps / n,
                     "alu_peak_without_packed_fp32": 78.6}
            else:
                total = gemm_flops(s) * (1 + sweeps) * n_iter * a.steps
                peak = PEAK[f"{a.precision}_matrix_TF"]
                e = {"bound": "mfma", "kernel": "gemm_kernel (global step)",
                     "algorithmic_flops": total / n}
            achieved = total / (ms * 1e-3) / 1e12
            e.update({"achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                      "frac": round(achieved / peak, 4), "avg_launch_us": round(avg_s * 1e6, 2),
                      "launches": n,
                      "traffic": (traffic or {}).get(kind)})
            entries[kind] = e
        dom = max(("local", "global"), key=lambda k: kt[k][0])
        roof = dict(entries[dom])
        roof.update({
            "dominant_kernel": dom,
            "other_kernel": entries["global" if dom == "local" else "local"],
            "kernel_ms_per_step": {k: round(v[0] / a.steps, 4) for k, v in kt.items()},
            "timing_pass_bitwise_equal": bitwise,
        })
        print(f"[bench] kernel times (ms/step): {roof['kernel_ms_per_step']}", file=sys.stderr,
              flush=True)

    # the same workload with a 16-bit global step plus correction sweeps
    mixed, snap_m = None, None
    if a.precision == "fp32" and a.compare_precision != "none":
        pos.copy_(x_init)
        vel.copy_(v_init)
        bm = solver.Batch(meshes, s.cell_class, pos, vel,
                          cell_weights=None if s.uniform_weights() else s.weights,
                          precision=a.compare_precision, autotune=not a.no_autotune,
                          n_refine=a.mixed_sweeps)
        for _ in range(cpu_steps):
            bm.step(f, dt, n_iter)
        bm.sync_status()
        snap_m = pos.double().cpu().numpy()
        cfg_m = [bm.config(k) for k in range(len(s.classes))]
        pos.copy_(x_init)
        vel.copy_(v_init)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            bm.step(f, dt, n_iter)
        torch.cuda.synchronize()
        el_m = time.perf_counter() - t0
        bm.sync_status()
        bm.close()
        mixed = {"precision": a.compare_precision, "dtype": DTYPE[a.compare_precision],
                 "value": round(cell_its / el_m, 1), "ms_per_step": round(el_m / a.steps * 1e3, 4),
                 "speedup_vs_fp32": round(elapsed / el_m, 4),
                 "sweeps": cfg_m[0][3], "gemm_tiles": [[c[1], c[2]] for c in cfg_m]}
        print(f"[bench] {a.compare_precision}: {mixed}", file=sys.stderr, flush=True)

    # forward + backward of the differentiation workload
    fwd_bwd = None
    if not a.no_adjoint and a.precision in ("fp32", "fp64"):
        sa = round_inputs(W.adjoint_rbcs(), a.precision)
        ba, pa, va, fa, _ = solver.batch_from_suspension(sa, precision=a.precision)
        tgt = torch.tensor(sa.extra["target"], dtype=pa.dtype, device=pa.device)
        x0a, v0a = pa.clone(), va.clone()
        n_st, n_it, every = sa.n_steps, sa.n_iter, sa.extra["ckpt_every"]

        def fwd_bwd_once():
            pa.copy_(x0a)
            va.copy_(v0a)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ba.rollout(fa, sa.dt, n_it, n_st, every)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ba.rollout_adjoint((2.0 * (pa - tgt)).contiguous())
            torch.cuda.synchronize()
            return t1 - t0, time.perf_counter() - t1

        fwd_bwd_once()  # graphs, checkpoint and tape buffers
        tf, tb = fwd_bwd_once()
        ba.sync_status()
        ba.close()
        fwd_bwd = {"workload": f"{sa.n_cells} RBC x 642 vertices, {n_st} steps x {n_it} PD "
                               f"iterations, checkpoints every {every} steps, "
                               "loss sum |x_T - target|^2",
                   "forward_ms": round(tf * 1e3, 3), "backward_ms": round(tb * 1e3, 3),
                   "fwd_bwd_ms": round((tf + tb) * 1e3, 3),
                   "backward_over_forward": round(tb / tf, 3)}
        print(f"[bench] forward+backward: {fwd_bwd}", file=sys.stderr, flush=True)

    cpu, parity = None, None
    if not a.no_cpu_baseline and snap is not None:
        ncores = min(a.cpu_cells, os.cpu_count() or 1, 16)
        cells = W.sample_cells(s, [ncores])[:ncores]
        ref, wall, cpu_s = cpu_baseline(s, cells, cpu_steps)
        ci = len(cells) * cpu_steps * n_iter
        cpu = {"value": round(ci / wall, 3), "unit": "cell-PD-iterations/s", "cores": int(ncores),
               "kind": "oracle",
               "sample": f"{len(cells)} sampled cells x {cpu_steps} steps x {n_iter} PD iterations, "
                         f"one process per cell, FP64 numpy/scipy, wall {wall:.1f} s"}
        from oracle import solver as S
        errs = [S.rel_position_error(snap[:, s.cell_slice(c)].T, x) for c, x in ref.items()]
        parity = {"max_rel_pos_err": float(max(errs)), "cells": [int(c) for c in cells],
                  "steps": cpu_steps, "bound": 1e-6 if a.precision == "fp32" else 1e-5}
        if mixed is not None and snap_m is not None:
            mixed["max_rel_pos_err"] = float(max(
                S.rel_position_error(snap_m[:, s.cell_slice(c)].T, x) for c, x in ref.items()))
        print(f"[bench] oracle: {cpu['value']} cell-it/s on {ncores} cores; parity {parity}",
              file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "cell-PD-iterations/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[a.precision],
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {desc}", "cells": s.n_cells, "pd_iterations": n_iter,
                   "launch": {s.classes[k].name: {"local_block": c[0], "gemm_tile": [c[1], c[2]],
                                                  "sweeps": c[3]} for k, c in enumerate(launch_cfgs)},
                   "dt": dt, "precision": a.precision},
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
        "mixed_precision": mixed,
        "fwd_bwd": fwd_bwd,
    }
    print(json.dumps(out), flush=True)
    b.close()


if __name__ == "__main__":
    main()
