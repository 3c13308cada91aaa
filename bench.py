"""Throughput of the batched projective-dynamics step on one MI355X.

One "step" is one implicit time step of every cell: predict, n_iter x (local
step + global GEMM [+ correction sweeps]), update. Default workload: the
precision-sweep suspension, 16384 RBCs (642 vertices, Evans-Fung shape) +
1638 platelets (162 vertices, oblate ellipsoid) on a 10 um lattice with random
rotations, forces N(0, 0.05^2), FP32, 10 PD iterations per step, dt = 1e-4.

Prints ONE JSON line:
* value: cell-PD-iterations per second over K timed steps (inputs resident in
  HBM, hipGraph replays);
* roofline: the dominant kernel's algorithmic work per launch over its average
  duration (per-kernel HIP events in a second, eagerly launched pass over the
  same steps), the other kernels' fractions (local step against the FP32
  VALU peak without packed FP32, 78.6 TFLOP/s; predict and update against
  HBM), and the whole step's ideal time
  sum_k max(flops_k / peak, bytes_k / HBM) over the measured step time;
* cpu_baseline: the FP64 oracle on the host cores on a bounded sample of
  cells (one process per cell on all cores used, and one cell alone on one
  core), with the CPU model;
* parity: the sampled cells' relative position error against the oracle
  after the first cpu-steps steps, and the volume drift |V - V_rest| / V_rest
  of GPU and oracle;
* precision_sweep: the same workload with the global step in BF16 and in
  FP16 MFMA (FP32 accumulation) with 2 correction sweeps each, with the
  automatic sweep count, and in FP64; throughput and error against the same
  oracle cells for each;
* uneven: the uneven batch (3000 RBC + 600 platelets + 64 large cells,
  per-cell weights +-20 %) in FP32 and with the FP16 global step, the speedup
  of the latter and both errors against the oracle;
* single_rbc_fp64: one RBC (162 vertices) in FP64, 100 steps x 20 iterations,
  against the oracle's full run;
* fwd_bwd: forward + backward time of the differentiation workload (1024
  RBCs, 50 steps x 10 iterations, checkpoints every 10 steps);
* next_rows: the further forms on the 4096-RBC lattice, each with its oracle
  error: viscous damping, wall contacts, the quasi-Newton step against PD at
  equal iteration counts on the stiff twin (error against the converged
  step), and the immersed-boundary interpolation and spreading on a periodic
  160^3 grid.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload precision_sweep]
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
    "fp64_vector_TF": 78.6,
}
# FP32 VALU peak this build can reach: 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# (FMA) x 2.4 GHz. The published 157.3 counts packed FP32 (two lanes per
# instruction), which this build does not emit (every kernel is compiled
# without packed-FP32 instructions).
ALU_FP32_UNPACKED_TF = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
DTYPE = {"fp32": "f32", "fp64": "f64", "bf16": "bf16+f32", "fp16": "f16+f32"}
BOUND = {"fp64": 1e-12, "fp32": 1e-6, "bf16": 1e-5, "fp16": 1e-5}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_workload(name, cells):
    from npfem_workload import suspensions as W
    if name == "rbc_lattice":
        s = W.rbc_lattice(n_cells=cells or 4096)
        desc = f"{s.n_cells} RBC x 642 vertices (Evans-Fung, icosphere L3), 10 um lattice, shear+noise forces"
    elif name == "uneven":
        s = W.uneven()
        desc = "3000 RBC (642 v) + 600 platelets (162 v) + 64 large cells (2562 v), weights +-20%"
    elif name in ("precision_sweep", "precision"):
        s = W.precision_sweep()
        desc = ("16384 RBC (642 v) + 1638 platelets (162 v), 10 um lattice, random rotations, "
                "forces N(0, 0.05^2)")
    elif name == "single_rbc":
        s = W.single_rbc()
        desc = "1 RBC x 162 vertices"
    else:
        raise SystemExit(f"unknown workload {name}")
    return s, desc


def round_inputs(s, precision="fp32"):
    """State and forces rounded to FP32 (what an FP32 run receives); FP64 runs
    are given the same values, so one oracle reference serves every precision."""
    from npfem_workload.suspensions import Suspension
    if precision == "fp64":
        return s
    r = lambda a: a.astype(np.float32).astype(np.float64)
    return Suspension(s.classes, s.cell_class, s.origins, r(s.x0), r(s.v0), r(s.forces),
                      (s.weights if s.uniform_weights() else r(s.weights)), s.dt, s.n_iter,
                      s.n_steps, s.name, dict(s.extra))


# ---------------------------------------------------------------- oracle leg

def _oracle_cell(args):
    """Worker: roll one cell out with the oracle, single-threaded BLAS."""
    susp, c, n_steps, n_iter = args
    _pin_threads()
    from oracle import operators as ops_mod
    from oracle import solver as S
    t0 = time.perf_counter()
    x, v = S.run_cell(susp, c, n_steps=n_steps, n_iter=n_iter)
    el = time.perf_counter() - t0
    mc = susp.classes[int(susp.cell_class[c])]
    o = S.operators_for(mc)
    return c, x, el, ops_mod.volume(x, o.tris), o.vol_rest


def _pin_threads():
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def oracle_cells(susp, cells, n_steps, n_iter, procs):
    """{cell: (x, oracle volume, rest volume)}, wall time, summed cell times."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(procs, initializer=_pin_threads) as pool:
        res = pool.map(_oracle_cell, [(susp, int(c), n_steps, n_iter) for c in cells])
    wall = time.perf_counter() - t0
    return {c: (x, vol, vr) for c, x, _, vol, vr in res}, wall, sum(t for _, _, t, _, _ in res)


def oracle_single_core(susp, c, n_steps, n_iter):
    """One cell alone in one process on one core: (cell-iterations/s, seconds)."""
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(1, initializer=_pin_threads) as pool:
        _, _, el, _, _ = pool.apply(_oracle_cell, ((susp, int(c), n_steps, n_iter),))
    return n_steps * n_iter / el, el


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def errors_vs_oracle(susp, x_gpu, vol_gpu, ref):
    """Max relative position error (max_v |dx| / R_cell) over the cells of
    ref, and the volume drifts |V - V_rest| / V_rest of GPU and oracle."""
    from oracle import solver as S
    pos, dg, do, dgo = [], [], [], []
    for c, (x, vo, vr) in ref.items():
        pos.append(S.rel_position_error(x_gpu[:, susp.cell_slice(c)].T, x))
        dg.append(abs(vol_gpu[c] - vr) / vr)
        do.append(abs(vo - vr) / vr)
        dgo.append(abs(vol_gpu[c] - vo) / vr)
    return {"max_rel_pos_err": float(max(pos)), "volume_drift_gpu": float(max(dg)),
            "volume_drift_oracle": float(max(do)), "volume_gpu_vs_oracle": float(max(dgo))}


# ------------------------------------------------------------- work counts

def class_counts(s):
    for k, mc in enumerate(s.classes):
        n_c = int((s.cell_class == k).sum())
        F = int(mc.tris.shape[0])
        yield n_c, mc.n_verts, F, 3 * F // 2


def npad(N):
    return (N + 15) // 16 * 16


def gemm_flops(s):
    """Algorithmic FLOPs of one global-step product: dense 2 N^2 per column,
    3 columns per cell, N the real (unpadded) vertex count."""
    return sum(2.0 * N * N * 3 * n_c for n_c, N, F, E in class_counts(s))


def gemm_bytes(s, elem=4, op_elem=4):
    """Algorithmic HBM bytes of one product: the right-hand side and the
    previous iterate read, the next iterate written (3 Npad per cell each),
    plus each class operator once."""
    return sum(n_c * elem * 9 * npad(N) + op_elem * npad(N) ** 2 for n_c, N, F, E in class_counts(s))


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
    return sum(n_c * elem * (9 * N + 3 * npad(N)) for n_c, N, F, E in class_counts(s))


def predict_bytes(s, elem=4):
    """Read x, v, f (3 N each), write the inertia term and the first increment (3 Npad each)."""
    return sum(n_c * elem * (9 * N + 6 * npad(N)) for n_c, N, F, E in class_counts(s))


def update_bytes(s, elem=4):
    """Read x and the increment, write x and v."""
    return sum(n_c * elem * (9 * N + 3 * npad(N)) for n_c, N, F, E in class_counts(s))


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2011_04332_amd", "csrc")
    for name in ("kernels_local.hip", "local_common.h", "projections.h", "kernels_gemm.hip",
                 "kernels_state.hip", "device_utils.h", "npfem_internal.h"):
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


# -------------------------------------------------------------- GPU runs

def make_batch(s, precision, **kw):
    from paper_2011_04332_amd import solver
    return solver.batch_from_suspension(s, precision=precision, **kw)


def timed_steps(b, f, dt, n_iter, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.step(f, dt, n_iter)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    b.sync_status()
    return el


def run_form(s, precision, n_iter, snap_steps, time_steps, warmup, n_refine=-1, autotune=True,
             qn=None):
    """One precision form of a workload: snapshot (positions, volumes) after
    snap_steps steps from the initial state, then time_steps timed steps from
    the initial state again. Returns a dict with the snapshot and timings.
    qn: (history, line-search rounds) for the quasi-Newton step."""
    import torch
    b, pos, vel, f, meshes = make_batch(s, precision, n_refine=n_refine, autotune=autotune)
    if qn is not None:
        b.set_quasi_newton(*qn)
    x0, v0 = pos.clone(), vel.clone()
    for _ in range(max(1, warmup)):
        b.step(f, s.dt, n_iter)
    b.sync_status()
    cfgs = [b.config(k) for k in range(len(s.classes))]
    pos.copy_(x0)
    vel.copy_(v0)
    for _ in range(snap_steps):
        b.step(f, s.dt, n_iter)
    b.sync_status()
    snap = pos.double().cpu().numpy()
    vols = b.volume()
    pos.copy_(x0)
    vel.copy_(v0)
    el = timed_steps(b, f, s.dt, n_iter, time_steps)
    b.close()
    del pos, vel, f
    torch.cuda.empty_cache()
    return {"snap": snap, "vols": vols, "elapsed": el, "steps": time_steps, "configs": cfgs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="precision_sweep")
    ap.add_argument("--cells", type=int, default=0)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16", "fp16"])
    ap.add_argument("--n-iter", type=int, default=10)
    ap.add_argument("--cpu-cells", default="16,4,2",
                    help="oracle sample: cells per mesh class (the parity and CPU-baseline cells)")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--cpu-procs", type=int, default=16, help="cap on oracle worker processes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--pin-config", default="",
                    help="local block,tile m,tile n,sweeps, one group per class separated by ';' "
                         "(a single group applies to every class; skips the autotuner); profiling "
                         "runs use it to launch exactly the configuration the timed run chose")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the BF16 / FP16 / FP64 forms of the workload")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the uneven batch, the single-RBC FP64 run and the forward + backward timing")
    ap.add_argument("--main-only", action="store_true",
                    help="only the timed run and the kernel-timing pass (profiling runs)")
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
    if a.main_only:
        a.no_cpu_baseline = a.no_sweep = a.no_extra = True

    import torch
    from paper_2011_04332_amd import solver
    from npfem_workload import suspensions as W

    wl = "precision_sweep" if a.workload == "precision" else a.workload
    s, desc = build_workload(wl, a.cells)
    s = round_inputs(s, a.precision)
    dt, n_iter = s.dt, a.n_iter
    cpu_steps = min(a.cpu_steps, a.steps)
    log(f"workload {wl}: {desc}; {a.precision}; steps {a.steps} warmup {a.warmup}")

    # ---- main timed run (hipGraph replays)
    pinned = None
    if a.pin_config:
        groups = [[int(v) for v in g.split(",")] for g in a.pin_config.split(";")]
        if len(groups) not in (1, len(s.classes)) or any(len(g) != 4 for g in groups):
            sys.exit(f"bench.py: --pin-config needs 1 or {len(s.classes)} groups of 4 integers")
        pinned = groups * len(s.classes) if len(groups) == 1 else groups
    b, pos, vel, f, meshes = make_batch(s, a.precision, autotune=not (a.no_autotune or pinned))
    if pinned:
        for k in range(len(s.classes)):
            b.set_config(k, pinned[k])
    x_init, v_init = pos.clone(), vel.clone()
    for _ in range(max(1, a.warmup)):
        b.step(f, dt, n_iter)
    b.sync_status()
    launch_cfgs = [b.config(k) for k in range(len(s.classes))]
    log(f"launch configs per class (local block, tile m, tile n, sweeps): {launch_cfgs}")
    pos.copy_(x_init)
    vel.copy_(v_init)
    elapsed = timed_steps(b, f, dt, n_iter, a.steps)
    cell_its = s.n_cells * n_iter * a.steps
    value = cell_its / elapsed
    x_timed = pos.clone()
    log(f"timed: {elapsed * 1e3:.1f} ms, {value:.4g} cell-it/s")

    # ---- second pass over the same steps, launched one by one with HIP events
    roof, kt, snap, vols = None, None, None, None
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
                bt.sync_status()
                snap = pos.double().cpu().numpy()
                vols = bt.volume()
        kt = bt.kernel_times()
        bt.sync_status()
        bitwise = bool(torch.equal(pos, x_timed))
        bt.close()
        roof = roofline(s, a, kt, launch_cfgs, elapsed, bitwise, wl)
        log(f"kernel times (ms/step): {roof['kernel_ms_per_step']}; whole step {roof['whole_step']}")
    b.close()

    # ---- oracle on sampled cells: CPU baseline and parity reference
    cpu, parity, ref = None, None, None
    if not a.no_cpu_baseline and snap is not None:
        per_class = [int(v) for v in a.cpu_cells.split(",")][:len(s.classes)]
        cells = W.sample_cells(s, per_class)
        procs = max(1, min(len(cells), os.cpu_count() or 1, a.cpu_procs))
        ref, wall, cpu_s = oracle_cells(s, cells, cpu_steps, n_iter, procs)
        c0 = int(cells[0])
        one_rate, one_s = oracle_single_core(s, c0, cpu_steps, n_iter)
        ci = len(cells) * cpu_steps * n_iter
        cpu = {"value": round(ci / wall, 3), "unit": "cell-PD-iterations/s", "cores": int(procs),
               "kind": "oracle",
               "sample": f"{len(cells)} sampled cells ({'+'.join(map(str, per_class))} per class) x "
                         f"{cpu_steps} steps x {n_iter} PD iterations, one process per cell on "
                         f"{procs} cores, FP64 numpy/scipy, wall {wall:.1f} s",
               "single_core_value": round(one_rate, 3),
               "single_core_sample": f"cell {c0} ({s.classes[int(s.cell_class[c0])].name}) alone, "
                                     f"{cpu_steps} steps x {n_iter} iterations, {one_s:.1f} s",
               "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}
        parity = errors_vs_oracle(s, snap, vols, ref)
        parity.update({"cells": [int(c) for c in cells], "steps": cpu_steps,
                       "bound": BOUND[a.precision]})
        log(f"oracle: {cpu['value']} cell-it/s on {procs} cores, {one_rate:.1f} on one; parity {parity}")

    # ---- the other precision forms of the same workload
    sweep = None
    if not a.no_sweep and a.precision == "fp32":
        sweep = {}
        forms = [("bf16_2sweeps", "bf16", 2), ("fp16_2sweeps", "fp16", 2),
                 ("fp16_auto", "fp16", -1), ("bf16_auto", "bf16", -1), ("fp64", "fp64", -1)]
        for key, prec, nref in forms:
            steps_t = min(a.steps, 20) if prec == "fp64" else a.steps
            r = run_form(s, prec, n_iter, cpu_steps if ref is not None else 0, steps_t, a.warmup,
                         n_refine=nref, autotune=not a.no_autotune)
            e = {"precision": prec, "dtype": DTYPE[prec], "sweeps": r["configs"][0][3],
                 "value": round(s.n_cells * n_iter * r["steps"] / r["elapsed"], 1),
                 "ms_per_step": round(r["elapsed"] / r["steps"] * 1e3, 4),
                 "speedup_vs_fp32": round((elapsed / a.steps) / (r["elapsed"] / r["steps"]), 4),
                 "gemm_tiles": [[c[1], c[2]] for c in r["configs"]]}
            if ref is not None:
                e.update(errors_vs_oracle(s, r["snap"], r["vols"], ref))
                e["bound"] = BOUND[prec]
            sweep[key] = e
            log(f"{key}: {e}")

    extra = {}
    if not a.no_extra:
        extra = extra_workloads(a)
        extra["next_rows"] = next_rows(a)

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
        "config": {"workload": f"{wl}: {desc}", "cells": s.n_cells,
                   "vertices": int(sum(N * n_c for n_c, N, F, E in class_counts(s))),
                   "pd_iterations": n_iter,
                   "launch": {s.classes[k].name: {"local_block": c[0], "gemm_tile": [c[1], c[2]],
                                                  "sweeps": c[3]} for k, c in enumerate(launch_cfgs)},
                   "dt": dt, "precision": a.precision},
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
        "precision_sweep": sweep,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


def roofline(s, a, kt, launch_cfgs, elapsed, bitwise, wl):
    """Per-kernel fractions from the kernel-timing pass and the whole step's
    ideal time over its measured time."""
    elem = 8 if a.precision == "fp64" else 4
    n_iter, steps = a.n_iter, a.steps
    traffic = measured_traffic(wl, a.precision)
    sweeps = launch_cfgs[0][3]
    vec_peak = PEAK["fp64_vector_TF"] if a.precision == "fp64" else ALU_FP32_UNPACKED_TF
    mat_peak = PEAK[f"{a.precision}_matrix_TF"]
    op_elem = {"fp64": 8, "fp32": 4}.get(a.precision, 2)
    work = {  # (flops, bytes) of all launches of a kind over the timed steps
        "local": (local_flops(s) * n_iter * steps, local_bytes(s, elem) * n_iter * steps),
        "global": (gemm_flops(s) * (1 + sweeps) * n_iter * steps,
                   gemm_bytes(s, elem, op_elem) * (1 + sweeps) * n_iter * steps),
        "predict": (0.0, predict_bytes(s, elem) * steps),
        "update": (0.0, update_bytes(s, elem) * steps),
    }
    entries = {}
    for kind in ("local", "global", "predict", "update"):
        ms, n = kt[kind]
        fl, by = work[kind]
        if n == 0:
            continue
        avg_s = ms / n * 1e-3
        if kind == "local":
            e = {"bound": "alu", "kernel": "local_kernel (projections + RHS gather)",
                 "algorithmic_flops": fl / n, "algorithmic_hbm_bytes": by / n,
                 "peak_derivation": "256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz (FP32 "
                                    "VALU without packed FP32, which this build does not emit)",
                 "published_fp32_vector_peak_packed": PEAK["fp32_vector_TF"]}
            ach, peak, unit = fl / (ms * 1e-3) / 1e12, vec_peak, "TFLOP/s"
            e["hbm_GBs"] = round(by / (ms * 1e-3) / 1e9, 1)
        elif kind == "global":
            e = {"bound": "mfma", "kernel": "gemm_kernel (global step)",
                 "algorithmic_flops": fl / n, "algorithmic_hbm_bytes": by / n}
            ach, peak, unit = fl / (ms * 1e-3) / 1e12, mat_peak, "TFLOP/s"
            e["hbm_GBs"] = round(by / (ms * 1e-3) / 1e9, 1)
        else:
            e = {"bound": "hbm", "kernel": f"{kind}_kernel", "algorithmic_hbm_bytes": by / n}
            ach, peak, unit = by / (ms * 1e-3) / 1e9, PEAK["hbm_GBs"], "GB/s"
        e.update({"achieved": round(ach, 3), "peak": peak, "unit": unit,
                  "frac": round(ach / peak, 4), "avg_launch_us": round(avg_s * 1e6, 2),
                  "launches": n, "traffic": (traffic or {}).get(kind)})
        entries[kind] = e
    dom = max(("local", "global"), key=lambda k: kt[k][0])
    roof = dict(entries[dom])
    # ideal step time: every kernel at its binding roof (flops at the published
    # peak of its unit, bytes at HBM bandwidth), summed
    t_ideal = 0.0
    for kind, (fl, by) in work.items():
        pk = vec_peak if kind == "local" else mat_peak
        t_ideal += max(fl / (pk * 1e12), by / (PEAK["hbm_GBs"] * 1e9))
    t_ideal /= steps
    t_meas = elapsed / steps
    fl_loc, _ = work["local"]
    t_ideal_pk = t_ideal - fl_loc / steps / (vec_peak * 1e12) + fl_loc / steps / (PEAK["fp32_vector_TF"] * 1e12)
    roof.update({
        "dominant_kernel": dom,
        "other_kernels": {k: v for k, v in entries.items() if k != dom},
        "kernel_ms_per_step": {k: round(v[0] / steps, 4) for k, v in kt.items()},
        "whole_step": {"t_ideal_ms": round(t_ideal * 1e3, 4), "t_measured_ms": round(t_meas * 1e3, 4),
                       "frac": round(t_ideal / t_meas, 4),
                       "frac_local_at_packed_157.3TF": round(t_ideal_pk / t_meas, 4)},
        "timing_pass_bitwise_equal": bitwise,
    })
    return roof


def extra_workloads(a):
    """Uneven batch (FP32 and FP16 global step), single RBC in FP64, forward +
    backward of the differentiation workload; each with its oracle error."""
    import torch
    from npfem_workload import suspensions as W
    from paper_2011_04332_amd import solver
    out = {}
    procs = max(1, min(os.cpu_count() or 1, a.cpu_procs))

    # uneven batch: 3000 RBC + 600 PLT + 64 large, per-cell weights
    su = round_inputs(W.uneven())
    snap_steps = 10
    cells = W.sample_cells(su, [2, 2, 2])
    ref = None
    if not a.no_cpu_baseline:
        ref, wall, _ = oracle_cells(su, cells, snap_steps, su.n_iter, min(procs, len(cells)))
    res = {}
    for key, prec in (("fp32", "fp32"), ("fp16_auto", "fp16")):
        r = run_form(su, prec, su.n_iter, snap_steps if ref is not None else 0, 100, a.warmup,
                     autotune=not a.no_autotune)
        e = {"precision": prec, "dtype": DTYPE[prec],
             "value": round(su.n_cells * su.n_iter * r["steps"] / r["elapsed"], 1),
             "vertex_iterations_per_s": round(su.x0.shape[1] * su.n_iter * r["steps"] / r["elapsed"], 1),
             "ms_per_step": round(r["elapsed"] / r["steps"] * 1e3, 4),
             "launch": [list(map(int, c)) for c in r["configs"]]}
        if ref is not None:
            e.update(errors_vs_oracle(su, r["snap"], r["vols"], ref))
        res[key] = e
    res["speedup_fp16_vs_fp32"] = round(res["fp16_auto"]["value"] / res["fp32"]["value"], 4)
    # overlap of the class branches in the step graph: each class alone (its
    # own batch and graph) against the three together
    alone = []
    for k in range(len(su.classes)):
        sk = su.subset(np.nonzero(su.cell_class == k)[0])
        rk = run_form(sk, "fp32", su.n_iter, 0, 100, a.warmup, autotune=not a.no_autotune)
        alone.append(rk["elapsed"] / rk["steps"] * 1e3)
    res["fp32"]["class_alone_ms_per_step"] = [round(t, 4) for t in alone]
    res["fp32"]["branch_overlap"] = round(sum(alone) / res["fp32"]["ms_per_step"], 4)
    # the same 100 steps as ONE graph launch (npfem_run)
    bu, pu, vu, fu, _ = make_batch(su, "fp32", autotune=not a.no_autotune)
    xu, uu = pu.clone(), vu.clone()
    bu.run(fu, su.dt, su.n_iter, 100)  # captures the run's graph
    bu.sync_status()
    pu.copy_(xu)
    vu.copy_(uu)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bu.run(fu, su.dt, su.n_iter, 100)
    torch.cuda.synchronize()
    res["fp32"]["one_launch_ms_per_step"] = round((time.perf_counter() - t0) / 100 * 1e3, 4)
    bu.sync_status()
    bu.close()
    res["workload"] = ("3000 RBC (642 v) + 600 platelets (162 v) + 64 large cells (2562 v), "
                       "weights +-20 % per cell, forces N(0, 0.05^2), 10 PD iterations, one graph "
                       "per step with a branch per class, autotuned launch shapes; errors after "
                       f"{snap_steps} steps on cells {[int(c) for c in cells]}; branch_overlap = "
                       "sum of the classes' step times alone / their step time together; "
                       "one_launch_ms_per_step: the 100 steps as one graph launch")
    out["uneven"] = res
    log(f"uneven: {res}")

    # one RBC in FP64, 100 steps x 20 iterations (the oracle runs it in full)
    s1 = W.single_rbc()
    b1, p1, v1, f1, _ = make_batch(s1, "fp64")
    b1.step(f1, s1.dt, s1.n_iter)
    b1.sync_status()
    p1.copy_(torch.tensor(s1.x0, dtype=torch.float64, device="cuda"))
    v1.zero_()
    el1 = timed_steps(b1, f1, s1.dt, s1.n_iter, s1.n_steps)
    x1 = p1.double().cpu().numpy()
    vol1 = b1.volume()
    b1.close()
    e1 = {"value": round(s1.n_iter * s1.n_steps / el1, 1), "ms_total": round(el1 * 1e3, 3),
          "workload": "1 RBC x 162 vertices, 100 steps x 20 PD iterations, FP64"}
    if not a.no_cpu_baseline:
        r1, wall1, _ = oracle_cells(s1, [0], s1.n_steps, s1.n_iter, 1)
        e1.update(errors_vs_oracle(s1, x1, vol1, r1))
        e1["bound"] = 1e-11
        e1["oracle_cell_iterations_per_s"] = round(s1.n_iter * s1.n_steps / wall1, 1)
    out["single_rbc_fp64"] = e1
    log(f"single_rbc_fp64: {e1}")

    # forward + backward of the differentiation workload
    sa = round_inputs(W.adjoint_rbcs())
    ba, pa, va, fa, _ = make_batch(sa, "fp32")
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
    out["fwd_bwd"] = {"workload": f"{sa.n_cells} RBC x 642 vertices, {n_st} steps x {n_it} PD "
                                  f"iterations, checkpoints every {every} steps, "
                                  "loss sum |x_T - target|^2, FP32",
                      "forward_ms": round(tf * 1e3, 3), "backward_ms": round(tb * 1e3, 3),
                      "fwd_bwd_ms": round((tf + tb) * 1e3, 3),
                      "backward_over_forward": round(tb / tf, 3)}
    log(f"forward+backward: {out['fwd_bwd']}")
    return out


def _oracle_qn(args):
    """Worker: the oracle's quasi-Newton rollout of one cell."""
    susp, c, n_iter, n_steps, hist, ls = args
    _pin_threads()
    from oracle import quasi_newton as Q
    from oracle import solver as S
    mc, x0, v0, f, w = susp.cell_arrays(int(c))
    cs = S.CellSolver(S.operators_for(mc), S.Params(tuple(w), mc.mass, susp.dt))
    x, _ = Q.rollout(cs, x0, v0, f, n_iter, n_steps, hist, ls)
    return int(c), x


def next_rows(a):
    """Throughput and oracle error of the solver's further forms on the
    4096-RBC lattice: viscous damping, wall contacts, the quasi-Newton step
    (stiff twin), and the immersed-boundary transfer."""
    import torch
    from npfem_workload import suspensions as W
    from oracle import solver as S
    from paper_2011_04332_amd import solver
    out = {}
    procs = max(1, min(os.cpu_count() or 1, a.cpu_procs))
    steps, snap = 50, 10
    base = lambda: round_inputs(W.rbc_lattice(n_steps=snap))
    cells = None

    def measure(key, s, n_iter=10, qn=None, oracle=True):
        nonlocal cells
        cells = W.sample_cells(s, [3])
        r = run_form(s, "fp32", n_iter, snap, steps, a.warmup, autotune=not a.no_autotune, qn=qn)
        e = {"value": round(s.n_cells * n_iter * r["steps"] / r["elapsed"], 1),
             "unit": "cell-PD-iterations/s", "ms_per_step": round(r["elapsed"] / r["steps"] * 1e3, 4)}
        if oracle and not a.no_cpu_baseline:
            ref, _, _ = oracle_cells(s, cells, snap, n_iter, min(procs, len(cells)))
            e.update(errors_vs_oracle(s, r["snap"], r["vols"], ref))
            e["bound"] = BOUND["fp32"]
        return e, r

    # viscous damping: alpha h = 0.02, beta/h = 1
    s = base()
    for mc in s.classes:
        mc.damping = (200.0, 1e-4)
    out["damping"], _ = measure("damping", s)
    out["damping"]["workload"] = ("4096 RBC lattice, C = alpha m I + beta K_d with alpha 200/s, "
                                  "beta 1e-4 s, FP32, 10 PD iterations")
    # wall contacts under every cell
    s = W.wall_contacts(base(), depth=0.3)
    out["contacts"], _ = measure("contacts", s)
    out["contacts"]["workload"] = ("4096 RBC lattice, each on a plane wall cutting 0.3 um into it, "
                                   "81 contact points per cell, weight 10, FP32, 10 PD iterations")
    # quasi-Newton vs PD on the stiff twin (dt 1e-2) from perturbed shapes:
    # one step's distance from the converged step (per cell, max over its
    # vertices / R) after equal iteration counts, median and max over cells
    s = W.stiff(W.rbc_lattice(n_cells=1024, n_steps=1), dt=1e-2)
    s.x0 = s.x0 + 0.1 * np.random.default_rng(4).standard_normal(s.x0.shape)
    s = round_inputs(s)
    R = 3.91
    ref = run_form(s, "fp64", 100, 1, 1, 1, autotune=False, qn=(5, 3))["snap"]

    def cell_errs(snap):
        d = np.abs(snap - ref).max(axis=0) / R
        return np.array([d[s.cell_slice(c)].max() for c in range(s.n_cells)])

    curve, rq = {}, None
    for k in (12, 24, 48):
        for name, qn in (("qn", (5, 3)), ("pd", None)):
            r = run_form(s, "fp32", k, 1, 20, a.warmup, autotune=not a.no_autotune, qn=qn)
            ce = cell_errs(r["snap"])
            curve[f"{name}_{k}"] = {"ms_per_step": round(r["elapsed"] / r["steps"] * 1e3, 4),
                                   "err_median": float(np.median(ce)), "err_max": float(ce.max())}
            if name == "qn" and k == 12:
                rq = r
    qn_e = dict(curve["qn_12"])
    if not a.no_cpu_baseline:
        import multiprocessing as mp
        cq = W.sample_cells(s, [2])
        with mp.get_context("spawn").Pool(len(cq), initializer=_pin_threads) as pool:
            res = pool.map(_oracle_qn, [(s, int(c), 12, 1, 5, 3) for c in cq])
        qn_e["max_rel_pos_err"] = float(max(S.rel_position_error(rq["snap"][:, s.cell_slice(c)].T, x)
                                            for c, x in res))
        qn_e["bound"] = BOUND["fp32"]
    out["quasi_newton"] = {"qn_12_iterations_vs_oracle": qn_e, "convergence": curve,
                           "workload": "1024 RBC, dt 1e-2 (stiff twin), shapes perturbed by "
                                       "N(0, 0.1^2) um, one step of k iterations (quasi-Newton: "
                                       "history 5, 3 line-search rounds; PD), FP32; errors per "
                                       "cell against the converged step (100 quasi-Newton "
                                       "iterations in FP64), in units of the cell radius"}
    # immersed-boundary transfer on a periodic 160^3 grid (dx 1 um)
    s = round_inputs(W.rbc_lattice(n_steps=1))
    b, pos, vel, f, _ = make_batch(s, "fp32")
    dims, dx, org0 = (160, 160, 160), 1.0, np.zeros(3)
    nn = int(np.prod(dims))
    rng = np.random.default_rng(6)
    u = torch.tensor(rng.standard_normal((3, nn)), dtype=torch.float32, device="cuda").contiguous()
    orgs = torch.tensor(s.origins + 5.0, dtype=torch.float64, device="cuda").contiguous()
    F = torch.tensor(0.05 * rng.standard_normal(tuple(pos.shape)), dtype=torch.float32,
                     device="cuda").contiguous()
    U = b.ibm_interpolate(orgs, u, dims, dx, org0)
    g = b.ibm_spread(orgs, F, dims, dx, org0)
    reps = 20
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(reps):
        b.ibm_interpolate(orgs, u, dims, dx, org0, out=U)
    ev[1].record()
    ev[2].record()
    for _ in range(reps):
        b.ibm_spread(orgs, F, dims, dx, org0, out=g)
    ev[3].record()
    torch.cuda.synchronize()
    b.sync_status()
    ti = ev[0].elapsed_time(ev[1]) / reps
    ts = ev[2].elapsed_time(ev[3]) / reps
    V = pos.shape[1]
    ibm_e = {"vertices": V, "grid": list(dims), "dx_um": dx,
             "interpolate_ms": round(ti, 4), "interpolate_vertices_per_s": round(V / (ti * 1e-3), 1),
             "interpolate_GBs": round((24 * V + 12 * V + 12 * nn) / (ti * 1e-3) / 1e9, 1),
             "spread_ms": round(ts, 4), "spread_vertices_per_s": round(V / (ts * 1e-3), 1),
             "spread_GBs": round((24 * V + 12 * V + 36 * nn) / (ts * 1e-3) / 1e9, 1),
             "bytes_note": "algorithmic: positions and vertex values once, each grid field once "
                           "(interpolation reads u; spreading clears, accumulates and converts)"}
    if not a.no_cpu_baseline:
        from oracle import ibm
        cs_ = W.sample_cells(s, [2])
        xh = pos.double().cpu().numpy()
        Uh = U.double().cpu().numpy()
        uh = u.double().cpu().numpy().reshape((3,) + dims, order="F")
        err = 0.0
        for c in cs_:
            sl = s.cell_slice(int(c))
            X = (s.origins[int(c)] + 5.0)[None, :] + xh[:, sl].T
            ref = ibm.interpolate(uh, X, org0, dx)
            err = max(err, float(np.abs(Uh[:, sl].T - ref).max() / np.abs(ref).max()))
        ibm_e["interpolate_max_rel_err"] = err
    b.close()
    out["ibm"] = ibm_e
    log(f"next rows: {out}")
    return out


if __name__ == "__main__":
    main()
