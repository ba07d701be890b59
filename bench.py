"""Timestep throughput of the Newton-PCG hot path on one MI355X.

Workload: heterogeneous block, 32^3 hexes x 6 tets (35,937 vertices,
196,608 tets), matrix E = 1e5 Pa with 20 seeded stiff inclusions at 1e10 Pa,
nu = 0.49, rho = 1000, bottom pinned, top driven down 0.01 m per step for 10
steps (then held), gravity, implicit Euler dt = 1/60.  Inputs are synthetic
(seeded generator), resident in HBM before the timed region.

A "step" is one implicit Euler timestep: every Newton iteration's element
and assembly kernels, the PCG solve, the line search and the update.
Prints one JSON line (see --help for the knobs).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=32)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--pc", choices=["jacobi", "two_level"], default="jacobi")
    ap.add_argument("--handles", type=int, default=43)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--spmv-reps", type=int, default=200)
    return ap.parse_args()


def cpu_baseline():
    """The CPU oracle (FP64 Newton + SuperLU) on a bounded sample: one
    timestep of the same generator at 16^3 (24,576 tets), one thread."""
    from threadpoolctl import threadpool_limits

    import scenes
    from oracle import fem, newton
    s = scenes.inclusion_block(16, seed=0, steps=1)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
        newton.newton_step(body, s["x0"], s["v0"], s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](1))
        dt = time.perf_counter() - t0
    # scaled to the 32^3 workload by its 8x tet count (linear scaling: a
    # lower bound on the oracle's cost, whose sparse solve grows faster)
    return dict(value=1.0 / (dt * 8.0), unit="timesteps/s", cores=1, kind="oracle",
                sample=f"one timestep of the same generator at 16^3 (24,576 tets) took {dt:.1f} s on 1 thread; "
                       f"value = 1/(8 x that), linear tet-count scaling to 32^3")


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the multi-GPU layout is design-only.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import scenes
    from paper_2508_13386_amd import ms

    s = scenes.inclusion_block(a.grid, seed=0, steps=a.warmup + a.steps)
    dev = ms.TorchDevice(0)
    ctx = ms.context_from_scene(dev, s)
    basis_s = None
    if a.pc == "two_level":
        t0 = time.perf_counter()
        ctx.ms_build_basis(n_handles=a.handles)
        basis_s = time.perf_counter() - t0
    params = ms.solver_defaults(precision=ms.PREC_MIXED if a.precision == "mixed" else ms.PREC_FP64,
                                preconditioner=ms.PC_TWO_LEVEL if a.pc == "two_level" else ms.PC_BLOCK_JACOBI)
    stats = []

    def step(k):
        ctx.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
        stats.append(ctx.ms_step(s["dt"], params))

    for k in range(1, a.warmup + 1):
        step(k)
    torch.cuda.synchronize()
    dev.stream.synchronize()
    stats.clear()
    t0 = time.perf_counter()
    for k in range(a.warmup + 1, a.warmup + a.steps + 1):
        step(k)
    dev.stream.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = a.steps / elapsed

    # Roofline of the sparse product: the Hessian at the final state in the
    # library's sliced BSR3 layout, timed with HIP events on the library's
    # stream (same kernel and launch shape as inside PCG's products).
    x, _ = ctx.ms_get_state()
    prec = ms.PREC_MIXED if a.precision == "mixed" else ms.PREC_FP64
    _, _, Hb = ctx.ms_eval(x, s["dt"], prec)
    rp, col = ctx.ms_get_pattern()
    dtype = 1 if a.precision == "mixed" else 0
    A = ms.Matrix(dev, rp, col, Hb, dtype)
    td = torch.float32 if dtype else torch.float64
    xs = torch.randn((len(x), 3), dtype=td, device="cuda")
    ys = torch.empty_like(xs)
    dev.stream.synchronize()
    for _ in range(10):
        A.spmv(xs.data_ptr(), ys.data_ptr())
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(dev.stream)
    for _ in range(a.spmv_reps):
        A.spmv(xs.data_ptr(), ys.data_ptr())
    ev1.record(dev.stream)
    ev1.synchronize()
    spmv_us = ev0.elapsed_time(ev1) * 1e3 / a.spmv_reps
    spmv_bytes = A.bytes
    achieved = spmv_bytes / (spmv_us * 1e-6) / 1e9
    A.close()
    ctx.close()

    out = {
        "metric": "Newton-PCG timesteps/s at <=1e-6 rel. disp. error; BSR SpMV HBM GB/s vs peak",
        "value": value,
        "unit": "timesteps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"heterogeneous block {a.grid}^3 hexes x 6 tets, 20 inclusions E=1e10 in E=1e5, "
                               f"nu=0.49, top driven 0.1 m over 10 steps, dt=1/60",
                   "n_verts": int(len(s["rest"])), "n_tets": int(len(s["tets"])),
                   "precision": a.precision, "preconditioner": a.pc,
                   "handles": a.handles if a.pc == "two_level" else None,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_spmv (sliced BSR3)",
                     "bytes_per_launch": spmv_bytes, "avg_launch_us": spmv_us},
        "solver": {"newton_iters": [st["newton_iters"] for st in stats],
                   "pcg_iters": [st["pcg_iters"] for st in stats],
                   "basis_build_s": basis_s},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
