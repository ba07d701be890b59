"""Timestep throughput of the Newton-PCG hot path on one MI355X.

Workload: heterogeneous block, 32^3 hexes x 6 tets (35,937 vertices,
196,608 tets), matrix E = 1e5 Pa with 20 seeded stiff inclusions at 1e10 Pa,
nu = 0.49, rho = 1000, bottom pinned, top driven down 0.01 m per step for 10
steps (then held), gravity, implicit Euler dt = 1/60.  Inputs are synthetic
(seeded generator), resident in HBM before the timed region.

A "step" is one implicit Euler timestep solved to the plain path's Newton
tolerance: every Newton iteration's element and assembly kernels, the
Galerkin coarse operator and its inverse, the PCG solve, the line search and
the update.  The timed form is the mixed-precision (FP32 Hessian, FP64
vectors / gradient / line search / coarse inverse) Newton-PCG with the
two-level preconditioner on the sparse material-aware basis; the plain FP64
block-Jacobi Newton-PCG runs the same steps as the reference form, and the
two trajectories are compared (relative displacement difference).

Prints one JSON line.
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
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_cg_spmv_heterogeneous_block_32.md")
# Newton iteration cap of every timed form: the first driven steps of the
# block can take close to 50 iterations (the library default)
MAX_NEWTON = 200
KERNEL_SOURCE = os.path.join(ROOT, "paper_2508_13386_amd", "csrc", "kernels_cg.hip")
METRIC = "Newton-PCG timesteps/s at <=1e-6 rel. disp. error; BSR SpMV HBM GB/s vs peak"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=32)
    ap.add_argument("--projection", choices=["clamp", "abs"], default="clamp",
                    help="projected element Hessians: negative eigenvalues clamped to zero or made positive")
    ap.add_argument("--scene", choices=["block", "gyroid", "sliding", "stacked"], default="block",
                    help="block: the heterogeneous block (--grid); gyroid: the contact scene, a gyroid-lattice "
                         "sphere voxelized at --grid^3 falling at 5 m/s onto a rigid half-space; sliding: a "
                         "--grid^3 cube sliding on the half-space with lagged friction (mu = 0.5)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed")
    ap.add_argument("--integrator", choices=["euler", "bdf2"], default="euler",
                    help="implicit Euler or BDF2 (first step implicit Euler) for every form in the run")
    ap.add_argument("--pc", choices=["jacobi", "two_level", "additive", "vcycle"], default="additive")
    ap.add_argument("--handles", type=int, default=None,
                    help="basis handles (144 on the benchmarked block, else 192)")
    ap.add_argument("--oversample", type=float, default=1.0, help="k-means++ seed oversampling of the basis build")
    ap.add_argument("--rigid", type=float, default=1e3,
                    help="basis weights constant on connected sets of tets with E >= RIGID x min E (0: off; "
                         "the heterogeneous block's inclusions are 1e5 x its matrix)")
    ap.add_argument("--jump", type=float, default=0.25,
                    help="jump penalty of the basis partitioning (stiffness factor on material interfaces)")
    ap.add_argument("--lattice", type=int, default=0, help="1: basis seeds on a fixed lattice (no pruning)")
    ap.add_argument("--eta-max", type=float, default=0.1, help="largest PCG forcing term (Eisenstat-Walker)")
    ap.add_argument("--eta-min", type=float, default=None,
                    help="smallest PCG forcing term (default 1e-3 for the block, 1e-4 for the other workloads)")
    ap.add_argument("--coarse-every", type=int, default=1,
                    help="rebuild U^T H U and its inverse every this many Newton iterations (0: once per step)")
    ap.add_argument("--smoother", type=int, default=None, choices=[0, 1],
                    help="block part of the preconditioner: 0 3x3 vertex blocks, 1 vertex aggregates of up to 8 "
                         "(1 on the benchmarked block, else 0)")
    ap.add_argument("--endgame-fp64", type=int, default=None,
                    help="mixed precision: FP64 Hessian in the Newton endgame (0 on the benchmarked block, else 1)")
    ap.add_argument("--newton-tol", type=float, default=1e-9,
                    help="Newton stop: a full step with ||d|| <= newton_tol * ||x - x^t||")
    ap.add_argument("--endgame-ratio", type=float, default=None,
                    help="endgame once ||d|| <= ratio * ||x - x^t|| (exact Hessian; FP64 with --endgame-fp64); "
                         "default 3e-2 for the block, 1e-3 for the other workloads")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the per-step error check against tightly converged FP64 steps")
    ap.add_argument("--coarse-move", type=float, default=None,
                    help="> 0: rebuild U^T H U once the iterate has moved by this fraction of the step's "
                         "displacement since the last rebuild (replaces --coarse-every; 0.8 on the benchmarked "
                         "block, else 0.2)")
    ap.add_argument("--workload", choices=["block32", "batch64", "learned", "spmv_sweep", "paper", "cubature"],
                    default="block32",
                    help="block32: the heterogeneous block (default); batch64: 64 uneven scenes stepped together; "
                         "learned: train the coarse warm start on trajectories and evaluate it on held-out seeds; "
                         "spmv_sweep: the PCG product kernel on the heterogeneous block at --sweep grid sizes; "
                         "paper: the paper's three-level step (Alg. 1/2) and its error against the exact step; "
                         "cubature: the coarse matrix integrated by modal moment-fitting cubature (Sec. 3.8)")
    ap.add_argument("--cub-tol", type=float, default=1e-9, help="cubature workload: moment residual tolerance")
    ap.add_argument("--cub-batch", type=int, default=16,
                    help="cubature workload: tets drawn initially and per round of the fit")
    ap.add_argument("--sweep", default="32,64,96,128", help="grid sizes of the spmv_sweep workload")
    ap.add_argument("--order", choices=["natural", "random", "rcm"], default="natural",
                    help="vertex numbering of the spmv_sweep meshes")
    ap.add_argument("--train-seeds", type=int, default=40)
    ap.add_argument("--eval-seeds", type=int, default=6)
    ap.add_argument("--traj-grid", type=int, default=16)
    ap.add_argument("--traj-steps", type=int, default=30)
    ap.add_argument("--traj-kind", choices=["inclusions", "drive"], default="inclusions",
                    help="learned workload: per-seed inclusions with a 43-handle lattice basis, or one fixed "
                         "geometry with a per-seed drive and one material-aware 43-handle basis")
    ap.add_argument("--no-reference", action="store_true", help="skip the plain FP64 block-Jacobi run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=200, help="back-to-back replays of the product kernel")
    ap.add_argument("--trace-summary", metavar="CSV",
                    help="only summarise a rocprofv3 kernel_trace.csv: per kernel, the mean duration over all "
                         "dispatches and over those that did work (longer than --work-us)")
    ap.add_argument("--work-us", type=float, default=4.0)
    ap.add_argument("--by-grid", action="store_true", help="with --trace-summary: split kernels by grid size")
    ap.add_argument("--tail", nargs=2, metavar=("NAME", "N"),
                    help="with --trace-summary: also split the dispatches of kernels whose name contains NAME "
                         "into their last N and the rest")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (scale for HBM byte counters)")
    a = ap.parse_args()
    # policy of the benchmarked block; the other workloads keep the policy they were measured with
    block = a.workload == "block32" and a.scene == "block"
    if a.eta_min is None:
        a.eta_min = 3e-2 if block else 1e-4
    if a.endgame_ratio is None:
        a.endgame_ratio = 1e-1 if block else 1e-3
    if a.handles is None:
        a.handles = 144 if block else 192
    if a.endgame_fp64 is None:
        a.endgame_fp64 = 0 if block else 1
    if a.smoother is None:
        a.smoother = 1 if block else 0
    if a.coarse_move is None:
        a.coarse_move = 0.8 if block else 0.2
    return a


def cpu_baseline(scene="block", grid=32, n_tets=None):
    """The CPU oracle (FP64 Newton + SuperLU, half-space barrier and CCD
    filter for the contact scene) on a bounded sample for the scenes other
    than the heterogeneous block: one timestep of the same generator at a
    lower resolution (half the grid; 3/8 of it for the contact scene, whose
    oracle step is costlier), one thread, scaled to the workload by its tet
    count (linear scaling: a lower bound on the oracle's cost, whose sparse
    solve grows faster)."""
    from threadpoolctl import threadpool_limits

    import scenes
    from oracle import fem, newton
    g = max(4, (3 * grid) // 8 if scene == "gyroid" else grid // 2)
    if scene == "stacked":  # the oracle's per-pair derivatives are costly: the smallest cubes
        g = 2
        s = scenes.stacked_cubes(N=g, steps=1)
    elif scene == "gyroid":
        s = scenes.gyroid_sphere(res=g)
    elif scene == "sliding":
        s = scenes.sliding_cube(g, steps=1)
    else:
        s = scenes.inclusion_block(g, seed=0, steps=1)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
        newton.newton_step(body, s["x0"], s["v0"], s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](1),
                           halfspace=s["halfspace"], selfcontact=s.get("selfcontact"))
        dt = time.perf_counter() - t0
    ratio = (n_tets or 8 * len(s["tets"])) / len(s["tets"])
    return dict(value=1.0 / (dt * ratio), unit="timesteps/s", cores=1, kind="oracle", cpu=cpu_model(),
                sample=f"one timestep of the same generator at {g}^3 ({len(s['tets']):,} tets) took {dt:.1f} s on "
                       f"1 thread; value = 1/({ratio:.2f} x that), linear tet-count scaling to the workload")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_on_workload(s, check, threads):
    """One Newton iteration of the CPU oracle on the benchmarked workload
    itself: the checked timestep k from the GPU's start state (x^t, v^t),
    with the oracle's Newton started at the GPU's converged state (the
    minimiser does not depend on the first iterate, so one exact Newton
    correction lands on the oracle's own minimiser).  Returns the seconds
    per oracle Newton iteration (mesh precompute excluded), the iterations,
    e_rel = ||x_gpu - x_orc|| / ||x_orc - x^t|| and the BLAS threads used."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import fem, newton
    x0, v0, x1, k = check["x0"], check["v0"], check["x1"], check["step"]
    body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
    with threadpool_limits(limits=threads):
        used = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
        t0 = time.perf_counter()
        xo, _, its = newton.newton_step(body, x0, v0, s["dt"], s["gravity"], s["dirichlet"], s["dbc_targets"](k),
                                        halfspace=s["halfspace"], x_start=x1)
        dt = time.perf_counter() - t0
    e = float(np.linalg.norm(x1 - xo) / np.linalg.norm(xo - x0))
    return dt / max(1, its), its, e, used


def cpu_baseline_on_workload(s, check):
    """cpu_baseline of the heterogeneous block: the oracle's seconds per
    Newton iteration measured on the workload itself (oracle_on_workload),
    times the Newton iterations of that timestep (the GPU's count: a whole
    oracle step, about ten minutes at this size, is more than a bounded
    sample), on one thread (SuperLU is sequential), and the same with all
    host threads."""
    per_it, its, e, _ = oracle_on_workload(s, check, 1)
    per_all, _, _, used = oracle_on_workload(s, check, None)
    n_it = check["newton_iters"]
    out = dict(value=1.0 / (per_it * n_it), unit="timesteps/s", cores=1, kind="oracle", cpu=cpu_model(),
               host_cores=os.cpu_count(),
               sample=f"one oracle Newton iteration (assembly, SuperLU factorisation and solve) on the "
                      f"{len(s['tets']):,}-tet workload itself, timestep {check['step']}: {per_it:.1f} s on 1 "
                      f"thread; value = 1/({n_it} Newton iterations x that)",
               all_cores=dict(value=1.0 / (per_all * n_it), cores=used,
                              sample=f"the same iteration with all host threads: {per_all:.1f} s"))
    return out, dict(step=check["step"], e_rel=e, oracle_newton_iters=its, bound=1e-6,
                     check="the GPU's converged state of this timestep against the oracle's minimiser "
                           "(FP64 Newton + SuperLU) from the same start state")


def measured_traffic(kernel_name, workload):
    """HBM bytes per launch of the product kernel from the committed counter
    summary (FETCH_SIZE x copy factor + WRITE_SIZE x copy factor), or None
    when the summary is missing, was taken on another workload, holds no
    figure for this kernel instance, or the kernel source has changed since
    the counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip().strip("`")] = v.strip().strip("`")
    src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != src or fields.get("workload") != workload:
        return None
    try:
        return float(fields["traffic_bytes_per_launch " + kernel_name])
    except (KeyError, ValueError):
        return None


def trace_summary(path, work_us, tail=None, by_grid=False):
    """Per-kernel dispatch statistics of a rocprofv3 kernel trace (per kernel
    and grid size with by_grid).  Kernels of the PCG loop that start after
    the solve has converged return at once; 'working' dispatches are those
    longer than work_us."""
    import csv
    acc = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            d = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-3
            grid = row.get("Grid_Size", row.get("Grid_Size_X", "?"))
            key = row["Kernel_Name"][:90] + (f" grid {grid}" if by_grid else "")
            a = acc.setdefault(key, [0, 0.0, 0, 0.0])
            a[0] += 1
            a[1] += d
            if d > work_us:
                a[2] += 1
                a[3] += d
    rows = sorted(acc.items(), key=lambda kv: -kv[1][1])
    for name, (n, tot, nw, totw) in rows[:25]:
        print(json.dumps({"kernel": name, "dispatches": n, "mean_us": tot / n, "working": nw,
                          "working_mean_us": (totw / nw) if nw else None, "total_ms": tot * 1e-3}))
    if tail:
        key, last = tail[0], int(tail[1])
        with open(path) as f:
            ds = sorted((int(r["Start_Timestamp"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
                        for r in csv.DictReader(f) if key in r["Kernel_Name"])
        for part, sel in (("last", ds[-last:]), ("rest", ds[:-last])):
            w = [d for _, d in sel if d > work_us]
            print(json.dumps({"kernel_contains": key, "part": part, "dispatches": len(sel), "working": len(w),
                              "working_mean_us": sum(w) / len(w) if w else None}))


def copy_probe(mib):
    """A fill kernel writing MIB MiB, then five plain copies of that buffer:
    the reference against which per-dispatch HBM byte counters are scaled."""
    import torch
    n = mib * 2**20 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "copies": 5}), flush=True)


def run(dev, s, params, warmup, steps, basis=None, handles=0, timed=True, oversample=1.0, lattice=0,
        cubature=None, jump=0.25, rigid=0.0):
    """Runs warmup + steps timesteps; returns (timesteps/s, per-step stats,
    states after each timed step, context, basis seconds).  cubature =
    (tets, weights) integrates the elastic part of the coarse matrix by
    cubature."""
    import torch

    from paper_2508_13386_amd import ms
    ctx = ms.context_from_scene(dev, s)
    basis_s = None
    if basis is not None:
        ctx.ms_set_basis(basis["origins"], basis["vptr"], basis["vhandle"], basis["vphi"])
    elif handles:
        t0 = time.perf_counter()
        ctx.ms_build_basis(n_handles=handles, oversample=oversample, lattice_seeding=lattice, jump_penalty=jump,
                           rigid_contrast=rigid)
        basis_s = time.perf_counter() - t0
    if cubature is not None:
        ctx.ms_set_cubature(*cubature)
        ctx.ms_set_coarse_integration(ms.COARSE_CUBATURE)
    stats, states = [], []
    for k in range(1, warmup + 1):
        ctx.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
        ctx.ms_step(s["dt"], params)
    dev.stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warmup + 1, warmup + steps + 1):
        ctx.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
        stats.append(ctx.ms_step(s["dt"], params))
    dev.stream.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    x, _ = ctx.ms_get_state()
    states.append(x)
    return steps / elapsed, elapsed, stats, states, ctx, basis_s


def step_errors(dev, s, ctx, params, warmup, steps):
    """Per-step error of the benchmarked form: the timed steps are replayed
    (deterministic, untimed) from the same start, and each one is compared
    with a tightly converged FP64 step (block-Jacobi PCG, ||d|| <= 1e-11
    ||x - x^t||, no a-posteriori stop) taken from the same state:
    e_rel = ||x_form - x_tight|| / ||x_tight - x^t||."""
    from paper_2508_13386_amd import ms
    tight = ms.context_from_scene(dev, s)
    tparams = ms.solver_defaults(precision=ms.PREC_FP64, preconditioner=ms.PC_BLOCK_JACOBI, forcing=0,
                                 newton_tol=1e-11, max_newton=100)
    ctx.ms_set_state(s["x0"], s["v0"])
    errs = []
    last = None
    for k in range(1, warmup + steps + 1):
        ctx.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
        x0, v0 = ctx.ms_get_state()
        st = ctx.ms_step(s["dt"], params)
        x1, _ = ctx.ms_get_state()
        if k <= warmup:
            continue
        last = dict(step=k, x0=x0, v0=v0, x1=x1, newton_iters=int(st["newton_iters"]))
        tight.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
        tight.ms_set_state(x0, v0)
        tight.ms_step(s["dt"], tparams)
        xt, _ = tight.ms_get_state()
        errs.append(float(np.linalg.norm(x1 - xt) / np.linalg.norm(xt - x0)))
    tight.close()
    return {"check": "each timed step vs the same step solved by FP64 block-Jacobi Newton-PCG to "
                     "||d|| <= 1e-11 ||x - x^t|| from the same state", "e_rel_per_step": errs,
            "e_rel_max": max(errs), "bound": 1e-6}, last


def batch_main(a):
    """64 uneven scenes (cubes / ellipsoids, 1e3-5e4 tets each, E log-uniform
    in [1e5, 1e9], bottom layer pinned, gravity) advanced by ms_batch_create /
    ms_batch_advance with the additive two-level preconditioner (a basis per
    scene, about one handle per 1,500 tets, at least four; basis builds are
    excluded from the timing) or block-Jacobi (--pc jacobi).  Reference
    forms: the same scenes stepped one after another by ms_step with the
    same preconditioner (bitwise the same states), and the batch with
    block-Jacobi.  Accuracy: the last step of every 16th scene against the
    oracle's minimiser from the same start state."""
    import torch

    import scenes
    from paper_2508_13386_amd import ms
    scs = scenes.batch_scenes(64, seed=0)
    dev = ms.TorchDevice(0)
    prec = ms.PREC_MIXED if a.precision == "mixed" else ms.PREC_FP64
    two_level = a.pc != "jacobi"
    jac = ms.solver_defaults(precision=prec, forcing=1, pcg_eta_max=a.eta_max, pcg_eta_min=a.eta_min)
    tl = ms.solver_defaults(precision=prec, forcing=1, pcg_eta_max=a.eta_max, pcg_eta_min=a.eta_min,
                            preconditioner=ms.PC_TWO_LEVEL_ADDITIVE, coarse_move=a.coarse_move)
    params = tl if two_level else jac
    dt = scs[0]["dt"]
    handles = [max(4, int(round(len(s["tets"]) / 1500))) for s in scs]

    def contexts(with_basis):
        ctxs = [ms.context_from_scene(dev, s) for s in scs]
        t0 = time.perf_counter()
        if with_basis:
            for c, m in zip(ctxs, handles):
                c.ms_build_basis(n_handles=m, seed=1)
        return ctxs, time.perf_counter() - t0

    def timed(step_all, with_basis, keep_last=False):
        ctxs, basis_s = contexts(with_basis)
        for _ in range(a.warmup):
            step_all(ctxs)
        dev.stream.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        starts = None
        for k in range(a.steps):
            if keep_last and k == a.steps - 1:
                starts = [c.ms_get_state() for c in ctxs]
            stats.append(step_all(ctxs))
        dev.stream.synchronize()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        xs = [c.ms_get_state()[0] for c in ctxs]
        return a.steps / el, el, stats, xs, starts, basis_s, ctxs

    def batched(ctxs, p, holder={}):
        if "b" not in holder or holder["ctxs"] is not ctxs:
            holder["b"], holder["ctxs"] = ms.Batch(ctxs), ctxs
        return holder["b"].advance(dt, p)

    value, elapsed, stats, xb, starts, basis_s, bctxs = timed(lambda cs: batched(cs, params), two_level,
                                                              keep_last=True)
    accuracy = None
    if not a.no_accuracy:
        from oracle import fem, newton
        errs = {}
        for q in range(0, len(scs), 16):
            s = scs[q]
            x0, v0 = starts[q]
            body = fem.Body(s["rest"], s["tets"], s["E"], s["nu"], s["rho"])
            xo, _, _ = newton.newton_step(body, x0, v0, dt, s["gravity"], s["dirichlet"],
                                          s["dbc_targets"](a.warmup + a.steps), x_start=xb[q])
            err, disp, xn = (float(np.linalg.norm(xb[q] - xo)), float(np.linalg.norm(xo - x0)),
                             float(np.linalg.norm(xo)))
            errs[q] = {"e_rel": err / disp, "disp_m": disp, "abs_err_m": err, "abs_err_over_x": err / xn,
                       "ok": bool(err <= 1e-6 * disp or err <= 1e-12 * xn)}
        accuracy = {"check": "last timed step of every 16th scene against the oracle's minimiser (FP64 Newton + "
                             "SuperLU) from the same start state; a step passes with e_rel <= 1e-6 or, for an "
                             "almost static step, an error below 1e-12 ||x|| (the resolution of FP64 positions)",
                    "per_scene": errs, "all_ok": bool(all(v["ok"] for v in errs.values()))}
    for c in bctxs:
        c.close()
    ref = None
    if not a.no_reference:
        rv, _, rstats, xr, _, _, rctxs = timed(lambda cs: [c.ms_step(dt, params) for c in cs], two_level)
        for c in rctxs:
            c.close()
        ref = {"form": "the same 64 scenes stepped one after another (ms_step), same preconditioner", "value": rv,
               "unit": "batch timesteps/s", "speedup": value / rv,
               "bitwise_equal_states": bool(all(np.array_equal(p, q) for p, q in zip(xb, xr)))}
        if two_level:
            jv, _, jstats, _, _, _, jctxs = timed(lambda cs: batched(cs, jac), False)
            for c in jctxs:
                c.close()
            ref["batched_block_jacobi"] = {"value": jv, "speedup_of_two_level": value / jv,
                                           "max_pcg_iters": [max(st["pcg_iters"] for st in step) for step in jstats]}
    out = {
        "metric": "batched Newton-PCG timesteps/s (all 64 scenes per step)",
        "value": value, "unit": "batch timesteps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if a.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": "64 uneven scenes, seed 0", "n_tets": int(sum(len(s["tets"]) for s in scs)),
                   "n_verts": int(sum(len(s["rest"]) for s in scs)), "precision": a.precision,
                   "preconditioner": "additive two-level" if two_level else "jacobi",
                   "handles_total": int(sum(handles)) if two_level else None, "parallelism": "single GPU"},
        "solver": {"max_newton_iters": [max(st["newton_iters"] for st in step) for step in stats],
                   "max_pcg_iters": [max(st["pcg_iters"] for st in step) for step in stats],
                   "basis_build_s": basis_s},
        "reference_form": ref,
        "accuracy": accuracy,
    }
    print(json.dumps(out), flush=True)


def learned_main(a):
    """Trajectories of the heterogeneous-block generator (per-seed inclusions,
    10-step ramp then held) at traj_grid^3 with a 64-handle lattice basis;
    the warm-start network is trained on the training seeds' coarse states
    (GPU, bf16 matrix cores) and the timesteps of held-out seeds are run with
    and without it.  Both runs solve every step to the plain-path tolerance;
    the gain is in Newton / PCG iterations and time."""
    import torch

    import scenes
    from paper_2508_13386_amd import ms
    dev = ms.TorchDevice(0)
    prec = ms.PREC_MIXED if a.precision == "mixed" else ms.PREC_FP64
    base = dict(precision=prec, preconditioner=ms.PC_TWO_LEVEL_ADDITIVE, forcing=1, pcg_eta_max=a.eta_max,
                pcg_eta_min=a.eta_min, max_newton=100, coarse_move=a.coarse_move, mixed_endgame_fp64=a.endgame_fp64)
    plain64 = dict(precision=ms.PREC_FP64, preconditioner=ms.PC_BLOCK_JACOBI, forcing=1, pcg_eta_max=a.eta_max,
                   pcg_eta_min=a.eta_min, max_newton=100)

    def trajectory(seed, warm=None, form=None):
        """Coarse states, step stats and states of one trajectory, or None if
        a step fails to converge (reported and left out)."""
        try:
            return _trajectory(seed, warm, form or base)
        except ms.MSError as e:
            print(f"trajectory seed {seed} warm {warm is not None}: {e}", file=sys.stderr, flush=True)
            return None

    fixed_basis = {}

    def _trajectory(seed, warm, form):
        if a.traj_kind == "drive":
            sc = scenes.learned_drive_scene(seed, N=a.traj_grid, steps=a.traj_steps)
        else:
            sc = scenes.learned_trajectory_scene(seed, N=a.traj_grid, steps=a.traj_steps)
        c = ms.context_from_scene(dev, sc)
        try:
            if a.traj_kind == "drive":
                # one geometry: one material-aware basis, built once and shared
                if not fixed_basis:
                    c.ms_build_basis(n_handles=43)
                    fixed_basis.update(c.ms_get_basis())
                else:
                    c.ms_set_basis(fixed_basis["origins"], fixed_basis["vptr"], fixed_basis["vhandle"],
                                   fixed_basis["vphi"])
            else:
                c.ms_build_basis(n_handles=43, lattice_seeding=1)
            r = 12 * c.ms_get_basis()["m"]
            if warm is not None:
                c.ms_set_warmstart(*warm)
            qs = [c.ms_get_coarse(r)]
            stats, xs = [], []
            for k in range(1, a.traj_steps + 1):
                c.ms_set_dirichlet(sc["dirichlet"], sc["dbc_targets"](k))
                stats.append(c.ms_step(sc["dt"], ms.solver_defaults(warm_start=1 if warm else 0, **form)))
                qs.append(c.ms_get_coarse(r))
                xs.append(c.ms_get_state()[0])
        finally:
            c.close()
        print(f"trajectory seed {seed} warm {warm is not None}: newton {sum(st['newton_iters'] for st in stats)}",
              file=sys.stderr, flush=True)
        return np.array(qs), stats, xs, r

    t0 = time.perf_counter()
    train = [t for t in (trajectory(sd) for sd in scenes.TRAIN_SEEDS[:a.train_seeds]) if t is not None]
    gen_s = time.perf_counter() - t0
    r = train[0][3]
    train = [t for t in train if t[3] == r]
    Xs, Ys = [], []
    for qs, _, _, _ in train:
        for k in range(1, len(qs) - 1):
            Xs.append(np.concatenate([qs[k - 1], qs[k]]))
            Ys.append(qs[k + 1] - (2 * qs[k] - qs[k - 1]))
    X, Y = np.array(Xs), np.array(Ys)
    # one scale per array (not per coordinate): coordinates that barely move
    # (handles near the pinned base) would otherwise have round-off-level
    # accelerations blown up to unit variance
    mean = X.mean(axis=0)
    std = np.full(X.shape[1], (X - mean).std() + 1e-30)
    oscale = np.full(Y.shape[1], Y.std() + 1e-30)
    Xn, Yn = ((X - mean) / std).astype(np.float32), (Y / oscale).astype(np.float32)
    p0 = scenes.mlp_init(2 * r, 256, r, seed=0)
    steps = 1500
    order = scenes.minibatch_order(len(Xn), 128, steps, seed=1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    params, losses, _ = ms.ms_mlp_train(dev, p0, Xn, Yn, order, lr=1e-3)
    train_s = time.perf_counter() - t1
    warm = (params, mean, std, oscale)
    rows, skipped = [], []
    for sd in scenes.HELDOUT_SEEDS[:a.eval_seeds]:
        t0_, t1_, t2_ = trajectory(sd), trajectory(sd, warm), trajectory(sd, form=plain64)
        if t0_ is None or t1_ is None or t2_ is None:
            skipped.append(dict(seed=sd, base_failed=t0_ is None, warm_failed=t1_ is None, plain_failed=t2_ is None))
            continue
        _, s0, x0, _ = t0_
        _, s1, x1, _ = t1_
        _, s2, x2, _ = t2_
        e = max(float(np.linalg.norm(p - q) / max(np.linalg.norm(p), 1e-300)) for p, q in zip(x0, x1))
        e2 = max(float(np.linalg.norm(p - q) / max(np.linalg.norm(p), 1e-300)) for p, q in zip(x2, x1))
        rows.append(dict(seed=sd, newton=[sum(st["newton_iters"] for st in s0), sum(st["newton_iters"] for st in s1)],
                         pcg=[sum(st["pcg_iters"] for st in s0), sum(st["pcg_iters"] for st in s1)],
                         ms=[sum(st["time_ms"] for st in s0), sum(st["time_ms"] for st in s1)],
                         plain_fp64_ms=sum(st["time_ms"] for st in s2),
                         used=sum(st["warm_start_used"] for st in s1), max_state_rel_diff=e,
                         max_state_rel_diff_vs_plain_fp64=e2))
    t_base = sum(rw["ms"][0] for rw in rows)
    t_warm = sum(rw["ms"][1] for rw in rows)
    t_plain = sum(rw["plain_fp64_ms"] for rw in rows)
    out = {
        "metric": "held-out timesteps/s with the learned coarse warm start",
        "value": 1e3 * a.traj_steps * len(rows) / t_warm, "unit": "timesteps/s", "n_gpus": 1,
        "steps": a.traj_steps * len(rows), "warmup": 0, "ms_per_step": t_warm / (a.traj_steps * len(rows)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": f"heterogeneous block {a.traj_grid}^3, "
                               + ("per-seed inclusions" if a.traj_kind == "inclusions" else
                                  "one geometry, per-seed drive (0.05-0.15 m over 6-14 steps)")
                               + f", {a.traj_steps} steps",
                   "handles": r // 12, "train_seeds": len(train), "samples": int(len(Xn)),
                   "network": f"{2 * r}-256-256-{r} SiLU, bf16 products", "parallelism": "single GPU"},
        "training": {"steps": steps, "batch": 128, "lr": 1e-3, "loss_first": float(losses[0]),
                     "loss_last": float(np.mean(losses[-50:])), "train_s": train_s, "data_gen_s": gen_s,
                     # matrix-core work: forward 2 flops per weight and sample, backward twice that
                     "gemm_tflops": 6.0 * 128 * steps * (2 * r * 256 + 256 * 256 + 256 * r) / train_s * 1e-12,
                     "bf16_dense_peak_tflops": 2500.0},
        "reference_form": {"form": "same held-out steps without the warm start (inertial predictor)",
                           "value": 1e3 * a.traj_steps * len(rows) / t_base, "unit": "timesteps/s",
                           "speedup": t_base / t_warm},
        "plain_fp64_form": {"form": "same held-out steps, plain FP64 Newton-PCG with 3x3 block-Jacobi",
                            "value": 1e3 * a.traj_steps * len(rows) / t_plain, "unit": "timesteps/s",
                            "speedup_of_learned_mixed": t_plain / t_warm},
        "per_seed": rows,
        "skipped": skipped,
        "train_trajectories_failed": a.train_seeds - len(train),
    }
    print(json.dumps(out), flush=True)


def paper_main(a):
    """The paper's three-level timestep (affine and sparse subspace levels,
    lagged-Hessian refinement, subspace-decrement stop) on the heterogeneous
    block and on the contact scene.  Each timed step starts from the paper
    trajectory's state; from the same state the exact step (plain mixed
    two-level Newton-PCG to the plain-path tolerance) is solved untimed, and
    the difference is reported as the paper measures it (per-vertex
    displacement difference over the bounding-box diagonal) and as e_rel."""
    import torch

    import scenes
    from paper_2508_13386_amd import ms
    dev = ms.TorchDevice(0)
    prec = ms.PREC_MIXED if a.precision == "mixed" else ms.PREC_FP64
    exact = ms.solver_defaults(precision=prec, preconditioner=ms.PC_TWO_LEVEL_ADDITIVE, forcing=1,
                               pcg_eta_max=a.eta_max, pcg_eta_min=a.eta_min, coarse_move=a.coarse_move,
                               mixed_endgame_fp64=a.endgame_fp64)
    pparams = ms.solver_defaults(mode=ms.MODE_PAPER, precision=prec, refine_iters=0, max_newton=100)
    cases = [("cube %d^3, per-tet E log-uniform in [1e5, 1e8], bottom pinned, gravity" % a.grid,
              scenes.plain_cube(a.grid, seed=0, steps=a.warmup + a.steps), a.handles),
             ("gyroid-lattice sphere at 32^3 falling onto a rigid half-space",
              scenes.gyroid_sphere(res=32), a.handles),
             ("heterogeneous block %d^3, 20 inclusions E=1e10 in E=1e5" % a.grid,
              scenes.inclusion_block(a.grid, seed=0, steps=a.warmup + a.steps), a.handles)]
    for name, s, m in cases:
        c = ms.context_from_scene(dev, s)
        c.ms_build_basis(n_handles=m, oversample=a.oversample)
        bbox = float(np.linalg.norm(s["rest"].max(axis=0) - s["rest"].min(axis=0)))
        times, etimes, errs, ebox, iters = [], [], [], [], []
        failure = None
        x, v = s["x0"].copy(), s["v0"].copy()
        for k in range(1, a.warmup + a.steps + 1):
            if len(s["dirichlet"]):
                c.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
            c.ms_set_state(x, v)
            dev.stream.synchronize()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                st = c.ms_step(s["dt"], pparams)
            except ms.MSError as e:
                failure = f"step {k}: {e}"
                break
            dev.stream.synchronize()
            t1 = time.perf_counter()
            xp, vp = c.ms_get_state()
            c.ms_set_state(x, v)
            dev.stream.synchronize()
            t2 = time.perf_counter()
            c.ms_step(s["dt"], exact)
            dev.stream.synchronize()
            t3 = time.perf_counter()
            xe, _ = c.ms_get_state()
            if k > a.warmup:
                times.append(t1 - t0)
                etimes.append(t3 - t2)
                errs.append(float(np.linalg.norm(xp - xe) / np.linalg.norm(xe - x)))
                ebox.append(float(np.linalg.norm(xp - xe, axis=1).max() / bbox))
                iters.append((st["newton_iters"], st["pcg_iters"]))
            x, v = xp, vp
        c.close()
        print(json.dumps({"workload": "paper", "scene": name, "n_verts": len(s["rest"]), "n_tets": len(s["tets"]),
                          "handles": m, "precision": a.precision,
                          "timesteps_per_s": len(times) / sum(times) if times else None,
                          "ms_per_step": 1e3 * sum(times) / len(times) if times else None, "steps": len(times),
                          "failure": failure,
                          "exact_step_timesteps_per_s": len(etimes) / sum(etimes) if etimes else None,
                          "newton_and_pcg_iters": iters, "e_rel_vs_exact_per_step": errs,
                          "max_vertex_error_over_bbox_per_step": ebox,
                          "note": "error of the paper's approximate step against the exact minimiser from the "
                                  "same state (the paper reports about 1e-2)"}), flush=True)


def cubature_main(a):
    """Modal moment-fitting cubature of the coarse matrix (Sec. 3.8, Alg. 3)
    on the heterogeneous block: the host fit, the coarse-matrix integration
    time (exact Galerkin product vs cubature), the difference of the two
    matrices, and the benchmarked plain form with the cubature coarse matrix
    against the same form with the exact one (timesteps/s, PCG iterations,
    per-step error).  Then paper mode on the cube with the cubature subspace
    matrix against exact integration, from the same states."""
    import scenes
    from paper_2508_13386_amd import ms
    dev = ms.TorchDevice(0)
    prec = ms.PREC_MIXED if a.precision == "mixed" else ms.PREC_FP64
    s = scenes.inclusion_block(a.grid, seed=0, steps=a.warmup + a.steps + 1)
    params = ms.solver_defaults(precision=prec, preconditioner=ms.PC_TWO_LEVEL_ADDITIVE, forcing=1,
                                pcg_eta_max=a.eta_max, pcg_eta_min=a.eta_min, coarse_every=a.coarse_every,
                                coarse_move=a.coarse_move, mixed_endgame_fp64=a.endgame_fp64,
                                endgame_ratio=a.endgame_ratio)
    v_ex, _, st_ex, states_ex, ctx, basis_s = run(dev, s, params, a.warmup, a.steps, handles=a.handles,
                                                  oversample=a.oversample)
    print(f"# exact coarse matrix: {v_ex:.3f} timesteps/s", flush=True)
    basis = ctx.ms_get_basis()
    t0 = time.perf_counter()
    worst = ctx.ms_build_cubature(tol=a.cub_tol, n_init=a.cub_batch, n_add=a.cub_batch, seed=0)
    fit_s = time.perf_counter() - t0
    tets, w = ctx.ms_get_cubature()
    print(f"# cubature fit: {len(tets)} of {len(s['tets'])} tets in {fit_s:.1f} s, worst residual {worst:.2e}",
          flush=True)
    x_now, _ = ctx.ms_get_state()
    r = 12 * basis["m"]
    integ = {}
    for pname, pr in (("fp64", ms.PREC_FP64), ("mixed", ms.PREC_MIXED)):
        out = {}
        for mode_name, mode in (("exact", ms.COARSE_EXACT), ("cubature", ms.COARSE_CUBATURE)):
            ctx.ms_set_coarse_integration(mode)
            ctx.ms_eval(x_now, s["dt"], prec=pr, hess=False)
            K = ctx.ms_get_coarse_matrix(r)
            us, _ = ctx.ms_time_kernel(6, pr, a.kernel_reps)
            out[mode_name] = (K, us)
        Ke, Kc = out["exact"][0], out["cubature"][0]
        integ[pname] = {"exact_us": out["exact"][1], "cubature_us": out["cubature"][1],
                        "speedup": out["exact"][1] / out["cubature"][1],
                        "rel_frobenius_difference": float(np.linalg.norm(Kc - Ke) / np.linalg.norm(Ke)),
                        "rel_max_difference": float(np.abs(Kc - Ke).max() / np.abs(Ke).max())}
    ctx.close()
    print("# coarse-matrix integration: " + json.dumps(integ), flush=True)
    v_cu, el_cu, st_cu, states_cu, cctx, _ = run(dev, s, params, a.warmup, a.steps, basis=basis,
                                                 cubature=(tets, w))
    print(f"# cubature coarse matrix: {v_cu:.3f} timesteps/s", flush=True)
    accuracy = None if a.no_accuracy else step_errors(dev, s, cctx, params, a.warmup, a.steps)[0]
    cctx.close()
    e_forms = float(np.linalg.norm(states_cu[-1] - states_ex[-1]) / np.linalg.norm(states_ex[-1] - s["x0"]))
    print(json.dumps({
        "workload": "cubature", "scene": f"heterogeneous block {a.grid}^3, 20 inclusions E=1e10 in E=1e5",
        "n_verts": len(s["rest"]), "n_tets": len(s["tets"]), "handles": a.handles, "precision": a.precision,
        "fit": {"points": int(len(tets)), "fraction_of_tets": len(tets) / len(s["tets"]), "seconds": fit_s,
                "worst_rel_moment_residual": worst, "tol": a.cub_tol, "n_init": a.cub_batch,
                "n_add": a.cub_batch, "threads": "all hardware threads of the host"},
        "basis_build_s": basis_s,
        "coarse_matrix_integration": integ,
        "steps": a.steps, "warmup": a.warmup,
        "exact_coarse": {"timesteps_per_s": v_ex, "pcg_iters": [st["pcg_iters"] for st in st_ex],
                         "newton_iters": [st["newton_iters"] for st in st_ex]},
        "cubature_coarse": {"timesteps_per_s": v_cu, "ms_per_step": 1e3 * el_cu / a.steps,
                            "pcg_iters": [st["pcg_iters"] for st in st_cu],
                            "newton_iters": [st["newton_iters"] for st in st_cu]},
        "e_rel_final_state_cubature_vs_exact_form": e_forms,
        "accuracy": accuracy}), flush=True)
    # paper mode: cubature subspace matrix vs exact integration, on a cube
    # with per-tet E over three decades and on a homogeneous one
    import torch
    for label, e_lo, e_hi in (("per-tet E log-uniform in [1e5, 1e8]", 1e5, 1e8), ("homogeneous E = 1e6", 1e6, 1e6)):
        sp_ = scenes.plain_cube(a.grid, seed=0, e_lo=e_lo, e_hi=e_hi, steps=a.warmup + a.steps)
        c = ms.context_from_scene(dev, sp_)
        c.ms_build_basis(n_handles=a.handles, oversample=a.oversample)
        t0 = time.perf_counter()
        worst_p = c.ms_build_cubature(tol=a.cub_tol, n_init=a.cub_batch, n_add=a.cub_batch, seed=0)
        fit_p = time.perf_counter() - t0
        npts = len(c.ms_get_cubature()[0])
        print(f"# paper-mode cube ({label}): cubature of {npts} tets in {fit_p:.1f} s", flush=True)
        # coarse matrices at the start state
        r = 12 * c.ms_get_basis()["m"]
        mats = {}
        for mode_name, mode in (("exact", ms.COARSE_EXACT), ("cubature", ms.COARSE_CUBATURE)):
            c.ms_set_coarse_integration(mode)
            c.ms_eval(sp_["x0"], sp_["dt"], prec=ms.PREC_FP64, hess=False)
            mats[mode_name] = c.ms_get_coarse_matrix(r)
        kdiff = float(np.linalg.norm(mats["cubature"] - mats["exact"]) / np.linalg.norm(mats["exact"]))
        pparams = ms.solver_defaults(mode=ms.MODE_PAPER, precision=prec, refine_iters=0, max_newton=100)
        times = {"exact": [], "cubature": []}
        errs, iters = [], []
        x, v = sp_["x0"].copy(), sp_["v0"].copy()
        for k in range(1, a.warmup + a.steps + 1):
            c.ms_set_dirichlet(sp_["dirichlet"], sp_["dbc_targets"](k))
            res = {}
            for mode_name, mode in (("exact", ms.COARSE_EXACT), ("cubature", ms.COARSE_CUBATURE)):
                c.ms_set_coarse_integration(mode)
                c.ms_set_state(x, v)
                dev.stream.synchronize()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = c.ms_step(sp_["dt"], pparams)
                dev.stream.synchronize()
                t1 = time.perf_counter()
                res[mode_name] = (c.ms_get_state(), st, t1 - t0)
            if k > a.warmup:
                for mname in times:
                    times[mname].append(res[mname][2])
                xe, xc = res["exact"][0][0], res["cubature"][0][0]
                errs.append(float(np.linalg.norm(xc - xe) / np.linalg.norm(xe - x)))
                iters.append((res["exact"][1]["newton_iters"], res["cubature"][1]["newton_iters"]))
            x, v = res["cubature"][0]
        c.close()
        print(json.dumps({
            "workload": "cubature", "scene": f"paper mode, cube {a.grid}^3, {label}",
            "n_tets": len(sp_["tets"]), "handles": a.handles, "precision": a.precision,
            "fit": {"points": npts, "fraction_of_tets": npts / len(sp_["tets"]), "seconds": fit_p,
                    "worst_rel_moment_residual": worst_p},
            "coarse_matrix_rel_frobenius_difference_at_rest": kdiff,
            "timesteps_per_s": {m: len(t) / sum(t) for m, t in times.items()},
            "newton_iters_exact_vs_cubature": iters,
            "e_rel_cubature_step_vs_exact_integration_step": errs,
            "note": "both steps start from the same state (the cubature trajectory)"}), flush=True)


def spmv_sweep_main(a):
    """The PCG product kernel (k_cg_spmv, fused with its dot partials) on the
    Hessian of the heterogeneous block at growing grid sizes: one Newton
    iteration of the first timestep assembles H, then the kernel is replayed
    back to back on it (--kernel-reps launches) in FP64 and in mixed storage.
    Beyond the last-level cache the launch is bound by HBM bandwidth."""
    import scenes
    from paper_2508_13386_amd import ms
    dev = ms.TorchDevice(0)
    reps = max(1, a.kernel_reps)
    for res in [int(v) for v in a.sweep.split(",") if v]:
        t0 = time.perf_counter()
        s = scenes.inclusion_block(res, seed=0, steps=1)
        if a.order != "natural":
            s = scenes.permute_vertices(s, scenes.vertex_order(s["rest"], s["tets"], a.order, seed=1))
        gen_s = time.perf_counter() - t0
        ctx = ms.context_from_scene(dev, s)
        ctx.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](1))
        x0, v0 = ctx.ms_get_state()
        for prec, name in ((ms.PREC_FP64, "fp64"), (ms.PREC_MIXED, "mixed")):
            ctx.ms_set_state(x0, v0)
            params = ms.solver_defaults(precision=prec, preconditioner=ms.PC_BLOCK_JACOBI, max_newton=1, max_pcg=4)
            try:
                ctx.ms_step(s["dt"], params)
            except ms.MSError as e:
                if e.code != ms.MS_E_NOCONV:
                    raise
            us, nbytes = ctx.ms_time_kernel(0, prec, reps)
            gbs = nbytes / us * 1e-3
            print(json.dumps({"workload": "spmv_sweep", "grid": res, "order": a.order, "vertices": len(s["rest"]),
                              "tets": len(s["tets"]), "storage": name, "kernel": "k_cg_spmv",
                              "algorithmic_bytes": nbytes, "avg_launch_us": us, "launches": reps,
                              "achieved_GBs": gbs, "frac_of_8TBs": gbs / HBM_PEAK_GBS,
                              "scene_gen_s": round(gen_s, 2)}), flush=True)
        ctx.close()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the multi-GPU layout is design-only.",
              file=sys.stderr)
        sys.exit(2)
    if a.copy_probe:
        copy_probe(a.copy_probe)
        return
    if a.trace_summary:
        trace_summary(a.trace_summary, a.work_us, a.tail, a.by_grid)
        return
    if a.workload == "batch64":
        batch_main(a)
        return
    if a.workload == "learned":
        learned_main(a)
        return
    if a.workload == "spmv_sweep":
        spmv_sweep_main(a)
        return
    if a.workload == "paper":
        paper_main(a)
        return
    if a.workload == "cubature":
        cubature_main(a)
        return
    import scenes
    from paper_2508_13386_amd import ms

    if a.scene == "stacked":
        s = scenes.stacked_cubes(N=a.grid, steps=a.warmup + a.steps)
        wname = (f"two cubes of {a.grid}^3 hexes x 6 tets (0.1 m and 0.08 m, E=1e5, nu=0.4), the upper one turned "
                 f"15 degrees and falling at 0.5 m/s onto the pinned lower one, IPC self-contact "
                 f"(point-triangle and edge-edge) d_hat=2e-3, dt=1/100")
    elif a.scene == "sliding":
        s = scenes.sliding_cube(a.grid, steps=a.warmup + a.steps)
        wname = (f"cube {a.grid}^3 hexes x 6 tets (0.2 m, E=1e6, nu=0.4) sliding at 1.1 m/s on a rigid half-space, "
                 f"IPC barrier d_hat=1e-3, lagged friction mu=0.5, eps_v=1e-3, dt=1/100")
    elif a.scene == "gyroid":
        s = scenes.gyroid_sphere(res=a.grid)
        wname = (f"gyroid-lattice sphere voxelized at {a.grid}^3 (E=1e7, nu=0.45) falling at 5 m/s onto a rigid "
                 f"half-space, IPC barrier d_hat=1e-3, dt=1/100")
    else:
        s = scenes.inclusion_block(a.grid, seed=0, steps=a.warmup + a.steps)
        wname = (f"heterogeneous block {a.grid}^3 hexes x 6 tets, 20 inclusions E=1e10 in E=1e5, "
                 f"nu=0.49, top driven 0.1 m over 10 steps, dt=1/60")
    x_start = s["x0"]
    dev = ms.TorchDevice(0)
    pc = {"jacobi": ms.PC_BLOCK_JACOBI, "two_level": ms.PC_TWO_LEVEL, "additive": ms.PC_TWO_LEVEL_ADDITIVE,
          "vcycle": ms.PC_TWO_LEVEL_VCYCLE}[a.pc]
    prec = ms.PREC_MIXED if a.precision == "mixed" else ms.PREC_FP64
    params = ms.solver_defaults(precision=prec, preconditioner=pc, forcing=1, pcg_eta_max=a.eta_max,
                                pcg_eta_min=a.eta_min, coarse_every=a.coarse_every, coarse_move=a.coarse_move,
                                max_newton=MAX_NEWTON,
                                mixed_endgame_fp64=a.endgame_fp64, endgame_ratio=a.endgame_ratio,
                                newton_tol=a.newton_tol, integrator=1 if a.integrator == "bdf2" else 0,
                                projection=1 if a.projection == "abs" else 0, smoother=a.smoother)
    value, elapsed, stats, states, ctx, basis_s = run(dev, s, params, a.warmup, a.steps,
                                                      handles=a.handles if pc != ms.PC_BLOCK_JACOBI else 0,
                                                      oversample=a.oversample, lattice=a.lattice, jump=a.jump,
                                                      rigid=a.rigid)
    # roofline of the dominant kernel, the PCG product fused with its dots:
    # one more timestep (outside the timed region) runs with every product
    # launch bracketed by HIP events on the library's stream, inside the real
    # PCG loop; the average over those launches is the kernel's duration.
    # These are the last product launches of the run.  In mixed precision
    # with the FP64 endgame both product instantiations run; the one that
    # ran more PCG iterations in the timed region is reported (a profile
    # picks its event-timed launches out as its last timed_step_pcg_iters_fp64
    # + timed_step_solves_fp64 dispatches for the FP64 instantiation, and the
    # remaining iterations and solves for the FP32 one).
    fp64_share = sum(st["pcg_iters_fp64"] for st in stats) / max(1, sum(st["pcg_iters"] for st in stats))
    kprec = ms.PREC_FP64 if fp64_share >= 0.5 else ms.PREC_MIXED
    # the kernel replayed back to back on the last Hessian (hot caches)
    r_us, _ = ctx.ms_time_kernel(0, kprec, a.kernel_reps)
    k = a.warmup + a.steps + 1
    ctx.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](k))
    tparams = ms.solver_defaults(precision=prec, preconditioner=pc, forcing=1, pcg_eta_max=a.eta_max,
                                 pcg_eta_min=a.eta_min, coarse_every=a.coarse_every, coarse_move=a.coarse_move,
                                 max_newton=MAX_NEWTON,
                                 mixed_endgame_fp64=a.endgame_fp64, endgame_ratio=a.endgame_ratio, time_kernels=1,
                                 newton_tol=a.newton_tol, integrator=1 if a.integrator == "bdf2" else 0,
                                 projection=1 if a.projection == "abs" else 0, smoother=a.smoother)
    tstat = ctx.ms_step(s["dt"], tparams)
    k_us, k_bytes = ctx.ms_time_kernel(0, kprec, 0)
    # slice height of the chosen layout, from the byte count of the product
    # (4 bytes per slice offset; the rest is fixed by nnzb and n)
    _, col = ctx.ms_get_pattern()
    n = len(s["rest"])
    vb = 8 if kprec == ms.PREC_FP64 else 4
    nslices = int(round((k_bytes - len(col) * (9 * vb + 4) - 73 * n) / 4)) - 1
    S = next(c for c in (16, 32, 64) if -(-n // c) == nslices)
    kernel_name = f"k_cg_spmv<{'double' if vb == 8 else 'float'}, {S}>"
    achieved = k_bytes / (k_us * 1e-6) / 1e9
    # the per-step check solves single steps from given states: implicit Euler only
    accuracy, check = (None, None) if (a.no_accuracy or a.integrator == "bdf2") else \
        step_errors(dev, s, ctx, params, a.warmup, a.steps)
    basis = ctx.ms_get_basis() if pc != ms.PC_BLOCK_JACOBI else None
    ctx.close()

    ref = None
    if not a.no_reference:
        pref = ms.solver_defaults(precision=ms.PREC_FP64, preconditioner=ms.PC_BLOCK_JACOBI, forcing=1,
                                  pcg_eta_max=a.eta_max, pcg_eta_min=a.eta_min, max_newton=MAX_NEWTON,
                                  integrator=1 if a.integrator == "bdf2" else 0)
        rv, _, rstats, rstates, rctx, _ = run(dev, s, pref, a.warmup, a.steps)
        rctx.close()
        xr, xg = rstates[-1], states[-1]
        e_rel = float(np.linalg.norm(xg - xr) / np.linalg.norm(xr - x_start))
        ref = {"form": "plain FP64 Newton-PCG, 3x3 block-Jacobi", "value": rv, "unit": "timesteps/s",
               "speedup": value / rv, "e_rel_final_state_vs_this_form": e_rel,
               "pcg_iters": [st["pcg_iters"] for st in rstats],
               "newton_iters": [st["newton_iters"] for st in rstats]}
        if basis is not None and prec == ms.PREC_MIXED:
            # the same preconditioner and policy in FP64 throughout, on the
            # same basis: isolates what the mixed-precision form gains
            p64 = ms.solver_defaults(precision=ms.PREC_FP64, preconditioner=pc, forcing=1, pcg_eta_max=a.eta_max,
                                     pcg_eta_min=a.eta_min, coarse_every=a.coarse_every, coarse_move=a.coarse_move,
                                     max_newton=MAX_NEWTON,
                                     integrator=1 if a.integrator == "bdf2" else 0, smoother=a.smoother)
            fv, _, fstats, fstates, fctx, _ = run(dev, s, p64, a.warmup, a.steps, basis=basis)
            fctx.close()
            ref["fp64_same_preconditioner"] = {
                "value": fv, "speedup_of_mixed": value / fv,
                "e_rel_final_state_vs_this_form": float(np.linalg.norm(xg - fstates[-1]) /
                                                        np.linalg.norm(fstates[-1] - x_start)),
                "pcg_iters": [st["pcg_iters"] for st in fstats]}

    out = {
        "metric": METRIC,
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
        "config": {"workload": wname,
                   "n_verts": int(len(s["rest"])), "n_tets": int(len(s["tets"])),
                   "precision": a.precision, "preconditioner": a.pc,
                   "handles": a.handles if pc != ms.PC_BLOCK_JACOBI else None, "pcg_eta_max": a.eta_max,
                   "coarse_every": a.coarse_every, "coarse_move": a.coarse_move, "endgame_fp64": a.endgame_fp64,
                   "smoother": ["3x3 vertex blocks", "vertex aggregates"][a.smoother],
                   "endgame_ratio": a.endgame_ratio, "pcg_eta_min": a.eta_min, "newton_tol": a.newton_tol,
                   "integrator": a.integrator, "projection": a.projection,
                   "basis": {"jump_penalty": a.jump, "oversample": a.oversample, "rigid_contrast": a.rigid},
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kernel_name, f"{a.scene}{a.grid}"),
                     "kernel": kernel_name + " (PCG product w = H u fused with its three dots, sliced BSR3)",
                     "bytes_per_launch": k_bytes, "avg_launch_us": k_us,
                     "timed_step_pcg_iters": int(tstat["pcg_iters"]),
                     "timed_step_pcg_iters_fp64": int(tstat["pcg_iters_fp64"]),
                     "timed_step_solves_fp64": int(tstat["pcg_solves_fp64"]),
                     "fp64_share_of_pcg_iters": fp64_share,
                     "timed_step_solves": int(tstat["newton_iters"]),
                     "replay_avg_launch_us": r_us,
                     "replay_frac": k_bytes / (r_us * 1e-6) / 1e9 / HBM_PEAK_GBS},
        "solver": {"pcg_us_per_iteration": 1e3 * sum(st["pcg_ms"] for st in stats) /
                   max(1, sum(st["pcg_iters"] for st in stats)),
                   "pcg_share_of_step": sum(st["pcg_ms"] for st in stats) / max(1e-9, 1e3 * elapsed),
                   "newton_iters": [st["newton_iters"] for st in stats],
                   "pcg_iters": [st["pcg_iters"] for st in stats],
                   "pcg_iters_fp64": [st["pcg_iters_fp64"] for st in stats],
                   "coarse_rebuilds": [st["hessian_refreshes"] for st in stats],
                   "precision_escalations": [st["precision_escalations"] for st in stats],
                   "basis_build_s": basis_s},
        "reference_form": ref,
        "accuracy": accuracy,
    }
    if not a.no_cpu_baseline:
        if a.scene == "block" and check is not None:
            out["cpu_baseline"], out["accuracy"]["oracle_check"] = cpu_baseline_on_workload(s, check)
        else:
            out["cpu_baseline"] = cpu_baseline(a.scene, a.grid, len(s["tets"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
