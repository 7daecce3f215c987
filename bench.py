#!/usr/bin/env python3
"""Benchmark of the angular-multigrid transport solver on one MI355X.

Workload (default): the 48^3 precision problem -- unit cube, 48^3
trilinear DG cells, angular level 3 (512 patches x 3 ordinates = 1536
angular dofs, 1.36e9 DoFs), HG g = 0.98 at Legendre order 32, multigrid
levels at orders (8, 8, 8, 32), checkerboard of 8^3-cell blocks (sigma_t
1 / 20, c 0.999 / 0.9), central unit source, vacuum, GMRES(10) to
||b - A x|| / ||b|| < 1e-8, right-hand side already in HBM.

One step = one solve with the FP32 angular-multigrid preconditioner (FP32
sweeps, scatter products and transfers on levels >= 1, FP64 coarsest
level; V(1,6) cycle with one post-smoothing sweep on the levels between
and 5 coarsest-level sweeps on the 48^3 problem, --cycle to change it)
inside FP64 flexible GMRES: every transport sweep, scatter product,
transfer, coarse Gauss-Seidel sweep, precision cast and Krylov update of
the solve runs inside the timed region.  value = sweep DoF-updates per
second of the whole solve (sum over all transport sweeps of ordinates x
spatial dofs, divided by the solve's wall time).  The same problem solved
with the FP64 preconditioner (the plain FP64 solve) is timed beside it:
time-to-1e-8 of both, their iteration counts and the difference of the two
solutions are in the line.  The roofline objects come from HIP events
around every launch of the timed steps, on the library's stream.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg2|cfg3]
"""
import argparse
import hashlib
import json
import math
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3
BF16_PEAK_TFS = 2500.0  # dense BF16 MFMA
METRIC = "sweep DoF-updates/s; time-to-1e-8 residual, FP32-MG vs FP64 plain, 1 GPU"


def kernel_sources_digest():
    """Digest of the sweep kernels' sources (their sections of kernels.hip
    and the local solve header): a committed counter summary is used only
    while it matches."""
    with open(os.path.join(ROOT, "paper_2010_04559_amd", "csrc", "kernels.hip")) as fh:
        src = fh.read()
    beg = src.index("// ------------------------------------------------------------------ sweep")
    end = src.index("// ------------------------------------------------------- coarse Gauss-Seidel")
    h = hashlib.sha256(src[beg:end].encode())
    with open(os.path.join(ROOT, "paper_2010_04559_amd", "csrc", "local_solve.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel, digest):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this workload's sweep kernel, if it was taken on the current sources."""
    path = os.path.join(ROOT, "profiles", "sweep_%s_counters.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel") != kernel or d.get("sources_digest") != digest:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(prob, max_patches):
    """The oracle's transport sweep on a bounded sample of the same
    workload: the finest-level sweep of an evenly spaced subset of the
    patches (at most max_patches, every octant represented) on the full
    grid, FP64 numpy on the host."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import numpy as np
    from oracle import angular as ang, spatial as sp, transport as otr
    grid = sp.Grid(prob.dim, prob.n, prob.length)
    patches = ang.AngularMesh.uniform(prob.angular.base_level).leaves()
    step = max(1, len(patches) // max_patches)
    sample = patches[::step]
    lv = otr.Level(grid, sample, prob.sigma_t, prob.sigma_s, [1.0])
    g = np.random.default_rng(0).standard_normal(lv.A * grid.S)
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    lv.sweep(g)
    t1 = time.perf_counter()
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    dofs = lv.A * grid.S
    return {"value": dofs / (t1 - t0), "unit": "DoF-updates/s", "cores": max(1, round(cpu / (t1 - t0))),
            "kind": "oracle",
            "sample": "one oracle transport sweep (coupled %dx%d local solves) over %d of the %d patches (every %d-th, "
                      "all octants) on the %s grid: %d DoF-updates in %.1f s"
                      % (3 * grid.ns, 3 * grid.ns, len(sample), len(patches), step,
                         "x".join(str(v) for v in prob.n[:prob.dim]), dofs, t1 - t0)}


def oracle_timings(args):
    """Host timings of the oracle (the CPU baseline leg, extended): one sweep,
    one scatter application and one V-cycle of the finest level, and the full
    GMRES solve where it finishes in minutes (the 2-D problem), FP64 numpy
    with the host's BLAS threads."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import numpy as np
    from oracle import krylov
    from oracle_problem import OracleProblem
    from paper_2010_04559_amd import inputs

    def timed(fn, what=""):
        r0 = resource.getrusage(resource.RUSAGE_SELF)
        t0 = time.perf_counter()
        out = fn()
        t1 = time.perf_counter()
        r1 = resource.getrusage(resource.RUSAGE_SELF)
        cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
        print("oracle %s: %.2f s" % (what, t1 - t0), file=sys.stderr, flush=True)
        return out, t1 - t0, cpu / max(t1 - t0, 1e-9)

    res = {"host_cpus": os.cpu_count(), "rows": []}
    for name, prob, full in (("cfg1", inputs.config1(), True), ("cfg2", inputs.config2(), False)):
        op, t_setup, _ = timed(lambda: OracleProblem(prob), name + " setup")
        lv = op.outer
        rng = np.random.default_rng(0)
        x = rng.standard_normal(lv.A * lv.grid.S)
        dofs = lv.A * lv.grid.S
        row = {"workload": name, "dofs": dofs, "setup_s": t_setup}
        _, t, c = timed(lambda: lv.sweep(x), name + " sweep")
        row["sweep_s"], row["sweep_dof_per_s"], row["sweep_cores"] = t, dofs / t, c
        _, t, c = timed(lambda: lv.apply_S(x), name + " scatter")
        row["scatter_s"], row["scatter_cores"] = t, c
        _, t, c = timed(lambda: op.mg.vcycle(x), name + " V-cycle")
        row["vcycle_s"], row["vcycle_cores"] = t, c
        if full:
            b = op.rhs()
            sol, t, c = timed(lambda: krylov.gmres(lv.apply_A, op.mg.vcycle, b, prob.tol, prob.restart),
                              name + " solve")
            row["solve_s"], row["solve_iters"], row["solve_cores"] = t, sol.iters, c
        res["rows"].append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    return res


def _chunked_rel_diff(x, y, chunk=1 << 27):
    """|x - y| / |y| (2-norm) and max|x - y| / max|y| without full-size
    temporaries."""
    import torch
    n = x.numel()
    d2 = y2 = 0.0
    dm = ym = 0.0
    for i in range(0, n, chunk):
        xa, ya = x[i:i + chunk], y[i:i + chunk]
        t = xa - ya
        d2 += float(torch.dot(t, t))
        y2 += float(torch.dot(ya, ya))
        dm = max(dm, float(t.abs().max()))
        ym = max(ym, float(ya.abs().max()))
        del t
    return math.sqrt(d2 / y2), dm / ym


def _timed_solves(tr, b, mode, steps, warmup, label):
    """Warm-up solves, then `steps` timed solves with HIP events around every
    launch (component and kernel times over the timed region)."""
    import torch
    for _ in range(warmup):
        x, st = tr.solve(b, mode=mode)
        del x
    torch.cuda.synchronize()
    acc = {}
    t0 = time.perf_counter()
    for i in range(steps):
        x, st = tr.solve(b, mode=mode, timing=True)
        for k, v in st.items():
            if k.startswith("ms_") or k.startswith("n_") or k == "coarse_steps":
                acc[k] = acc.get(k, 0) + v
        print("%s step %d: iters %d rel_res %.2e %.1f ms" % (label, i, st["iters"], st["rel_res"], st["ms_total"]),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    return x, st, ms, acc


def headline(args):
    import torch
    from paper_2010_04559_amd import inputs
    from paper_2010_04559_amd.transport import Transport
    make = {"cfg2": inputs.config2, "cfg3": inputs.config3}[args.workload]
    prob = make()
    # the V-cycle of the timed solves (FP32-MG and FP64 alike)
    if args.cycle != "problem":
        cyc = inputs.CFG3_CYCLE if args.cycle == "auto" and args.workload == "cfg3" else (
            (prob.nu_pre, prob.nu_post, prob.nu_coarse, prob.nu_post_coarse) if args.cycle == "auto" else
            tuple(int(v) for v in args.cycle.split(",")))
        if len(cyc) == 3:
            cyc = cyc + (0,)
        prob.nu_pre, prob.nu_post, prob.nu_coarse, prob.nu_post_coarse = cyc
    t_setup = time.perf_counter()
    tr = Transport(prob)
    b = tr.rhs()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    free, total = torch.cuda.mem_get_info()
    print("setup %.1f s, patches %s, S=%d, scatter forms %s, device memory %.1f of %.1f GB free"
          % (t_setup, tr.patches, tr.S, tr.scatter_forms, free / 1e9, total / 1e9), file=sys.stderr, flush=True)
    L = tr.nlev - 1
    A = 3 * tr.patches[L]
    dofs = A * tr.S

    # the step: FP32 angular-MG preconditioner inside FP64 flexible GMRES
    xm, stm, ms_step, accm = _timed_solves(tr, b, "mixed", args.steps, args.warmup, "fp32-mg")
    value = stm["sweep_dof_updates"] / (ms_step * 1e-3)
    # the plain FP64 solve of the same problem
    reps64 = max(1, min(args.steps, args.fp64_steps))
    x64, st64, ms64, acc64 = _timed_solves(tr, b, "f64", reps64, 1, "fp64")
    rel2, relmax = _chunked_rel_diff(xm, x64)
    del xm
    torch.cuda.empty_cache()
    # the same FP32 preconditioner with its scatter products formed from
    # split-BF16 operands (three BF16 matrix-core products, FP32 accumulate)
    xb, stb, msb, accb = _timed_solves(tr, b, "mixed_bf16", reps64, 1, "fp32-mg-split-bf16")
    relb2, relbmax = _chunked_rel_diff(xb, x64)
    del xb
    free, _ = torch.cuda.mem_get_info()
    print("after solves: %.1f GB free" % (free / 1e9), file=sys.stderr, flush=True)

    def per_solve(acc, n):
        return {k[3:]: round(v / n, 3) for k, v in acc.items() if k.startswith("ms_")}

    # dominant kernels of the step, from the events around every launch of
    # the timed region: the finest-level FP32 sweep (HBM) and the scatter
    # products (matrix cores)
    ms_sw = accm["ms_sweep_finest"] / accm["n_sweep_finest"]
    sweep_bytes = dofs * 8  # FP32: read the right-hand side + write the solution, 4 B each
    achieved = sweep_bytes / (ms_sw * 1e-3) / 1e9
    digest = kernel_sources_digest()
    sweep_kernel = tr.sweep_kernel_name(L, "f32")
    traffic = measured_traffic(args.workload, sweep_kernel, digest)
    ms_outer = accm["ms_scatter_outer"] / accm["n_scatter_outer"]
    # the finest multigrid level's FP32 scatter products (the solve's
    # largest kernel time with the benchmark cycle)
    ms_mg = accm["ms_scatter_finest"] / max(1, accm["n_scatter_finest"])
    fl_mg = tr.scatter_flops(L)
    tf_mg = fl_mg / (ms_mg * 1e-3) / 1e12 if accm["n_scatter_finest"] else 0.0
    fl_outer = tr.scatter_flops(L, outer=True)
    tf_outer = fl_outer / (ms_outer * 1e-3) / 1e12
    # back-to-back launches of single kernels (the same kernels, outside a solve)
    ms_sw64 = tr.time_sweep_kernel(L, "f64", reps=5)
    ms_sw32 = tr.time_sweep_kernel(L, "f32", reps=5)
    ms_g32 = tr.time_scatter_kernel(L, outer=False, prec="f32", reps=5)
    ms_gb = tr.time_scatter_kernel(L, outer=False, prec="bf16x3", reps=5)
    fl_lv = tr.scatter_flops(L)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "DoF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": prob.name + ": " + (make.__doc__ or "").strip().replace("\n", " "),
                   "cells": tr.C, "spatial_dofs": tr.S, "angular_dofs": A, "dofs": dofs,
                   "step": "one solve to 1e-8: FP64 flexible GMRES(%d) + FP32 angular MG V(%d,%d) (post-smoothing %d "
                           "on the levels between), FP64 coarsest level (%d Gauss-Seidel sweeps)"
                           % (prob.restart, prob.nu_pre, prob.nu_post, prob.nu_post_coarse or prob.nu_post,
                              prob.nu_coarse),
                   "parallelism": "single GPU"},
        "time_to_tol_ms": {"fp32_mg": ms_step, "fp64_plain": ms64, "fp64_over_fp32_mg": ms64 / ms_step,
                           "fp32_mg_split_bf16": msb, "fp64_over_fp32_mg_split_bf16": ms64 / msb},
        "iters": {"fp32_mg": stm["iters"], "fp64_plain": st64["iters"], "fp32_mg_split_bf16": stb["iters"]},
        "explicit_rel_res": {"fp32_mg": stm["rel_res"], "fp64_plain": st64["rel_res"],
                             "fp32_mg_split_bf16": stb["rel_res"]},
        "fp32_mg_vs_fp64_solution": {"rel_l2": rel2, "rel_max": relmax},
        "fp32_mg_split_bf16_vs_fp64_solution": {"rel_l2": relb2, "rel_max": relbmax},
        "sweep_dof_updates_per_s": {"fp32_mg": value, "fp64_plain": st64["sweep_dof_updates"] / (ms64 * 1e-3),
                                    "fp32_mg_split_bf16": stb["sweep_dof_updates"] / (msb * 1e-3)},
        "breakdown_ms_per_solve": {"fp32_mg": per_solve(accm, args.steps), "fp64_plain": per_solve(acc64, reps64),
                                   "fp32_mg_split_bf16": per_solve(accb, reps64)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": sweep_kernel + " (finest-level FP32 transport sweep)",
                     "ms_per_launch": ms_sw, "launches": accm["n_sweep_finest"], "bytes_per_launch": sweep_bytes},
        "roofline_scatter": {"bound": "mfma", "achieved": tf_outer, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                             "frac": tf_outer / FP64_PEAK_TFS,
                             "kernel": "problem-operator scatter, FP64 %s form" % ("octant-block" if tr.outer_axes
                                                                                  else "dense"),
                             "ms_per_launch": ms_outer, "launches": accm["n_scatter_outer"],
                             "flop_per_launch": fl_outer,
                             "dense_equivalent_tflops": 2.0 * A * A * tr.S / (ms_outer * 1e-3) / 1e12},
        "roofline_scatter_mg": {"bound": "mfma", "achieved": tf_mg, "peak": FP32_PEAK_TFS, "unit": "TFLOP/s",
                                "frac": tf_mg / FP32_PEAK_TFS,
                                "kernel": "finest multigrid level's scatter, FP32 %s form"
                                          % ("octant-block" if tr.scatter_forms[L][0] == "octant"
                                             else tr.scatter_forms[L][0]),
                                "ms_per_launch": ms_mg, "launches": accm["n_scatter_finest"],
                                "flop_per_launch": fl_mg},
        "kernels_back_to_back": {
            "sweep_f64_ms": ms_sw64, "sweep_f64_dof_per_s": dofs / (ms_sw64 * 1e-3),
            "sweep_f64_hbm_frac": dofs * 16 / (ms_sw64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "sweep_f32_ms": ms_sw32, "sweep_f32_dof_per_s": dofs / (ms_sw32 * 1e-3),
            "sweep_f32_hbm_frac": dofs * 8 / (ms_sw32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "scatter_f32_finest_ms": ms_g32, "scatter_f32_finest_tflops": fl_lv / (ms_g32 * 1e-3) / 1e12,
            "scatter_f32_finest_frac": fl_lv / (ms_g32 * 1e-3) / 1e12 / FP32_PEAK_TFS,
            "scatter_split_bf16_finest_ms": ms_gb,
            "scatter_split_bf16_finest_tflops": 3 * fl_lv / (ms_gb * 1e-3) / 1e12,
            "scatter_split_bf16_finest_frac": 3 * fl_lv / (ms_gb * 1e-3) / 1e12 / BF16_PEAK_TFS},
        "scatter_forms": [list(f) for f in tr.scatter_forms],
        "coarse_gs": coarse_gs_line(accm, args.steps),
        "setup_s": t_setup,
    }
    del x64, b
    tr.close()
    torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_patches)
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=3, help="timed FP64-preconditioned solves (at most --steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-patches", type=int, default=64, help="patches in the oracle sweep sample")
    ap.add_argument("--workload", default="cfg3", choices=["cfg1", "cfg2", "cfg3", "cfg4", "cfg5"],
                    help="cfg3 (default, the 48^3 precision problem) and cfg2 (32^3) print the benchmark line; "
                         "the others a measurement line of their own (2-D square, 32^3 beam gradient, cone mesh)")
    ap.add_argument("--fd-cells", type=int, default=6, help="finite-difference cells for cfg4/cfg5")
    ap.add_argument("--cycle", default="auto",
                    help="V-cycle of the timed solves as PRE,POST,COARSE[,POST_BETWEEN] sweeps; 'auto': the "
                         "measured choice for cfg3 (inputs.CFG3_CYCLE), the problem's own otherwise; 'problem': "
                         "the problem's own")
    ap.add_argument("--oracle-timings", action="store_true",
                    help="only time the oracle on the host (sweep, scatter and V-cycle of the 2-D and 32^3 "
                         "problems, full solve of the 2-D problem)")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only launch the kernels whose hardware counters are recorded: a 1 GiB device copy "
                         "(counter calibration), then the finest-level sweeps and scatter products of the workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (the multi-GPU angular sharding is a design "
              "note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.oracle_timings:
        print(json.dumps(oracle_timings(args)))
        return
    if args.profile_kernels:
        print(json.dumps(profile_kernels(args)))
        return
    if args.workload not in ("cfg2", "cfg3"):
        print(json.dumps(other_workload(args)))
        return
    print(json.dumps(headline(args)))


def coarse_gs_line(acc, steps):
    """Latency figures of the coarsest-level Gauss-Seidel solve: time per
    solve and per dependent step of its schedule."""
    if not acc.get("n_coarse") or not acc.get("coarse_steps"):
        return None
    ms = acc["ms_coarse"] / acc["n_coarse"]
    nsteps = acc["coarse_steps"] / steps
    return {"ms_per_solve": ms, "dependent_steps": nsteps, "us_per_step": 1e3 * ms / nsteps}


def profile_kernels(args):
    """A short program for rocprofv3 counter passes (see --profile-kernels)."""
    import torch
    from paper_2010_04559_amd import inputs
    from paper_2010_04559_amd.transport import Transport
    n_copy = 1 << 27
    src = torch.ones(n_copy, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print("copy of %d bytes done" % (8 * n_copy), file=sys.stderr, flush=True)
    del src, dst
    prob = {"cfg2": inputs.config2, "cfg3": inputs.config3}.get(args.workload, inputs.config3)()
    tr = Transport(prob)
    L = tr.nlev - 1
    out = {"copy_bytes": 8 * n_copy, "workload": prob.name, "dofs": 3 * tr.patches[L] * tr.S,
           "sweep_f64_ms": tr.time_sweep_kernel(L, "f64", reps=3),
           "sweep_f32_ms": tr.time_sweep_kernel(L, "f32", reps=3),
           "scatter_outer_f64_ms": tr.time_scatter_kernel(L, outer=True, prec="f64", reps=2),
           "scatter_f32_ms": tr.time_scatter_kernel(L, outer=False, prec="f32", reps=2),
           "sweep_kernel_f32": tr.sweep_kernel_name(L, "f32"), "sources_digest": kernel_sources_digest()}
    torch.cuda.synchronize()
    tr.close()
    return out


def _solve_timed(tr, b, mode, steps, warmup):
    import torch
    for _ in range(warmup):
        x, st = tr.solve(b, mode=mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x, st = tr.solve(b, mode=mode)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    return x, st, ms


def other_workload(args):
    """Measurements of the other problem configurations (not the headline)."""
    import numpy as np
    import torch
    from paper_2010_04559_amd import inputs
    from paper_2010_04559_amd.transport import Transport
    make = {"cfg1": inputs.config1, "cfg3": inputs.config3, "cfg4": inputs.config4, "cfg5": inputs.config5}
    prob = make[args.workload]()
    t_setup = time.perf_counter()
    tr = Transport(prob)
    b = tr.rhs()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    print("%s setup %.1f s, patches %s, S=%d" % (prob.name, t_setup, tr.patches, tr.S), file=sys.stderr, flush=True)
    out = {"workload": prob.name, "patches": tr.patches, "spatial_dofs": tr.S,
           "dofs": 3 * tr.patches[-1] * tr.S, "setup_s": t_setup, "solves": {}}
    modes = ["f64", "mixed", "mixed_bf16"]
    xs = {}
    for mode in modes:
        x, st, ms = _solve_timed(tr, b, mode, args.steps, args.warmup)
        r = b - tr.apply(x)
        xs[mode] = x
        out["solves"][mode] = {"ms": ms, "iters": st["iters"], "rel_res": st["rel_res"],
                               "explicit_rel_res": float(torch.linalg.norm(r) / torch.linalg.norm(b)),
                               "sweep_dof_updates_per_s": st["sweep_dof_updates"] / (ms * 1e-3)}
        print(mode, out["solves"][mode], file=sys.stderr, flush=True)
    out["mixed_vs_fp64_rel_diff"] = float(torch.linalg.norm(xs["mixed"] - xs["f64"]) / torch.linalg.norm(xs["f64"]))
    out["mixed_bf16_vs_fp64_rel_diff"] = float(torch.linalg.norm(xs["mixed_bf16"] - xs["f64"]) /
                                               torch.linalg.norm(xs["f64"]))
    _, stt = tr.solve(b, timing=True)
    out["breakdown_ms_fp64"] = {k: round(stt[k], 3) for k in ("ms_total", "ms_sweep", "ms_scatter", "ms_transfer",
                                                              "ms_coarse", "ms_apply", "ms_orth", "ms_other")}
    if prob.detector is not None:
        w = tr.detector()
        x = xs["f64"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gt, gs, lam, sta = tr.adjoint_grad(w, x, mode="mixed")
        torch.cuda.synchronize()
        out["adjoint"] = {"ms": (time.perf_counter() - t0) * 1e3, "iters": sta["iters"], "rel_res": sta["rel_res"],
                          "reciprocity_rel": abs(float(torch.dot(w, x)) - float(torch.dot(lam, b)))
                          / abs(float(torch.dot(w, x)))}
        # central differences (h = 1e-6 relative) on seeded cells, solves to 1e-13
        gt13, gs13, _, _ = tr.adjoint_grad(w, tr.solve(b, tol=1e-13, mode="mixed")[0], tol=1e-13, mode="mixed")
        gt13, gs13 = gt13.cpu().numpy(), gs13.cpu().numpy()
        errs = []
        cells = list(prob.fd_cells[:args.fd_cells])
        st0, ss0 = prob.sigma_t.copy(), prob.sigma_s.copy()
        for j in cells:
            for which in ("t", "s"):
                base = (st0 if which == "t" else ss0)[j]
                h = 1e-6 * base
                vals = []
                for sgn in (1, -1):
                    st_, ss_ = st0.copy(), ss0.copy()
                    (st_ if which == "t" else ss_)[j] = base + sgn * h
                    tr.set_sigma(st_, ss_)
                    xs_, _ = tr.solve(b, tol=1e-13, mode="mixed")
                    vals.append(float(torch.dot(w, xs_)))
                fd = (vals[0] - vals[1]) / (2 * h)
                ref = gt13 if which == "t" else gs13
                errs.append(abs(fd - ref[j]) / np.abs(ref).max())
            print("fd cell", j, errs[-2:], file=sys.stderr, flush=True)
        tr.set_sigma(st0, ss0)
        out["fd_check"] = {"cells": [int(c) for c in cells], "max_err_rel_to_max_grad": max(errs),
                           "h_rel": 1e-6, "solve_tol": 1e-13}
    return out


if __name__ == "__main__":
    main()
