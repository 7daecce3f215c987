#!/usr/bin/env python3
"""Benchmark of the angular-multigrid transport solver on one MI355X.

One step = one full solve of the 3-D heterogeneous problem (unit cube,
32^3 trilinear DG cells, angular level 2 = 128 patches x 3 ordinates, HG
g = 0.95 at Legendre order 16, lognormal sigma_t, c = 0.98, central unit
source, vacuum) to ||b - A x|| / ||b|| < 1e-8 with FP64 GMRES(10) and the
FP64 angular-multigrid V(1,1) preconditioner, right-hand side already in HBM.
Every transport sweep, scatter GEMM, transfer, coarse Gauss-Seidel sweep and
Krylov update of the solve runs inside the timed region.

value = sweep DoF-updates per second of the whole solve: the sum over all
transport sweeps of (ordinates x spatial dofs), divided by the solve's wall
time.  Also reported: the same solve with the FP32 V-cycle, the component
breakdown, and the roofline of the finest-level sweep kernel measured with
HIP events on the library's stream.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
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


def kernel_sources_digest():
    """Digest of the sources of the LDS sweep kernel (its section of
    kernels.hip and the local solve header): the committed counter summary
    is used only while it matches."""
    with open(os.path.join(ROOT, "paper_2010_04559_amd", "csrc", "kernels.hip")) as fh:
        src = fh.read()
    beg = src.index("// ------------------------------------------------------------ LDS sweep")
    end = src.index("// ------------------------------------------------------- coarse Gauss-Seidel")
    h = hashlib.sha256(src[beg:end].encode())
    with open(os.path.join(ROOT, "paper_2010_04559_amd", "csrc", "local_solve.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, digest):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "sweep_fp64_cfg2_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel") != kernel or d.get("sources_digest") != digest:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(prob):
    """The oracle's transport sweep on a bounded sample of the same workload:
    one whole finest-level sweep (all 128 patches) on the 32^3 grid, FP64
    numpy on the host."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import numpy as np
    from oracle import angular as ang, spatial as sp, transport as otr
    grid = sp.Grid(prob.dim, prob.n, prob.length)
    patches = ang.AngularMesh.uniform(prob.angular.base_level).leaves()
    lv = otr.Level(grid, patches, prob.sigma_t, prob.sigma_s, [1.0])
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
            "sample": "one oracle transport sweep (coupled 24x24 local solves) over all %d patches on the "
                      "%d^3 grid: %d DoF-updates in %.1f s" % (len(patches), prob.n[0], dofs, t1 - t0)}


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
    for name, prob, full in (("cfg1", inputs.config1(), True), ("cfg2", inputs.config2(args.n), False)):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32, help="cells per axis")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--workload", default="cfg2", choices=["cfg1", "cfg2", "cfg3", "cfg4", "cfg5"],
                    help="cfg2 (default) is the headline line; the others print a measurement line of "
                         "their own (2-D square, 48^3 precision study, 32^3 beam gradient, cone mesh)")
    ap.add_argument("--fd-cells", type=int, default=6, help="finite-difference cells for cfg4/cfg5")
    ap.add_argument("--oracle-timings", action="store_true",
                    help="only time the oracle on the host (sweep, scatter and V-cycle of the 2-D and 32^3 "
                         "problems, full solve of the 2-D problem)")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only launch the kernels whose hardware counters are recorded: a 1 GiB device copy "
                         "(counter calibration), then the finest-level FP64 and FP32 sweeps (3 launches each) "
                         "and FP64 scatter GEMMs (2 launches) of the headline problem")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the multi-GPU angular sharding is a design "
              "note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.oracle_timings:
        print(json.dumps(oracle_timings(args)))
        return
    import torch
    from paper_2010_04559_amd import inputs
    from paper_2010_04559_amd.transport import Transport

    if args.profile_kernels:
        print(json.dumps(profile_kernels(args)))
        return
    if args.workload != "cfg2":
        print(json.dumps(other_workload(args)))
        return
    prob = inputs.config2(args.n)
    t_setup = time.perf_counter()
    tr = Transport(prob)
    b = tr.rhs()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    print("setup %.1f s, patches %s, S=%d" % (t_setup, tr.patches, tr.S), file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        x, st = tr.solve(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        x, st = tr.solve(b)
        print("step %d: iters %d rel_res %.2e" % (i, st["iters"], st["rel_res"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) / args.steps * 1e3
    value = st["sweep_dof_updates"] / (ms_step * 1e-3)

    # explicit residual check of the last solve through the library's operator
    r = b - tr.apply(x)
    rel_res = float(torch.linalg.norm(r) / torch.linalg.norm(b))

    # FP32 V-cycle inside FP64 GMRES
    mixed = None
    if not args.no_mixed:
        xm, stm = tr.solve(b, mode="mixed")
        torch.cuda.synchronize()
        tm0 = time.perf_counter()
        for _ in range(args.steps):
            xm, stm = tr.solve(b, mode="mixed")
        torch.cuda.synchronize()
        ms_mixed = (time.perf_counter() - tm0) / args.steps * 1e3
        dx = float(torch.linalg.norm(xm - x) / torch.linalg.norm(x))
        mixed = {"ms": ms_mixed, "iters": stm["iters"], "rel_res": stm["rel_res"], "rel_diff_vs_fp64": dx}
        print("mixed: %.1f ms, iters %d" % (ms_mixed, stm["iters"]), file=sys.stderr, flush=True)
        # the same V-cycle with split-BF16 scatter products; used only where
        # its iteration count equals the FP32 one
        xs, sts = tr.solve(b, mode="mixed_bf16")
        torch.cuda.synchronize()
        tm0 = time.perf_counter()
        for _ in range(args.steps):
            xs, sts = tr.solve(b, mode="mixed_bf16")
        torch.cuda.synchronize()
        ms_split = (time.perf_counter() - tm0) / args.steps * 1e3
        mixed["split_bf16"] = {"ms": ms_split, "iters": sts["iters"], "rel_res": sts["rel_res"],
                               "rel_diff_vs_fp64": float(torch.linalg.norm(xs - x) / torch.linalg.norm(x)),
                               "same_iterations_as_fp32": sts["iters"] == stm["iters"]}
        print("mixed split-bf16: %.1f ms, iters %d" % (ms_split, sts["iters"]), file=sys.stderr, flush=True)

    # component breakdown (HIP events around every launch group)
    _, stt = tr.solve(b, timing=True)
    breakdown = {k: round(stt[k], 3) for k in ("ms_total", "ms_sweep", "ms_scatter", "ms_transfer", "ms_coarse",
                                               "ms_apply", "ms_orth", "ms_other")}

    # roofline of the finest-level FP64 sweep kernel: algorithmic bytes per
    # DoF-update = 16 (read the right-hand side, write the solution)
    L = tr.nlev - 1
    dofs = 3 * tr.patches[L] * tr.S
    ms_sweep = tr.time_sweep_kernel(L, "f64", reps=20)
    achieved = dofs * 16 / (ms_sweep * 1e-3) / 1e9
    digest = kernel_sources_digest()
    traffic = measured_traffic("k_sweep_lds<double,3,false,false,true,true>", digest)
    ms_sweep32 = tr.time_sweep_kernel(L, "f32", reps=20)
    ms_gemm = tr.time_scatter_kernel(L, outer=False, prec="f64", reps=10)
    A = 3 * tr.patches[L]
    gemm_tfs = 2.0 * A * A * tr.S / (ms_gemm * 1e-3) / 1e12
    ms_gemm32 = tr.time_scatter_kernel(L, outer=False, prec="f32", reps=10)
    gemm32_tfs = 2.0 * A * A * tr.S / (ms_gemm32 * 1e-3) / 1e12
    ms_gemm16 = tr.time_scatter_kernel(L, outer=False, prec="bf16x3", reps=10)
    gemm16_tfs = 2.0 * A * A * tr.S / (ms_gemm16 * 1e-3) / 1e12

    line = {
        "metric": "sweep DoF-updates/s; time-to-1e-8 residual, FP32-MG vs FP64 plain, 1 GPU",
        "value": value,
        "unit": "DoF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3-D unit cube %d^3 trilinear DG, angular level 2 (128 patches x 3), HG g=0.95 "
                               "L=16, lognormal sigma_t (median 5, log-sd 1, seed 0), c=0.98, central 4^3 unit "
                               "source, vacuum; GMRES(10) + FP64 angular MG V(1,1), tol 1e-8" % args.n,
                   "cells": tr.C, "spatial_dofs": tr.S, "angular_dofs": A, "dofs": dofs,
                   "parallelism": "single GPU"},
        "time_to_tol_ms": {"fp64_plain": ms_step, "fp32_mg": mixed["ms"] if mixed else None,
                           "fp32_mg_split_bf16": mixed["split_bf16"]["ms"] if mixed else None},
        "iters": {"fp64_plain": st["iters"], "fp32_mg": mixed["iters"] if mixed else None,
                  "fp32_mg_split_bf16": mixed["split_bf16"]["iters"] if mixed else None},
        "explicit_rel_res": rel_res,
        "mixed": mixed,
        "breakdown_ms": breakdown,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_sweep_lds<double,3,false,false,true,true> (finest-level FP64 transport sweep)",
                     "ms_per_launch": ms_sweep, "bytes_per_launch": dofs * 16},
        "sweep_kernel": {"fp64_dof_per_s": dofs / (ms_sweep * 1e-3), "fp32_dof_per_s": dofs / (ms_sweep32 * 1e-3),
                         "fp32_ms": ms_sweep32},
        "scatter_gemm": {"fp64_ms": ms_gemm, "fp64_tflops": gemm_tfs, "fp64_frac": gemm_tfs / FP64_PEAK_TFS,
                         "fp32_ms": ms_gemm32, "fp32_tflops": gemm32_tfs, "fp32_frac": gemm32_tfs / FP32_PEAK_TFS,
                         "split_bf16_ms": ms_gemm16, "split_bf16_tflops_fp32_equiv": gemm16_tfs,
                         "split_bf16_mfma_frac": 3 * gemm16_tfs / BF16_PEAK_TFS},
        "coarse_gs": coarse_gs_line(stt),
        "setup_s": t_setup,
    }
    if not args.no_cpu_baseline:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(line))


def coarse_gs_line(stt):
    """Latency figures of the coarsest-level Gauss-Seidel solve: time per
    solve and per dependent step of its step schedule."""
    if not stt["n_coarse"] or not stt["coarse_steps"]:
        return None
    ms = stt["ms_coarse"] / stt["n_coarse"]
    return {"ms_per_solve": ms, "dependent_steps": stt["coarse_steps"],
            "us_per_step": 1e3 * ms / stt["coarse_steps"]}


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
    prob = inputs.config2(args.n)
    tr = Transport(prob)
    L = tr.nlev - 1
    out = {"copy_bytes": 8 * n_copy, "dofs": 3 * tr.patches[L] * tr.S,
           "sweep_f64_ms": tr.time_sweep_kernel(L, "f64", reps=3),
           "sweep_f32_ms": tr.time_sweep_kernel(L, "f32", reps=3),
           "gemm_f64_ms": tr.time_scatter_kernel(L, outer=False, prec="f64", reps=2)}
    torch.cuda.synchronize()
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
