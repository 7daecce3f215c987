"""Writes the oracle reference solutions of the 3-D workloads (test
infrastructure; calls only the oracle, the seeded input generators and the
oracle's problem builder).

Every file holds what the oracle's FP64 GMRES(m) with the FP64 angular
multigrid V(1,1) preconditioner (coarse level: 10 Gauss-Seidel sweeps of
Section 5.2) gives for one workload: the iteration count to
||b - A x|| / ||b|| < 1e-8 (Section 5.1's criterion), the cell-average
scalar flux (all cells on the 16^3 grids, a seeded sample plus the source,
detector and beam boxes on the 32^3 grids), sums of the scalar flux per
x-plane, and for the beam workloads the detector response and its adjoint
gradient on the finite-difference cells.

    python tests/golden/make_goldens.py cfg2_32 cfg4_32 cfg3_16 cfg5_16

Each workload takes minutes to tens of minutes of host time.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from oracle import krylov, adjoint  # noqa: E402
from oracle_problem import OracleProblem  # noqa: E402
from paper_2010_04559_amd import inputs  # noqa: E402

WORKLOADS = {
    # 32^3 headline problem: lognormal medium, central source
    "cfg2_32": lambda: inputs.config2(32),
    # 32^3 beam problem with the detector (gradient workload)
    "cfg4_32": lambda: inputs.config4(32),
    # the precision problem's angular mesh (512 patches) and orders
    # (8, 8, 8, 32) on 16^3 cells: checkerboard of 8^3-cell blocks
    "cfg3_16": lambda: inputs.config3(16),
    # the cone mesh (368 patches, orders 4, 4, 4, 16, 16, 16 under L = 64)
    # on 16^3 cells with its beam and detector
    "cfg5_16": lambda: inputs.config5(16),
}


def sample_cells(prob, count=1024):
    """Seeded sample of cells plus every cell of the source, detector and beam
    boxes (sorted, unique)."""
    C = prob.cells
    cells = set(np.random.default_rng(12345).choice(C, min(count, C), replace=False).tolist())
    n = prob.n
    ix = lambda i, j, k: i + n[0] * (j + n[1] * k)
    cells.update(np.nonzero(prob.q_cell)[0].tolist())
    boxes = []
    if prob.detector is not None:
        boxes.append(prob.detector)
    if prob.inflow is not None:
        f = prob.inflow
        boxes.append(((0, f.lo[1], f.lo[2]), (3, f.hi[1], f.hi[2])))
    for lo, hi in boxes:
        for k in range(lo[2], hi[2] + 1):
            for j in range(lo[1], hi[1] + 1):
                for i in range(lo[0], hi[0] + 1):
                    cells.add(ix(i, j, k))
    return sorted(int(c) for c in cells)


def make(name):
    prob = WORKLOADS[name]()
    t0 = time.perf_counter()
    op = OracleProblem(prob)
    b = op.rhs()
    print(name, "setup %.1f s" % (time.perf_counter() - t0), flush=True)
    sol = krylov.gmres(op.outer.apply_A, op.mg.vcycle, b, prob.tol, prob.restart)
    print(name, "solve: %d iterations, rel_res %.3e, %.1f s" % (sol.iters, sol.rel_res, time.perf_counter() - t0),
          flush=True)
    phi = op.outer.scalar_flux_cell_avg(sol.x)
    n = prob.n
    out = {
        "workload": name, "problem": prob.name, "cells": prob.cells, "patches": [len(t) for t in op.T],
        "order": prob.order, "mg_orders": list(prob.mg_orders), "tol": prob.tol, "restart": prob.restart,
        "oracle_iters": sol.iters, "oracle_restarts": sol.restarts, "oracle_rel_res": sol.rel_res,
        "converged": bool(sol.converged),
        "phi_x_plane_sums": phi.reshape(n[2], n[1], n[0]).sum(axis=(0, 1)).tolist(),
        "phi_total": float(phi.sum()),
    }
    if prob.cells <= 4096:
        out["phi_cells"] = list(range(prob.cells))
        out["phi_cell_avg"] = phi.tolist()
    else:
        cells = sample_cells(prob)
        out["phi_cells"] = cells
        out["phi_cell_avg"] = phi[cells].tolist()
    if prob.detector is not None:
        w = op.detector()
        adj = adjoint.solve_adjoint(op.outer, op.mg, w, prob.tol, prob.restart)
        gt, gs = adjoint.gradients(op.outer, adj.x, sol.x)
        fd = [int(c) for c in prob.fd_cells]
        out.update({"response": float(w @ sol.x), "adjoint_iters": adj.iters, "grad_cells": fd,
                    "grad_sigma_t": gt[fd].tolist(), "grad_sigma_s": gs[fd].tolist(),
                    "grad_sigma_t_maxabs": float(np.abs(gt).max()), "grad_sigma_s_maxabs": float(np.abs(gs).max())})
        print(name, "adjoint: %d iterations" % adj.iters, flush=True)
    out["oracle_seconds"] = time.perf_counter() - t0
    out["generated_by"] = "tests/golden/make_goldens.py (oracle only)"
    path = os.path.join(HERE, "oracle_%s.json" % name)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    for arg in sys.argv[1:] or list(WORKLOADS):
        make(arg)
