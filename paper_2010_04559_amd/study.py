"""The paper's Section 5 studies on the 5 cm cube, run through the library.

Every case is a BiCGStab solve (Section 3's outer solver) to
||r|| / ||b|| < 1e-8 of ``inputs.paper_box`` (Fokker-Planck-equivalent
moments of order N, transport cross section 1, no absorption), with either
the single-grid sweep preconditioner (SG: one transport sweep per
application) or the angular multigrid V(nu_pre, nu_post) cycle:

* ``table1``: Section 5.1 (Table 1, Lin or Const basis): uniform angular levels
  1-3, N = 4, 8, 16, SG and V(1,1) / V(2,1) with the coarse order N_r on
  the coarsest level only and an accurate coarse solve (``--nu-coarse``
  Gauss-Seidel sweeps; the paper solved it to 1e-5);
* ``nr``: Section 5.3 (figure of the N_r effect): level 3, N_r on every
  preconditioner level, 10 coarse sweeps, V(1,0) and V(1,1), N_r from 1 to
  N (a subset, with the optimal value);
* ``final``: Section 5.4: SG against V(1,0) and V(1,1) with the optimal
  N_r of Section 5.3 (2, 4, 6, 7, 8, 9 for N = 4 .. 24);
* ``beam``: Section 5.5: the z pencil beam on the z-band meshes
  l_max = 1 .. 6, SG against V(1,0) and V(1,1) with the optimal N_r.

One JSON object per solve goes to stdout (iterations, wall time of the
solve with the right-hand side already on the device, DoFs), then a
markdown table of the study.

    python -m paper_2010_04559_amd.study table1 [--n 30] [--N 4,8,16]
"""
import argparse
import json
import math
import sys
import time

from . import inputs
from .transport import Transport

# Section 5.3's optimal multigrid scatter orders
OPTIMAL_NR = {4: 2, 8: 4, 12: 6, 16: 7, 20: 8, 24: 9}


def _torch():
    import torch
    return torch


def solve_case(prob, mode, tol=1e-8, max_iters=2000, method="bicgstab"):
    """Set up ``prob``, solve once, return iterations and timings."""
    torch = _torch()
    t0 = time.perf_counter()
    tr = Transport(prob)
    try:
        t_setup = time.perf_counter() - t0
        b = tr.rhs()
        restart = prob.restart
        max_restarts = max(0, math.ceil(max_iters / restart) - 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = tr.solve(b, tol=tol, mode=mode, method=method, max_restarts=max_restarts, check=False)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0
        return {"case": prob.name, "mode": mode, "method": method, "iters": st["iters"],
                "converged": bool(st["converged"]), "rel_res": st["rel_res"], "solve_s": round(t_solve, 4),
                "setup_s": round(t_setup, 3), "patches": tr.patches[-1], "levels": tr.nlev,
                "dofs": (3 if prob.angular.basis == "lin" else 1) * tr.patches[-1] * prob.cells * 8,
                "basis": prob.angular.basis, "mg_orders": list(prob.mg_orders),
                "nu": [prob.nu_pre, prob.nu_post, prob.nu_coarse]}
    finally:
        tr.close()
        del tr
        torch.cuda.empty_cache()


def _emit(rec, out):
    print(json.dumps(rec), flush=True)
    out.append(rec)


def table1(n=30, levels=(1, 2, 3), Ns=(4, 8, 16), nrs=(0, 1, 2, 3), nu_coarse=40, basis="lin", out=None):
    out = [] if out is None else out
    for lev in levels:
        for N in Ns:
            p = inputs.paper_box(N, level=lev, n=n, nu_coarse=nu_coarse, basis=basis)
            _emit(dict(solve_case(p, "sg"), study="table1", level=lev, N=N, nr=None, cycle="SG"), out)
            for nr in nrs:
                if nr >= N:
                    continue
                for pre, post in ((1, 1), (2, 1)):
                    p = inputs.paper_box(N, level=lev, nr=nr, n=n, nu_pre=pre, nu_post=post, nr_levels="coarsest",
                                         nu_coarse=nu_coarse, basis=basis)
                    _emit(dict(solve_case(p, "f64"), study="table1", level=lev, N=N, nr=nr,
                               cycle="V(%d,%d)" % (pre, post)), out)
    return out


def nr_effect(n=30, level=3, Ns=(4, 8, 12, 16, 20, 24), nu_coarse=10, nrs=(1, 2, 3, 4, 6, 8, 10, 12, 16, 20, 24),
              basis="lin", out=None):
    out = [] if out is None else out
    for N in Ns:
        for nr in sorted(set(v for v in nrs if v <= N) | {OPTIMAL_NR.get(N, N)}):
            for pre, post in ((1, 0), (1, 1)):
                p = inputs.paper_box(N, level=level, nr=nr, n=n, nu_pre=pre, nu_post=post, nu_coarse=nu_coarse,
                                     basis=basis)
                _emit(dict(solve_case(p, "f64"), study="nr", level=level, N=N, nr=nr,
                           cycle="V(%d,%d)" % (pre, post)), out)
    return out


def final(n=30, level=3, Ns=(4, 8, 12, 16, 20, 24), nu_coarse=10, sg_max_N=20, beam=False, lmaxs=(None,),
          basis="lin", out=None):
    out = [] if out is None else out
    for lmax in lmaxs:
        for N in Ns:
            kw = dict(n=n, nu_coarse=nu_coarse, beam=beam, band_lmax=lmax or 0, level=level, basis=basis)
            if N <= sg_max_N:
                p = inputs.paper_box(N, **kw)
                _emit(dict(solve_case(p, "sg"), study="beam" if beam else "final", level=lmax or level, N=N,
                           nr=None, cycle="SG"), out)
            for pre, post in ((1, 0), (1, 1)):
                p = inputs.paper_box(N, nr=OPTIMAL_NR[N], nu_pre=pre, nu_post=post, **kw)
                _emit(dict(solve_case(p, "f64"), study="beam" if beam else "final", level=lmax or level, N=N,
                           nr=OPTIMAL_NR[N], cycle="V(%d,%d)" % (pre, post)), out)
    return out


def markdown(recs):
    """One row per (level, N, N_r, cycle): iterations and solve seconds."""
    lines = ["| study | basis | level | N | N_r | cycle | DoFs | iterations | solve s | converged |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for r in recs:
        lines.append("| %s | %s | %s | %d | %s | %s | %.3g | %d | %.3f | %s |" % (
            r["study"], r["basis"], r["level"], r["N"], "-" if r["nr"] is None else r["nr"], r["cycle"], r["dofs"],
            r["iters"], r["solve_s"], "yes" if r["converged"] else "no"))
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("study", choices=["table1", "nr", "final", "beam"])
    ap.add_argument("--n", type=int, default=30, help="cells per axis (30 in the paper)")
    ap.add_argument("--N", default=None, help="comma-separated scatter orders")
    ap.add_argument("--levels", default=None, help="comma-separated angular levels (table1) or l_max (beam)")
    ap.add_argument("--nu-coarse", type=int, default=None)
    ap.add_argument("--sg-max-N", type=int, default=20, help="largest N with a single-grid solve")
    ap.add_argument("--basis", default="lin", choices=["lin", "const"], help="angular basis (Section 2.2)")
    a = ap.parse_args(argv)
    ints = lambda s: tuple(int(v) for v in s.split(","))
    if a.study == "table1":
        recs = table1(n=a.n, levels=ints(a.levels) if a.levels else (1, 2, 3), Ns=ints(a.N) if a.N else (4, 8, 16),
                      nu_coarse=a.nu_coarse or 40, basis=a.basis)
    elif a.study == "nr":
        recs = nr_effect(n=a.n, Ns=ints(a.N) if a.N else (4, 8, 12, 16, 20, 24), nu_coarse=a.nu_coarse or 10,
                         basis=a.basis)
    elif a.study == "final":
        recs = final(n=a.n, Ns=ints(a.N) if a.N else (4, 8, 12, 16, 20, 24), nu_coarse=a.nu_coarse or 10,
                     sg_max_N=a.sg_max_N, basis=a.basis)
    else:
        recs = final(n=a.n, Ns=ints(a.N) if a.N else (4, 8, 12, 16, 20, 24), nu_coarse=a.nu_coarse or 10,
                     sg_max_N=a.sg_max_N, beam=True, lmaxs=ints(a.levels) if a.levels else (1, 2, 3, 4, 5, 6),
                     basis=a.basis)
    print(markdown(recs), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
