"""GPU checks of the paper-replication path: the BiCGStab outer solver
(Section 3), the Fokker-Planck-equivalent moments (eq. scatter_moments),
the z-band angular meshes and the z pencil beam (Section 5.5), each against
the oracle on small problems: identical iteration counts and solutions to
1e-10 with the FP64 preconditioner, 1e-7 with the FP32 one."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import krylov
from paper_2010_04559_amd import inputs
from gpu_util import Pair, small, to_dev, to_np, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kw", [dict(dim=3, n=4, level=1, order=6, seed=41), dict(dim=2, n=5, level=2, order=8, seed=42)])
def test_bicgstab_matches_oracle(kw):
    prob = small(g=0.9, c=0.97, **kw)
    print("case", prob.name, flush=True)
    pr = Pair(prob)
    b = pr.op.rhs()
    ref = krylov.bicgstab(pr.op.outer.apply_A, pr.op.mg.vcycle, b, 1e-10)
    assert ref.converged
    x, st = pr.tr.solve(to_dev(b), tol=1e-10, method="bicgstab")
    assert st["converged"] == 1 and st["iters"] == ref.iters
    assert rel(to_np(x), ref.x) < 1e-10
    xm, sm = pr.tr.solve(to_dev(b), tol=1e-10, method="bicgstab", mode="mixed")
    assert sm["converged"] == 1 and rel(to_np(xm), ref.x) < 1e-7


def _paper_small(beam):
    """The paper's cube workload shrunk to 6^3 cells (5 cm, FP moments N = 4,
    transport cross section 1), on a z-band mesh (l_max = 2) for the beam and
    on the level-1 mesh for the volume source."""
    prob = inputs.paper_box(4, level=1, nr=2, n=6, beam=beam, band_lmax=2 if beam else 0, restart=10)
    return prob


@pytest.mark.parametrize("beam", [False, True])
def test_paper_workload_matches_oracle(beam):
    prob = _paper_small(beam)
    print("case", prob.name, flush=True)
    pr = Pair(prob)
    if beam:
        assert pr.tr.patches == [8, 20, 32]
    b = pr.op.rhs()
    assert rel(to_np(pr.tr.rhs()), b) < 1e-13
    for method, solver in (("gmres", lambda: krylov.gmres(pr.op.outer.apply_A, pr.op.mg.vcycle, b, 1e-10,
                                                           prob.restart)),
                           ("bicgstab", lambda: krylov.bicgstab(pr.op.outer.apply_A, pr.op.mg.vcycle, b, 1e-10))):
        ref = solver()
        assert ref.converged
        x, st = pr.tr.solve(to_dev(b), tol=1e-10, method=method)
        assert st["converged"] == 1 and st["iters"] == ref.iters, (method, st["iters"], ref.iters)
        assert rel(to_np(x), ref.x) < 1e-10, method
