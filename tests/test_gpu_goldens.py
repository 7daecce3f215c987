"""GPU solves of the 3-D workloads against the oracle's reference
solutions (tests/golden/oracle_*.json, written by make_goldens.py from the
oracle alone): the same GMRES iteration count with the FP64 preconditioner
and the cell-average scalar flux to 1e-10 (FP64) and 1e-7 (FP32
preconditioner inside FP64 GMRES); for the beam workloads the detector
response and its adjoint gradient on the finite-difference cells.

Workloads: the 32^3 headline and beam problems, and the precision problem's
angular mesh and orders (512 patches, 8/8/8/32) and the cone mesh (368
patches, L = 64) on 16^3 cells."""
import json
import os

import numpy as np
import pytest

from oracle import angular as ang, spatial as sp, transport as otr
from paper_2010_04559_amd import inputs
from oracle_problem import angular_mesh
from gpu_util import to_np, torch_mod

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
WORKLOADS = {"cfg2_32": lambda: inputs.config2(32), "cfg4_32": lambda: inputs.config4(32),
             "cfg3_16": lambda: inputs.config3(16), "cfg5_16": lambda: inputs.config5(16)}


def _golden(name):
    path = os.path.join(GOLDEN, "oracle_%s.json" % name)
    if not os.path.exists(path):
        pytest.skip("no oracle reference %s (make_goldens.py not run for it)" % name)
    with open(path) as fh:
        return json.load(fh)


def _cell_avg(prob, x):
    """Cell-average scalar flux on the device, with the oracle's angular and
    spatial basis integrals."""
    torch = torch_mod()
    grid = sp.Grid(prob.dim, prob.n, prob.length)
    leaves = angular_mesh(prob.angular).leaves()
    rule = ang.PatchRule(leaves)
    ipsi = np.concatenate([rule.basis_integral(q) for q in range(len(leaves))])
    ip = torch.as_tensor(ipsi, device="cuda")
    bi = torch.as_tensor(grid.basis_int, device="cuda")
    v = x.view(len(ipsi), grid.C, grid.ns)
    out = torch.zeros(grid.C, dtype=torch.float64, device="cuda")
    for a0 in range(0, len(ipsi), 64):
        out += torch.einsum("a,acl,l->c", ip[a0:a0 + 64], v[a0:a0 + 64], bi)
    return (out / float(np.prod(grid.h))).cpu().numpy()


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_solve_matches_oracle_reference(name):
    from paper_2010_04559_amd.transport import Transport
    ref = _golden(name)
    prob = WORKLOADS[name]()
    assert prob.name == ref["problem"]
    print("case", name, flush=True)
    tr = Transport(prob)
    assert tr.patches == ref["patches"]
    b = tr.rhs()
    cells = np.asarray(ref["phi_cells"])
    want = np.asarray(ref["phi_cell_avg"])
    x, st = tr.solve(b)
    assert st["converged"] == 1 and st["iters"] == ref["oracle_iters"]
    phi = _cell_avg(prob, x)
    assert np.abs(phi[cells] - want).max() < 1e-10 * np.abs(want).max()
    assert abs(phi.sum() - ref["phi_total"]) < 1e-10 * abs(ref["phi_total"])
    xm, stm = tr.solve(b, mode="mixed")
    assert stm["converged"] == 1 and stm["iters"] <= ref["oracle_iters"] + 1
    phim = _cell_avg(prob, xm)
    assert np.abs(phim[cells] - want).max() < 1e-7 * np.abs(want).max()
    if "response" in ref:
        w = tr.detector()
        R = tr.response(w, x)
        assert abs(R - ref["response"]) < 1e-9 * abs(ref["response"])
        gt, gs, lam, sta = tr.adjoint_grad(w, x)
        assert sta["converged"] == 1 and sta["iters"] == ref["adjoint_iters"]
        fd = np.asarray(ref["grad_cells"])
        gt, gs = to_np(gt), to_np(gs)
        assert np.abs(gt[fd] - ref["grad_sigma_t"]).max() < 1e-8 * ref["grad_sigma_t_maxabs"]
        assert np.abs(gs[fd] - ref["grad_sigma_s"]).max() < 1e-8 * ref["grad_sigma_s_maxabs"]
    tr.close()


def test_cfg2_coarse_gs_matches_oracle():
    """The ten-sweep coarse Gauss-Seidel solve of the 32^3 problem in the
    launch configuration the solver uses (2 x 2 x 2 bricks, 1310 dependent
    steps), forward and adjoint, against the oracle's sequential sweeps."""
    from oracle_problem import OracleProblem
    from paper_2010_04559_amd.transport import Transport
    prob = inputs.config2()
    print("case cfg2 coarse GS", flush=True)
    tr = Transport(prob)
    op = OracleProblem(prob)
    f = np.random.default_rng(9).standard_normal(tr.n(0))
    torch = torch_mod()
    fd = torch.as_tensor(f, device="cuda")
    for adj in (False, True):
        got = to_np(tr.coarse_gs(fd, prob.nu_coarse, adjoint=adj))
        want = op.mg.coarse_gs(f, prob.nu_coarse, adjoint=adj)
        assert np.abs(got - want).max() < 1e-11 * np.abs(want).max(), adj
    tr.close()
