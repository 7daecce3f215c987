"""Pins of the oracle's Const angular basis (Section 2.2: one constant
function per patch), against closed forms and properties the mathematics
fixes:

* octant patches: |q| = pi/2 and int_q Omega_xi = s_xi pi/4 (so the mean
  direction of an octant is (1, 1, 1)/2 up to signs); the areas tile the
  sphere and int Omega over the sphere vanishes;
* scatter: order 0 gives S~ = f_0 |q||p| / (4 pi); S~ 1 = f_0 |q| for any
  order (only n = 0 survives integration over the sphere); the X-based S~
  equals the addition-theorem S~ (convention-free);
* prolongation: daughters take the parent's value, so P 1 = 1 and the
  coarse mass equals P^T M_fine P;
* transport: the sweep inverts L exactly; the infinite-medium solution is
  reproduced for every scatter order (the Const scatter keeps an isotropic
  state exact, unlike the Lin basis with the 3-point rule);
* solver: the coarse Gauss-Seidel sweep converges to the dense coarse
  solve, the multigrid GMRES and BiCGStab solutions equal dense solves, and
  multigrid needs fewer iterations than the single-sweep preconditioner.
"""
import math

import numpy as np
import pytest

from oracle import angular as ang
from oracle import spatial as sp
from oracle import transport as tr
from oracle import multigrid as mgm
from oracle import krylov


def test_octant_integrals_closed_form():
    patches = ang.AngularMesh.uniform(0).leaves()
    rule = ang.PatchRule(patches, basis="const")
    for q, p in enumerate(patches):
        s = ang.octant_signs(p.octant)
        assert abs(rule.mass(q)[0, 0] - math.pi / 2) < 1e-14
        for xi in range(3):
            assert abs(rule.jacobian(q, xi)[0, 0] - s[xi] * math.pi / 4) < 1e-14


@pytest.mark.parametrize("level", [1, 2])
def test_areas_and_first_moments_tile_the_sphere(level):
    patches = ang.AngularMesh.uniform(level).leaves()
    rule = ang.PatchRule(patches, basis="const")
    area = sum(rule.mass(q)[0, 0] for q in range(len(patches)))
    assert abs(area - 4 * math.pi) < 1e-12
    for xi in range(3):
        mom = [rule.jacobian(q, xi)[0, 0] for q in range(len(patches))]
        assert abs(sum(mom)) < 1e-13
        # the patches of one octant add up to its pi/4
        for o in range(8):
            part = sum(m for m, p in zip(mom, patches) if p.octant == o)
            assert abs(abs(part) - math.pi / 4) < 1e-13


def test_scatter_closed_forms_and_addition_theorem():
    patches = ang.AngularMesh.uniform(1).leaves()
    area = np.array([ang.spherical_area(p.verts) for p in patches])
    S0 = ang.scatter_matrix(patches, [0.7], basis="const")
    assert np.abs(S0 - 0.7 * np.outer(area, area) / (4 * math.pi)).max() < 1e-14
    mom = ang.hg_moments(0.85, 7)
    S = ang.scatter_matrix(patches, mom, basis="const")
    assert S.shape == (32, 32)
    assert np.abs(S @ np.ones(32) - area).max() < 1e-13
    oct8 = ang.AngularMesh.uniform(0).leaves()
    S8 = ang.scatter_matrix(oct8, mom, basis="const")
    Sa = ang.scatter_matrix_addition(oct8, mom, basis="const")
    assert np.abs(S8 - Sa).max() < 1e-13 * np.abs(S8).max()
    rows = ang.scatter_rows_addition(patches, mom, 5, basis="const")
    assert np.abs(rows - S[5:6]).max() < 1e-13 * np.abs(S).max()


def test_const_prolongation_injects():
    T = ang.AngularMesh.cone((1.0, 0.0, 0.0), 20.0, 1, 2).levels()
    for l in range(1, len(T)):
        P = ang.prolongation(T[l - 1], T[l], basis="const")
        assert np.abs(P @ np.ones(len(T[l - 1])) - 1).max() == 0
        Mf = np.diag([ang.spherical_area(p.verts) for p in T[l]])
        Mc = np.diag([ang.spherical_area(p.verts) for p in T[l - 1]])
        assert np.abs(P.T @ Mf @ P - Mc).max() < 1e-13


def _level(dim, n, level, g=0.8, order=4, c=0.8, seed=0):
    grid = sp.Grid(dim, n)
    rng = np.random.default_rng(seed)
    st = rng.uniform(0.5, 3.0, grid.C)
    ss = c * st * rng.uniform(0.5, 1.0, grid.C)
    return tr.Level(grid, ang.AngularMesh.uniform(level).leaves(), st, ss, ang.hg_moments(g, order),
                    basis="const")


@pytest.mark.parametrize("dim,n", [(2, (3, 4)), (3, (2, 3, 2))])
def test_const_sweep_is_exact_inverse(dim, n):
    lv = _level(dim, n, 1)
    assert lv.A == lv.P
    x = np.random.default_rng(1).standard_normal(lv.A * lv.grid.S)
    assert np.abs(lv.apply_L(lv.sweep(x)) - x).max() < 1e-12
    assert np.abs(lv.apply_LT(lv.sweep_T(x)) - x).max() < 1e-12


@pytest.mark.parametrize("dim,n,order,g", [(2, (3, 3), 6, 0.9), (3, (2, 2, 2), 9, 0.7)])
def test_const_infinite_medium(dim, n, order, g):
    grid = sp.Grid(dim, n)
    st, ss, q = 2.0, 1.6, 1.0
    lv = tr.Level(grid, ang.AngularMesh.uniform(1).leaves(), np.full(grid.C, st), np.full(grid.C, ss),
                  ang.hg_moments(g, order), basis="const")
    phic = q / (st - ss)
    b = lv.rhs_volume(np.full(grid.C, q))
    for xi in range(dim):
        for side in (0, 1):
            b = b + lv.rhs_inflow_iso(xi, side, (0, 0, 0), (99, 99, 99), phic)
    x = np.full(lv.A * grid.S, phic)
    assert np.abs(lv.apply_A(x) - b).max() < 1e-13 * np.abs(b).max()
    xs = np.linalg.solve(lv.dense(lv.apply_A), b)
    assert np.abs(lv.scalar_flux_cell_avg(xs) - 4 * math.pi * phic).max() < 1e-10


def _const_mg(dim=2, n=3, level=1, order=6, g=0.9, seed=0, nu_coarse=10):
    grid = sp.Grid(dim, (n,) * dim)
    rng = np.random.default_rng(seed)
    st = rng.uniform(0.5, 3.0, grid.C)
    ss = 0.9 * st
    mesh = ang.AngularMesh.uniform(level)
    return mgm.AngularMG(grid, mesh, st, ss, ang.hg_moments(g, order), [order] * (level + 1),
                         nu_coarse=nu_coarse, basis="const")


def test_const_coarse_gauss_seidel_converges_to_coarse_solve():
    mg = _const_mg()
    lv0 = mg.levels[0]
    assert lv0.A == 8
    f = np.random.default_rng(2).standard_normal(lv0.A * lv0.grid.S)
    ref = np.linalg.solve(lv0.dense(lv0.apply_A), f)
    assert np.abs(mg.coarse_gs(f, 40) - ref).max() < 1e-11 * np.abs(ref).max()
    refa = np.linalg.solve(lv0.dense(lv0.apply_AT), f)
    assert np.abs(mg.coarse_gs(f, 40, adjoint=True) - refa).max() < 1e-11 * np.abs(refa).max()


def test_const_mg_solvers_match_dense_solve():
    mg = _const_mg(dim=2, n=3, level=2, order=8, g=0.95, nu_coarse=10)
    lv = mg.levels[-1]
    b = lv.rhs_volume(np.ones(lv.grid.C)) + lv.rhs_beam((1.0, 0.3, 0.0), 0, 0, (0, 0, 0), (9, 9, 9))
    ref = np.linalg.solve(lv.dense(lv.apply_A), b)
    res = krylov.gmres(lv.apply_A, mg.vcycle, b, 1e-11, 10)
    assert res.converged and np.abs(res.x - ref).max() < 1e-9 * np.abs(ref).max()
    bic = krylov.bicgstab(lv.apply_A, mg.vcycle, b, 1e-11)
    assert bic.converged and np.abs(bic.x - ref).max() < 1e-9 * np.abs(ref).max()
    sg = krylov.gmres(lv.apply_A, lv.sweep, b, 1e-11, 10)
    assert sg.converged and res.iters < sg.iters
