"""Pins of the oracle's transport operators: exact inverses, the 1-D upwind
DG closed form, the infinite-medium solution, conservation and symmetry."""
import math

import numpy as np
import pytest

from oracle import angular as ang
from oracle import spatial as sp
from oracle import transport as tr
from oracle import multigrid as mgm
from oracle import krylov


def _level(dim, n, level, g=0.8, order=4, c=0.8, seed=0, uniform=False):
    grid = sp.Grid(dim, n)
    rng = np.random.default_rng(seed)
    if uniform:
        st = np.full(grid.C, 2.0)
        ss = c * st
    else:
        st = rng.uniform(0.5, 3.0, grid.C)
        ss = c * st * rng.uniform(0.5, 1.0, grid.C)
    return tr.Level(grid, ang.AngularMesh.uniform(level).leaves(), st, ss, ang.hg_moments(g, order))


@pytest.mark.parametrize("dim,n", [(2, (3, 4)), (3, (2, 3, 2))])
def test_sweep_is_exact_inverse(dim, n):
    lv = _level(dim, n, 1)
    x = np.random.default_rng(1).standard_normal(lv.A * lv.grid.S)
    assert np.abs(lv.apply_L(lv.sweep(x)) - x).max() < 1e-12
    assert np.abs(lv.apply_LT(lv.sweep_T(x)) - x).max() < 1e-12


def test_transposed_operators_are_transposes():
    lv = _level(2, (2, 3), 0)
    L = lv.dense(lv.apply_L)
    LT = lv.dense(lv.apply_LT)
    S = lv.dense(lv.apply_S)
    assert np.abs(L.T - LT).max() < 1e-15
    assert np.abs(S - S.T).max() < 1e-14 * np.abs(S).max()


def _pade(z):
    """(1,2) Pade approximant of exp(-z): the per-cell outflow factor of
    upwind DG with linear elements for a pure absorber."""
    return (1 - z / 3) / (1 + 2 * z / 3 + z * z / 6)


def test_pade_factor_approximates_exponential():
    z = np.array([1e-3, 1e-2, 1e-1])
    err = np.abs(_pade(z) - np.exp(-z))
    assert (err < z ** 4 / 50).all()


@pytest.mark.parametrize("dim,n", [(2, (5, 4)), (3, (4, 3, 3))])
def test_x_only_solution_has_pade_outflow(dim, n):
    """A pure absorber with unit isotropic inflow on x=0 and data independent
    of the transverse coordinates: in every cell away from the transverse
    boundaries each ordinate's nodal values are those of the 1-D upwind DG
    solution, outflow R(z)^i after i cells, z = sigma_t h / Omega_x."""
    grid = sp.Grid(dim, n)
    sig = 3.0
    lv = tr.Level(grid, ang.AngularMesh.uniform(1).leaves(), np.full(grid.C, sig),
                  np.zeros(grid.C), [1.0])
    h = grid.h[0]
    phi = np.zeros((lv.A, grid.C, grid.ns))
    bx = np.arange(grid.ns) & 1
    ix = grid.coords[:, 0]
    for q in range(lv.P):
        sel = lv.rule.owner == q
        om = lv.rule.omega[sel]
        u = np.zeros((3, grid.C, grid.ns))
        for k in range(3):
            if om[k, 0] <= 0:
                continue
            z = sig * h / om[k, 0]
            R = _pade(z)
            left = R ** ix * (1 + 2 * z / 3) / (1 + 2 * z / 3 + z * z / 6)
            right = R ** (ix + 1)
            u[k] = np.where(bx[None, :] == 0, left[:, None], right[:, None])
        # nodal ordinate values -> Lin coefficients: u_k = sum_d psi_d(Omega_k) phi_d
        phi[3 * q:3 * q + 3] = np.linalg.solve(lv.rule.psi[q], u.reshape(3, -1)).reshape(3, grid.C, grid.ns)
    res = lv.apply_L(phi.reshape(-1)) - lv.rhs_inflow_iso(0, 0, (0, 0, 0), (99, 99, 99), 1.0)
    res = res.reshape(lv.A, grid.C, grid.ns)
    inner = np.ones(grid.C, dtype=bool)
    for a in range(1, dim):
        inner &= (grid.coords[:, a] > 0) & (grid.coords[:, a] < grid.n[a] - 1)
    assert inner.any()
    assert np.abs(res[:, inner]).max() < 1e-13


@pytest.mark.parametrize("dim,n,order,g", [(2, (3, 3), 6, 0.9), (3, (2, 2, 2), 4, 0.7), (2, (2, 3), 12, 0.95)])
def test_infinite_medium(dim, n, order, g):
    """Uniform medium, uniform isotropic source q and isotropic inflow
    q / (sigma_t - sigma_s) on every boundary face: the exact solution is that
    constant for any scatter order, and the discrete one reproduces it."""
    grid = sp.Grid(dim, n)
    st, ss, q = 2.0, 1.6, 1.0
    lv = tr.Level(grid, ang.AngularMesh.uniform(1).leaves(), np.full(grid.C, st),
                  np.full(grid.C, ss), ang.hg_moments(g, order))
    phic = q / (st - ss)
    b = lv.rhs_volume(np.full(grid.C, q))
    for xi in range(dim):
        for side in (0, 1):
            b = b + lv.rhs_inflow_iso(xi, side, (0, 0, 0), (99, 99, 99), phic)
    x = np.full(lv.A * grid.S, phic)
    assert np.abs(lv.apply_A(x) - b).max() < 1e-13 * np.abs(b).max()
    # and the scalar flux of the solve equals 4 pi phic in every cell
    xs = np.linalg.solve(lv.dense(lv.apply_A), b)
    assert np.abs(lv.scalar_flux_cell_avg(xs) - 4 * math.pi * phic).max() < 1e-10


def test_scatter_conserves_particles():
    """Total scattered-in source equals sigma_s times the integrated flux:
    only the n = 0 moment survives integration over the sphere."""
    lv = _level(3, (2, 2, 3), 1, g=0.9, order=8)
    x = np.random.default_rng(7).standard_normal(lv.A * lv.grid.S)
    g = lv.grid
    tot = lv.apply_S(x).reshape(lv.A, g.C, g.ns).sum(axis=(0, 2))
    ipsi = np.concatenate([ang.lin_basis(p, om).T @ w for p in lv.patches
                           for om, w in [ang.quad_accurate(p)]])
    ref = lv.sigma_s * np.einsum('a,acl,l->c', ipsi, x.reshape(lv.A, g.C, g.ns), g.basis_int)
    assert np.abs(tot - ref).max() < 1e-12 * np.abs(ref).max()


def test_spatial_matrices_closed_forms():
    g = sp.Grid(3, (2, 3, 4), (1.0, 2.0, 3.0))
    vol = np.prod(g.h)
    assert abs(g.N.sum() - vol) < 1e-15
    assert np.allclose(g.basis_int, vol / 8)
    for xi in range(3):
        # int grad_xi Phi_l summed over l vanishes (sum of basis = 1)
        assert np.abs(g.V[xi].sum(axis=0)).max() < 1e-15
        for side in (0, 1):
            assert abs(g.F[xi][side].sum() - vol / g.h[xi]) < 1e-14


def test_symmetry_of_scalar_flux():
    """Uniform cube, centred source, octahedrally symmetric angular mesh: the
    cell-average scalar flux is invariant under the cube's symmetries."""
    n = 4
    grid = sp.Grid(3, (n, n, n))
    mesh = ang.AngularMesh.uniform(1)
    C = grid.C
    st, ss = np.full(C, 1.5), np.full(C, 1.2)
    mg = mgm.AngularMG(grid, mesh, st, ss, ang.hg_moments(0.7, 4), [4, 4])
    lv = mg.levels[-1]
    q = np.zeros(C)
    q[grid.box_cells((1, 1, 1), (2, 2, 2))] = 1.0
    b = lv.rhs_volume(q)
    res = krylov.gmres(lv.apply_A, mg.vcycle, b, 1e-12, 10)
    assert res.converged
    f = lv.scalar_flux_cell_avg(res.x).reshape(n, n, n)      # [iz, iy, ix]
    for t in (f[:, :, ::-1], f[:, ::-1, :], f[::-1, :, :], f.transpose(0, 2, 1), f.transpose(2, 1, 0)):
        assert np.abs(t - f).max() < 1e-9 * np.abs(f).max()
