"""Pins of the oracle's angular discretisation against the paper's numbers,
closed forms and library routines."""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import angular as ang

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_counts():
    rows = []
    with open(os.path.join(GOLDEN, "band_mesh_counts.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                a, b = line.split()
                rows.append((int(a), int(b)))
    return rows


@pytest.mark.parametrize("lmax,count", _golden_counts())
def test_band_mesh_counts_match_paper(lmax, count):
    assert len(ang.AngularMesh.band_z(lmax).leaves()) == count


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_uniform_counts(level):
    m = ang.AngularMesh.uniform(level)
    assert len(m.leaves()) == 8 * 4 ** level
    assert [len(T) for T in m.levels()] == [8 * 4 ** l for l in range(level + 1)]


def _max_neighbour_jump(leaves):
    return max(abs(leaves[i].level - leaves[j].level) for i, j in ang.edge_neighbours(leaves))


def test_cone_mesh_closure_two_irregular():
    lit = ang.AngularMesh.cone([1, 0, 0], 15.0, 2, 3, closure=False)
    clo = ang.AngularMesh.cone([1, 0, 0], 15.0, 2, 3, closure=True)
    assert _max_neighbour_jump(lit.leaves()) == 3
    assert _max_neighbour_jump(clo.leaves()) <= 2
    assert len(lit.leaves()) == 356 and len(clo.leaves()) == 368
    assert [len(T) for T in clo.levels()] == [8, 32, 128, 152, 200, 368]


@pytest.mark.parametrize("mesh", [ang.AngularMesh.uniform(3), ang.AngularMesh.band_z(4),
                                  ang.AngularMesh.cone([1, 0, 0], 15.0, 2, 3)])
def test_patch_areas_tile_the_sphere(mesh):
    leaves = mesh.leaves()
    assert abs(sum(ang.spherical_area(p.verts) for p in leaves) - 4 * math.pi) < 1e-12
    w3 = ang.PatchRule(leaves).w
    assert abs(w3.sum() - 4 * math.pi) < 1e-12
    assert (w3 > 0).all()


def test_accurate_rule_matches_exact_area():
    # the collapsed Gauss rule with the gnomonic Jacobian against the
    # Van Oosterom-Strackee closed form, patch by patch
    for p in ang.AngularMesh.band_z(3).leaves():
        _, w = ang.quad_accurate(p)
        assert abs(w.sum() - ang.spherical_area(p.verts)) < 1e-14


def test_harmonics_integrate_to_closed_form():
    # int_4pi Y_no = sqrt(4 pi) delta_{n0}; int Y_a Y_b = delta_ab
    leaves = ang.AngularMesh.band_z(3).leaves()
    order = 6
    tot = np.zeros((order + 1) ** 2)
    gram = np.zeros(((order + 1) ** 2,) * 2)
    for p in leaves:
        om, w = ang.quad_accurate(p, 2 * order)
        Y = ang.real_harmonics(order, om)
        tot += Y.T @ w
        gram += (Y * w[:, None]).T @ Y
    ref = np.zeros_like(tot)
    ref[0] = math.sqrt(4 * math.pi)
    assert np.abs(tot - ref).max() < 1e-13
    assert np.abs(gram - np.eye(len(tot))).max() < 1e-12


def test_lin_basis_nodal_and_partition_of_unity():
    rng = np.random.default_rng(3)
    for p in ang.AngularMesh.cone([1, 0, 0], 15.0, 2, 3).leaves()[::7]:
        assert np.abs(ang.lin_basis(p, p.verts) - np.eye(3)).max() < 1e-13
        lam = rng.dirichlet(np.ones(3), 5)
        om = lam @ p.verts
        om /= np.linalg.norm(om, axis=1)[:, None]
        assert np.abs(ang.lin_basis(p, om).sum(axis=1) - 1).max() < 1e-13


@pytest.mark.parametrize("mesh", [ang.AngularMesh.uniform(2), ang.AngularMesh.cone([1, 0, 0], 15.0, 2, 3)])
def test_prolongation_reproduces_gnomonic_linear_functions(mesh):
    # a function linear in the projected coordinates of every octant is in
    # every Lin space (Section 4.1: nested spaces, prolongation exact)
    rng = np.random.default_rng(5)
    coef = rng.standard_normal((8, 3))

    def f(p, pts):
        s = ang.octant_signs(p.octant)
        return ang.gnomonic(pts, s) @ coef[p.octant]

    T = mesh.levels()
    for l in range(1, len(T)):
        P = ang.prolongation(T[l - 1], T[l])
        xc = np.concatenate([f(p, p.verts) for p in T[l - 1]])
        xf = np.concatenate([f(p, p.verts) for p in T[l]])
        assert np.abs(P @ xc - xf).max() < 1e-12


def test_scatter_matrix_addition_theorem():
    for lev, L in [(0, 3), (1, 6)]:
        pts = ang.AngularMesh.uniform(lev).leaves()
        mom = ang.hg_moments(0.8, L)
        a = ang.scatter_matrix(pts, mom)
        b = ang.scatter_matrix_addition(pts, mom)
        assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()
        assert np.abs(a - a.T).max() < 1e-15


def test_scatter_rows_by_recurrence_match_full_matrix():
    pts = ang.AngularMesh.uniform(1).leaves()
    mom = ang.hg_moments(0.9, 7)
    full = ang.scatter_matrix(pts, mom)
    for q in (0, 13):
        rows = ang.scatter_rows_addition(pts, mom, q, chunk=50)
        assert np.abs(rows - full[3 * q:3 * q + 3]).max() < 1e-12 * np.abs(full).max()


def test_scatter_isotropic_cases():
    pts = ang.AngularMesh.uniform(1).leaves()
    ipsi = np.concatenate([(ang.lin_basis(p, om).T @ w) for p in pts
                           for om, w in [ang.quad_accurate(p)]])
    s0 = ang.scatter_matrix(pts, [1.0])
    assert np.abs(s0 - np.outer(ipsi, ipsi) / (4 * math.pi)).max() < 1e-14
    # an isotropic flux scatters isotropically for any order: only n = 0 survives
    s = ang.scatter_matrix(pts, ang.hg_moments(0.9, 12))
    assert np.abs(s @ np.ones(len(ipsi)) - ipsi).max() < 1e-13


def test_scatter_spectrum_bounded_by_moments():
    # S~ is the Galerkin compression of an operator with eigenvalues f_n, so
    # relative to the exact Lin mass matrix its spectrum lies in [min f, max f]
    pts = ang.AngularMesh.uniform(1).leaves()
    mom = ang.hg_moments(0.95, 10)
    S = ang.scatter_matrix(pts, mom)
    rule = ang.PatchRule(pts, lambda p: ang.quad_accurate(p, 4))
    M = sl.block_diag(*[rule.mass(q) for q in range(len(pts))])
    ev = sl.eigh(S, M, eigvals_only=True)
    assert ev.max() <= mom.max() + 1e-12 and ev.min() >= min(mom.min(), 0.0) - 1e-12


def test_x_integrals_converged():
    pts = ang.AngularMesh.uniform(2).leaves()[:6]
    X = ang.x_integrals(pts, 16)
    ref = np.zeros_like(X)
    for q, p in enumerate(pts):
        n = ang.accurate_points(16, p) + 16
        om, w = ang._flat_rule_on_patch(p, *ang.collapsed_gauss(n))
        ref[3 * q:3 * q + 3] = (ang.lin_basis(p, om) * w[:, None]).T @ ang.real_harmonics(16, om)
    assert np.abs(X - ref).max() < 1e-14


def test_quad3_collocation_structure():
    # psi_d(Omega_k) is the same matrix (3 I + J) / 6 on every patch
    pts = ang.AngularMesh.cone([1, 0, 0], 15.0, 2, 3).leaves()
    rule = ang.PatchRule(pts)
    ref = (3 * np.eye(3) + np.ones((3, 3))) / 6
    for ps in rule.psi:
        assert np.abs(ps - ref).max() < 1e-13


def _octant_perm(leaves, mask):
    """Row maps of the reflection group of the axes in ``mask``: the patch of
    octant o at position k goes to position k of octant o ^ s (asserted by
    reflecting its vertices)."""
    by_oct = {o: [p for p in leaves if p.octant == o] for o in range(8)}
    for o in range(8):
        for d in range(3):
            if mask & (1 << d):
                o2 = o ^ (1 << d)
                assert len(by_oct[o]) == len(by_oct[o2])
                for p, p2 in zip(by_oct[o], by_oct[o2]):
                    v = p.verts.copy()
                    v[:, d] *= -1
                    assert np.abs(v - p2.verts).max() < 1e-14
    start, off = {}, 0
    for o in range(8):
        start[o] = off
        off += 3 * len(by_oct[o])
    return by_oct, start


@pytest.mark.parametrize("mesh,mask", [("uniform2", 7), ("cone", 6), ("band", 3)])
def test_scatter_matrix_reflection_structure(mesh, mask):
    """On a mesh mapped onto itself by the reflections of the axes in mask,
    the scatter matrix depends on two octants only through their sign
    difference, and the Walsh-Hadamard transform over the reflected sign
    patterns splits it into 2^R diagonal blocks of size A / 2^R (the form
    the library's scatter product uses)."""
    leaves = {"uniform2": lambda: ang.AngularMesh.uniform(2).leaves(),
              "cone": lambda: ang.AngularMesh.cone((1, 0, 0), 15.0, 1, 2).leaves(),
              "band": lambda: ang.AngularMesh.band_z(3).leaves()}[mesh]()
    St = ang.scatter_matrix(leaves, ang.hg_moments(0.9, 6))
    by_oct, start = _octant_perm(leaves, mask)
    bits = [d for d in range(3) if mask & (1 << d)]
    R = len(bits)
    pats = [sum(1 << bits[b] for b in range(R) if i & (1 << b)) for i in range(2 ** R)]
    reps = [f for f in range(8) if not f & mask]
    urow = np.array([[start[f | s] + k for f in reps for k in range(3 * len(by_oct[f]))] for s in pats])
    nc = urow.shape[1]
    assert nc * 2 ** R == St.shape[0]
    # M[(i1,t1),(i2,t2)] = M[(0,t1),(i1^i2,t2)]
    for i1 in range(2 ** R):
        for i2 in range(2 ** R):
            a = St[np.ix_(urow[i1], urow[i2])]
            b = St[np.ix_(urow[0], urow[i1 ^ i2])]
            assert np.abs(a - b).max() < 1e-13 * np.abs(St).max()
    # block form of the product
    sign = np.array([[(-1) ** bin(i & j).count("1") for i in range(2 ** R)] for j in range(2 ** R)], float)
    B = [sum(sign[j, i] * St[np.ix_(urow[0], urow[i])] for i in range(2 ** R)) / 2 ** R for j in range(2 ** R)]
    u = np.random.default_rng(0).standard_normal((St.shape[0], 5))
    uh = [sum(sign[j, i] * u[urow[i]] for i in range(2 ** R)) for j in range(2 ** R)]
    ch = [B[j] @ uh[j] for j in range(2 ** R)]
    c = np.zeros_like(u)
    for i in range(2 ** R):
        c[urow[i]] = sum(sign[j, i] * ch[j] for j in range(2 ** R))
    assert np.abs(c - St @ u).max() < 1e-13 * np.abs(St @ u).max()
