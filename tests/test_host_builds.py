"""Host (CPU) builds of the library's own code, checked against the oracle:

* the per-cell ordinate solve of local_solve.h (compiled with g++): for
  every orientation in 2-D and 3-D, forward and transposed, it inverts the
  ordinate block of the weak form built from the oracle's spatial DG
  matrices, K = sum_xi (|Omega_xi| F_out,xi - Omega_xi V_xi) + sigma N (the
  forward sweep receives the prepared right-hand side N^-1 g, the adjoint
  applies N^-1 after its transposed solve);
* the angular setup (angular_setup.cpp), built with the address and
  undefined-behaviour sanitizers: meshes, ordinates, weights, basis
  integrals, prolongation blocks and the scatter matrix against the oracle's
  own (independent) construction.
"""
import ctypes
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from oracle import angular as ang
from oracle import spatial as sp

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2010_04559_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def ls_lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("host") / "ls.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", out,
                    os.path.join(HERE, "host", "local_solve_shim.cpp")], check=True)
    lib = ctypes.CDLL(out)
    for fn in (lib.ls_solve, lib.ls_spectral):
        fn.restype = None
        fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                       ctypes.POINTER(ctypes.c_double), ctypes.c_double]
    return lib


def _ordinate_block(dim, h, omega, sigma):
    grid = sp.Grid(dim, (1,) * dim, h)
    K = sigma * grid.N
    for xi in range(dim):
        out = 1 if omega[xi] > 0 else 0
        K = K + abs(omega[xi]) * grid.F[xi][out] - omega[xi] * grid.V[xi]
    return K, grid


@pytest.mark.parametrize("dim", [2, 3])
def test_local_solve_inverts_the_oracle_block(ls_lib, dim):
    rng = np.random.default_rng(dim)
    ns = 2 ** dim
    for flip in range(2 ** dim):
        for trial in range(4):
            h = tuple(rng.uniform(0.02, 0.5, dim))
            om = rng.uniform(0.05, 1.0, 3)
            om /= np.linalg.norm(om)
            om = np.array([-om[d] if (flip >> d) & 1 else om[d] for d in range(3)])
            sigma = float(rng.uniform(0.0, 30.0) if trial else 0.0)
            K, grid = _ordinate_block(dim, h, om[:dim], sigma)
            c = np.zeros(3)
            c[:dim] = np.abs(om[:dim]) / np.array(h)
            cp = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            g = rng.standard_normal(ns)
            vol = float(np.prod(h))
            for fn in (ls_lib.ls_solve, ls_lib.ls_spectral):
                # forward: the sweep receives N^-1 g
                v = np.linalg.solve(grid.N, g)
                fn(dim, 0, flip, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cp, sigma)
                want = np.linalg.solve(K, g)
                assert np.abs(v - want).max() < 1e-12 * np.abs(want).max(), (flip, trial)
                # transposed: solve, then the inverse mass shape and 1 / vol
                v = g.copy()
                fn(dim, 1, flip, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cp, sigma)
                v /= vol
                want = np.linalg.solve(K.T, g)
                assert np.abs(v - want).max() < 1e-12 * np.abs(want).max(), (flip, trial, "T")


@pytest.fixture(scope="module")
def setup_dump(tmp_path_factory):
    d = tmp_path_factory.mktemp("setup")
    exe = str(d / "setup_dump")
    # host-only code: the sanitizers instrument it completely
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-o", exe, os.path.join(HERE, "host", "setup_dump.cpp"),
                    os.path.join(CSRC, "angular_setup.cpp")], check=True)
    return exe, d


def test_band_meshes_match_the_paper_counts(setup_dump):
    """Section 5.5: the z-band rule gives 20, 32, 44, 128, 440, 1388
    elements for l_max = 1..6 (tests/golden/band_mesh_counts.txt)."""
    rows = [tuple(int(v) for v in line.split()) for line in open(os.path.join(HERE, "golden", "band_mesh_counts.txt"))
            if line.strip() and not line.startswith("#")]
    for lmax, count in rows:
        levels, _ = _run_dump(setup_dump, (0, 0, 0, 1, 0, 0, 0, lmax, 0, 0.5, 0))
        assert levels[-1]["P"] == count, (lmax, levels[-1]["P"])
        assert len(levels) == lmax + 1


def _run_dump(setup_dump, args):
    exe, d = setup_dump
    out = str(d / ("t_%d.bin" % abs(hash(tuple(args)))))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([exe] + [str(a) for a in args] + [out], capture_output=True, text=True, env=env)
    assert res.returncode == 0, res.stderr[-3000:]
    raw = open(out, "rb").read()
    arrays, pos = [], 0
    while pos < len(raw):
        n = int(struct.unpack_from("d", raw, pos)[0])
        pos += 8
        arrays.append(np.frombuffer(raw, dtype=np.float64, count=n, offset=pos).copy())
        pos += 8 * n
    nlev = int(arrays[0][0])
    levels, k = [], 1
    for _ in range(nlev):
        P = int(arrays[k][0])
        verts, omega, w, ipsi, iom, owner, pblk = arrays[k + 1:k + 8]
        levels.append(dict(P=P, verts=verts.reshape(P, 3, 3), omega=omega.reshape(-1, 3), w=w, ipsi=ipsi,
                           iom=iom.reshape(-1, 3), owner=owner.astype(int), pblk=pblk.reshape(-1, 3, 3)))
        k += 8
    St = arrays[k]
    return levels, St


@pytest.mark.parametrize("spec", [(2, 0, 0, 1, 0, 0, 1, 0, 8, 0.9), (1, 1, 0, 0, 15.0, 2, 1, 0, 6, 0.85),
                                  (1, 0.3, 0.5, 0.81, 25.0, 2, 1, 0, 4, 0.8), (0, 0, 0, 1, 0, 0, 0, 3, 6, 0.9)])
def test_setup_tables_match_oracle(setup_dump, spec):
    base, cx, cy, cz, half, extra, closure, band, order, g = spec
    levels, St = _run_dump(setup_dump, spec + (0,))
    if band:
        mesh = ang.AngularMesh.band_z(band)
    elif extra:
        mesh = ang.AngularMesh.cone((cx, cy, cz), half, base, extra, closure=bool(closure))
    else:
        mesh = ang.AngularMesh.uniform(base)
    T = mesh.levels()
    assert [L["P"] for L in levels] == [len(t) for t in T]
    for l, (L, patches) in enumerate(zip(levels, T)):
        overts = np.array([p.verts for p in patches])
        assert np.abs(L["verts"] - overts).max() < 1e-15
        rule = ang.PatchRule(patches)
        assert np.abs(L["omega"] - rule.omega).max() < 1e-14
        assert np.abs(L["w"] - rule.w).max() < 1e-14 * rule.w.max()
        ipsi = np.concatenate([rule.basis_integral(q) for q in range(len(patches))])
        assert np.abs(L["ipsi"] - ipsi).max() < 1e-14
        for xi in range(3):
            iom = np.concatenate([rule.psi[q].T @ (rule.w[rule.owner == q] * rule.omega[rule.owner == q, xi])
                                  for q in range(len(patches))])
            assert np.abs(L["iom"][:, xi] - iom).max() < 1e-14
        if l > 0:
            P = ang.prolongation(T[l - 1], patches)
            for c in range(len(patches)):
                p = L["owner"][c]
                assert np.abs(P[3 * c:3 * c + 3, 3 * p:3 * p + 3] - L["pblk"][c]).max() < 1e-14
                others = np.delete(P[3 * c:3 * c + 3], np.s_[3 * p:3 * p + 3], axis=1)
                assert not others.any()
    ref = ang.scatter_matrix(T[-1], ang.hg_moments(g, order))
    A = ref.shape[0]
    assert np.abs(St.reshape(A, A) - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("spec", [(1, 0, 0, 1, 0, 0, 1, 0, 6, 0.9), (1, 1, 0, 0, 15.0, 2, 1, 0, 4, 0.85),
                                  (0, 0, 0, 1, 0, 0, 0, 2, 5, 0.8)])
def test_const_setup_tables_match_oracle(setup_dump, spec):
    """The Const basis carried as three coincident ordinates: each patch's
    ordinates are the oracle's mean direction int_q Omega / |q| with a third
    of |q| each, its X rows a third of int_q Y (so S~ is the oracle's Const
    scatter matrix over 9 in every 3x3 block), and a daughter's
    prolongation block is J / 3 (the parent's value in all three)."""
    base, cx, cy, cz, half, extra, closure, band, order, g = spec
    levels, St = _run_dump(setup_dump, spec + (1,))
    if band:
        mesh = ang.AngularMesh.band_z(band)
    elif extra:
        mesh = ang.AngularMesh.cone((cx, cy, cz), half, base, extra, closure=bool(closure))
    else:
        mesh = ang.AngularMesh.uniform(base)
    T = mesh.levels()
    for l, (L, patches) in enumerate(zip(levels, T)):
        rule = ang.PatchRule(patches, basis="const")
        for q in range(len(patches)):
            area = rule.mass(q)[0, 0]
            mean = np.array([rule.jacobian(q, xi)[0, 0] for xi in range(3)]) / area
            for k in range(3):
                assert np.abs(L["omega"][3 * q + k] - mean).max() < 1e-14
                assert abs(L["w"][3 * q + k] - area / 3) < 1e-14 * area
                assert abs(L["ipsi"][3 * q + k] - area / 3) < 1e-14 * area
                assert np.abs(L["iom"][3 * q + k] - mean * area / 3).max() < 1e-14
        if l > 0:
            for c in range(len(patches)):
                blk = L["pblk"][c]
                assert np.allclose(blk, np.full((3, 3), 1 / 3), rtol=0, atol=1e-15) or np.allclose(blk, np.eye(3))
    ref = ang.scatter_matrix(T[-1], ang.hg_moments(g, order), basis="const")
    A = 3 * len(T[-1])
    assert np.abs(St.reshape(A, A) - np.kron(ref, np.ones((3, 3))) / 9).max() < 1e-13 * np.abs(ref).max()
