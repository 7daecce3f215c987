"""Spatial DG discretisation on a Cartesian mesh (oracle; test infrastructure).

Section 2.3 defines the element integrals N (mass), V (volume streaming,
gradient on the test function) and the face integrals of the streaming term.
The paper leaves the spatial order open; the reading used throughout is the
nodal Q1 (bilinear in 2-D, trilinear in 3-D) Lagrange basis on each cell,
with nodes at the cell vertices, local node index b = bx + 2 by (+ 4 bz).

Cell index j = ix + nx (iy + ny iz); the domain is [0, len_x] x [0, len_y]
(x [0, len_z]).
"""
import numpy as np


def mass_1d(h):
    """int_0^h l_a l_b for the two linear Lagrange functions."""
    return h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])


# int_0^h l_a' l_b (derivative on the test function), independent of h
DERIV_1D = np.array([[-0.5, -0.5], [0.5, 0.5]])
# values of (l_0, l_1) at the left (0) and right (h) end of the cell
TRACE_1D = (np.array([1.0, 0.0]), np.array([0.0, 1.0]))


def kron_nodes(factors):
    """Tensor product of per-axis 2x2 factors, axis 0 (x) fastest."""
    out = factors[0]
    for f in factors[1:]:
        out = np.kron(f, out)
    return out


class Grid:
    """Uniform Cartesian mesh with ``n[xi]`` cells of width ``h[xi]``."""

    def __init__(self, dim, n, length=None):
        self.dim = dim
        self.n = tuple(int(v) for v in n[:dim])
        length = length if length is not None else (1.0,) * dim
        self.length = tuple(float(v) for v in length[:dim])
        self.h = tuple(L / k for L, k in zip(self.length, self.n))
        self.ns = 2 ** dim
        self.C = int(np.prod(self.n))
        self.S = self.C * self.ns
        idx = np.arange(self.C)
        coords = []
        rem = idx
        for k in self.n:
            coords.append(rem % k)
            rem = rem // k
        self.coords = np.stack(coords, axis=1)          # (C, dim)
        self.stride = [int(np.prod(self.n[:a])) for a in range(dim)]

        M1 = [mass_1d(h) for h in self.h]
        self.N = kron_nodes(M1)
        self.V = []
        for xi in range(dim):
            f = [DERIV_1D if a == xi else M1[a] for a in range(dim)]
            self.V.append(kron_nodes(f))
        # F[xi][side]: int_face Phi_l Phi_i on the own face (side 0 = low, 1 = high)
        # Fn[xi][side]: int_face Phi_l Phi^nbr_i with the neighbour across that face
        self.F, self.Fn, self.face_int = [], [], []
        for xi in range(dim):
            fs, fns, fi = [], [], []
            for side in (0, 1):
                own = TRACE_1D[side]
                other = TRACE_1D[1 - side]
                fs.append(kron_nodes([np.outer(own, own) if a == xi else M1[a] for a in range(dim)]))
                fns.append(kron_nodes([np.outer(own, other) if a == xi else M1[a] for a in range(dim)]))
                vec = [own if a == xi else M1[a].sum(axis=1) for a in range(dim)]
                v = vec[0]
                for w in vec[1:]:
                    v = np.kron(w, v)
                fi.append(v)
            self.F.append(fs)
            self.Fn.append(fns)
            self.face_int.append(fi)
        # int_{V_j} Phi_i
        self.basis_int = self.N.sum(axis=1)

    def neighbour(self, xi, side):
        """Neighbour cell index across face (xi, side) or -1 at the boundary."""
        c = self.coords[:, xi]
        if side == 0:
            ok = c > 0
            return np.where(ok, np.arange(self.C) - self.stride[xi], -1)
        ok = c < self.n[xi] - 1
        return np.where(ok, np.arange(self.C) + self.stride[xi], -1)

    def sweep_planes(self, signs):
        """Cells grouped by upwind distance for direction signs ``signs``:
        plane k holds the cells whose oriented coordinates sum to k.  Every
        upwind neighbour of a cell lies in an earlier plane."""
        oriented = np.zeros(self.C, dtype=np.int64)
        for xi in range(self.dim):
            c = self.coords[:, xi]
            oriented += c if signs[xi] > 0 else (self.n[xi] - 1 - c)
        return [np.nonzero(oriented == k)[0] for k in range(int(oriented.max()) + 1)]

    def box_cells(self, lo, hi):
        """Cells with lo[xi] <= i_xi <= hi[xi] on every axis."""
        ok = np.ones(self.C, dtype=bool)
        for xi in range(self.dim):
            ok &= (self.coords[:, xi] >= lo[xi]) & (self.coords[:, xi] <= hi[xi])
        return np.nonzero(ok)[0]
