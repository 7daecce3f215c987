"""The discrete transport problem on one angular mesh (oracle; test
infrastructure only).

Unknowns phi_{[j,q]}^{i,d} (eq. Expansion) are stored flat with index
a * S + j * ns + i, a = nd q + d the angular dof (patch-major; nd = 3 for
the Lin basis, 1 for Const), j the cell, i the spatial node.  A (j,q)
block is ordered (d, i) -> d * ns + i, so an angular factor A and a
spatial factor F combine as kron(A, F).

The weak form is eq. complete with eq. Surface_Integral: face streaming
term, volume streaming term -sum_xi V_xi (x) A^xi, removal N (x) M, and the
source.  Readings (listed in the design notes):
  * removal uses Sigma_t (eq. LBE), the scatter source includes n = 0;
  * the numerical flux is full upwinding: on the Cartesian mesh every patch
    lies inside one octant, so Omega^xi has one sign s_xi on the whole patch
    and each face is wholly inflow or outflow for it; inflow faces take the
    neighbour's trace of the same patch (or the boundary data), so the
    explicit part L_E of the Section 3 split vanishes and the sweep is an
    exact inverse of L;
  * the scatter operator is S = sigma_s N (x) S~ with S~ of Section 5.2.
"""
import numpy as np

from . import angular as ang


class Level:
    """Transport operator L, scatter operator S and source terms on the
    angular mesh ``patches`` for a Cartesian ``grid``."""

    def __init__(self, grid, patches, sigma_t, sigma_s, moments, rule=None, basis="lin"):
        self.grid = grid
        self.patches = patches
        self.basis = basis
        self.nd = ang.basis_dofs(basis)
        self.P = len(patches)
        self.A = self.nd * self.P
        self.sigma_t = np.asarray(sigma_t, dtype=np.float64)
        self.sigma_s = np.asarray(sigma_s, dtype=np.float64)
        self.moments = np.asarray(moments, dtype=np.float64)
        self.rule = ang.PatchRule(patches, rule, basis)
        self.signs = [ang.octant_signs(p.octant) for p in patches]
        d, ns = grid.dim, grid.ns
        self.Mq = [self.rule.mass(q) for q in range(self.P)]
        self.Aq = [[self.rule.jacobian(q, xi) for xi in range(3)] for q in range(self.P)]
        self.Stilde = ang.scatter_matrix(patches, self.moments, basis)
        self.K_stream, self.K_mass, self.couple = [], [], []
        for q in range(self.P):
            K = np.zeros((self.nd * ns, self.nd * ns))
            cpl = []
            for xi in range(d):
                Ax = self.Aq[q][xi]
                s = self.signs[q][xi]
                out_side, in_side = (1, 0) if s > 0 else (0, 1)
                sigma_out = 1.0 if out_side == 1 else -1.0
                sigma_in = -sigma_out
                # outflow face: own trace; volume term with the test gradient
                K += sigma_out * np.kron(Ax, grid.F[xi][out_side])
                K -= np.kron(Ax, grid.V[xi])
                # inflow face: neighbour's trace (coupling, moved to the RHS in a sweep)
                cpl.append((xi, in_side, sigma_in * np.kron(Ax, grid.Fn[xi][in_side])))
            self.K_stream.append(K)
            self.K_mass.append(np.kron(self.Mq[q], grid.N))
            self.couple.append(cpl)
        self.nbr = {(xi, side): grid.neighbour(xi, side) for xi in range(d) for side in (0, 1)}

    # --------------------------------------------------------- layouts
    def blocks(self, x):
        """flat (A*S,) -> (P, C, nd*ns) per-(cell, patch) blocks."""
        g, nd = self.grid, self.nd
        return x.reshape(self.P, nd, g.C, g.ns).transpose(0, 2, 1, 3).reshape(self.P, g.C, nd * g.ns)

    def flat(self, b):
        g, nd = self.grid, self.nd
        return b.reshape(self.P, g.C, nd, g.ns).transpose(0, 2, 1, 3).reshape(-1).copy()

    # --------------------------------------------------------- operators
    def apply_L(self, x):
        """y = L x (homogeneous inflow)."""
        xb = self.blocks(x)
        yb = np.empty_like(xb)
        for q in range(self.P):
            y = xb[q] @ self.K_stream[q].T + self.sigma_t[:, None] * (xb[q] @ self.K_mass[q].T)
            for xi, side, Cm in self.couple[q]:
                nb = self.nbr[(xi, side)]
                ok = nb >= 0
                y[ok] += xb[q][nb[ok]] @ Cm.T
            yb[q] = y
        return self.flat(yb)

    def apply_LT(self, x):
        """y = L^T x."""
        xb = self.blocks(x)
        yb = np.empty_like(xb)
        for q in range(self.P):
            y = xb[q] @ self.K_stream[q] + self.sigma_t[:, None] * (xb[q] @ self.K_mass[q])
            for xi, side, Cm in self.couple[q]:
                nb = self.nbr[(xi, side)]
                ok = nb >= 0
                # row (nb, q) of L holds Cm against column (j, q); transpose it
                np.add.at(y, nb[ok], xb[q][ok] @ Cm)
            yb[q] = y
        return self.flat(yb)

    def apply_S(self, x):
        """y = S x = sigma_s N (x) S~ x (Section 5.2, discrete source)."""
        g = self.grid
        z = (self.Stilde @ x.reshape(self.A, g.S)).reshape(self.A, g.C, g.ns)
        z = np.einsum('acj,lj->acl', z, g.N)
        return (z * self.sigma_s[None, :, None]).reshape(-1)

    def apply_ST(self, x):
        g = self.grid
        z = np.einsum('acl,lj->acj', x.reshape(self.A, g.C, g.ns) * self.sigma_s[None, :, None], g.N)
        return (self.Stilde.T @ z.reshape(self.A, g.S)).reshape(-1)

    def apply_A(self, x):
        return self.apply_L(x) - self.apply_S(x)

    def apply_AT(self, x):
        return self.apply_LT(x) - self.apply_ST(x)

    def sweep(self, g_rhs):
        """phi = L^{-1} g: octant by octant, cells in upwind plane order, one
        coupled (nd ns) x (nd ns) local solve per (cell, patch) (Section 3)."""
        gb = self.blocks(g_rhs)
        phi = np.zeros_like(gb)
        for o in range(8):
            Q = [q for q in range(self.P) if self.patches[q].octant == o]
            if not Q:
                continue
            for J in self.grid.sweep_planes(ang.octant_signs(o)):
                for q in Q:
                    K = self.K_stream[q][None] + self.sigma_t[J][:, None, None] * self.K_mass[q][None]
                    rhs = gb[q][J].copy()
                    for xi, side, Cm in self.couple[q]:
                        nb = self.nbr[(xi, side)][J]
                        ok = nb >= 0
                        rhs[ok] -= phi[q][nb[ok]] @ Cm.T
                    phi[q][J] = np.linalg.solve(K, rhs[..., None])[..., 0]
        return self.flat(phi)

    def sweep_T(self, g_rhs):
        """lambda = L^{-T} g: the transposed blocks, visited downwind first."""
        gb = self.blocks(g_rhs)
        lam = np.zeros_like(gb)
        for o in range(8):
            Q = [q for q in range(self.P) if self.patches[q].octant == o]
            if not Q:
                continue
            for J in reversed(self.grid.sweep_planes(ang.octant_signs(o))):
                for q in Q:
                    K = self.K_stream[q][None] + self.sigma_t[J][:, None, None] * self.K_mass[q][None]
                    KT = np.swapaxes(K, 1, 2)
                    rhs = gb[q][J].copy()
                    for xi, side, Cm in self.couple[q]:
                        # cells whose upwind neighbour across (xi, side) is in J
                        other = 1 - side
                        down = self.nbr[(xi, other)][J]
                        ok = down >= 0
                        rhs[ok] -= lam[q][down[ok]] @ Cm
                    lam[q][J] = np.linalg.solve(KT, rhs[..., None])[..., 0]
        return self.flat(lam)

    # --------------------------------------------------------- sources
    def basis_integral(self):
        """int_{D_q} psi_{q,m} for every angular dof, shape (A,)."""
        return np.concatenate([self.rule.basis_integral(q) for q in range(self.P)])

    def rhs_volume(self, q_cell):
        """Isotropic volume source Q = q_j (per steradian) in cell j."""
        g = self.grid
        b = np.einsum('a,c,l->acl', self.basis_integral(), np.asarray(q_cell, float), g.basis_int)
        return b.reshape(-1)

    def _face_cells(self, xi, side, lo, hi):
        g = self.grid
        c = g.coords
        ok = c[:, xi] == (0 if side == 0 else g.n[xi] - 1)
        for a in range(g.dim):
            if a != xi:
                ok &= (c[:, a] >= lo[a]) & (c[:, a] <= hi[a])
        return np.nonzero(ok)[0]

    def rhs_inflow_iso(self, xi, side, lo, hi, value):
        """Isotropic inflow phi_in = value on boundary face (xi, side) for the
        cells of the face box: the inflow part of the face term of eq.
        complete moved to the right-hand side."""
        g = self.grid
        b = np.zeros((self.A, g.C, g.ns))
        cells = self._face_cells(xi, side, lo, hi)
        sigma_f = -1.0 if side == 0 else 1.0
        fi = g.face_int[xi][side]
        for q in range(self.P):
            if sigma_f * self.signs[q][xi] >= 0:
                continue
            sel = self.rule.owner == q
            om_psi = self.rule.psi[q].T @ (self.rule.w[sel] * self.rule.omega[sel, xi])
            for m in range(self.nd):
                b[self.nd * q + m][cells] += -sigma_f * value * om_psi[m] * fi[None, :]
        return b.reshape(-1)

    def rhs_beam(self, direction, xi, side, lo, hi, current=1.0):
        """Dirac beam in space-angle entering through face (xi, side): unit
        current per area in ``direction``.  The angular Dirac is split
        equally over every patch whose closure contains the direction (the
        Lin functions' values there; the Const function is 1)."""
        g = self.grid
        d = np.asarray(direction, float)
        d = d / np.linalg.norm(d)
        hits = []
        for q, p in enumerate(self.patches):
            if np.dot(self.signs[q], d) <= 1e-14:
                continue
            lam = ang.lin_basis(p, d[None, :])[0]
            if (lam >= -1e-12).all():
                hits.append((q, lam if self.nd == 3 else np.ones(1)))
        b = np.zeros((self.A, g.C, g.ns))
        cells = self._face_cells(xi, side, lo, hi)
        fi = g.face_int[xi][side]
        for q, lam in hits:
            for m in range(self.nd):
                b[self.nd * q + m][cells] += current * lam[m] / len(hits) * fi[None, :]
        return b.reshape(-1)

    def detector_weights(self, lo, hi):
        """Weights w with R = w . phi = integrated scalar flux over a cell box."""
        g = self.grid
        mask = np.zeros(g.C)
        mask[g.box_cells(lo, hi)] = 1.0
        return np.einsum('a,c,l->acl', self.basis_integral(), mask, g.basis_int).reshape(-1)

    def scalar_flux_cell_avg(self, phi):
        """Cell-average scalar flux: int_{V_j} int_4pi phi / |V_j|."""
        g = self.grid
        x = phi.reshape(self.A, g.C, g.ns)
        tot = np.einsum('a,acl,l->c', self.basis_integral(), x, g.basis_int)
        return tot / np.prod(g.h)

    def dense(self, op):
        """Explicit matrix of a linear map (tiny meshes only)."""
        n = self.A * self.grid.S
        M = np.zeros((n, n))
        e = np.zeros(n)
        for k in range(n):
            e[k] = 1.0
            M[:, k] = op(e)
            e[k] = 0.0
        return M
