"""Angular multigrid preconditioner (oracle; test infrastructure only).

Section 4 and Fig. lmg: the recursive linear V-cycle LMG(phi_l, f_l, l) with
source-iteration smoothing L_l phi^{k+1} = S_l phi^k + f_l, restriction
R = P^T, Galerkin prolongation P between the nested angular spaces (Lin or
Const basis), coarse
operators by direct rediscretisation on T_l (DCA), and on T_0 the block
Gauss-Seidel sweep of Section 5.2: every (cell, patch) block is solved with
its own scatter coupling implicit and all other unknowns at their latest
values, octant by octant and cell by cell in the order of the standard
sweep, nu_coarse sweeps from zero.

Readings (listed in the design notes):
  * the scatter order of each level is a per-level schedule ``orders``
    (coarsest level first) -- Section 5.3 lowers it in the preconditioner;
  * the coarse solve is a fixed number (default 10) of Gauss-Seidel sweeps,
    so the preconditioner is a fixed linear map;
  * octants are visited in id order 0..7 unless ``octant_order`` is given;
  * the adjoint preconditioner is the same cycle built from the transposed
    level operators: transposed sweeps, S^T, and the Gauss-Seidel sweep on
    A_0^T visiting each octant's cells downwind first.
"""
import numpy as np

from . import angular as ang
from .transport import Level


class AngularMG:
    def __init__(self, grid, mesh, sigma_t, sigma_s, moments, orders,
                 nu_pre=1, nu_post=1, nu_coarse=10, octant_order=tuple(range(8)),
                 rule=None, basis="lin"):
        self.grid = grid
        self.T = mesh.levels()
        self.nlev = len(self.T)
        if len(orders) != self.nlev:
            raise ValueError("one scatter order per level T_0..T_L is required")
        moments = np.asarray(moments, dtype=np.float64)
        self.levels = [Level(grid, self.T[l], sigma_t, sigma_s, moments[:orders[l] + 1], rule, basis)
                       for l in range(self.nlev)]
        self.P = [None] + [ang.prolongation(self.T[l - 1], self.T[l], basis) for l in range(1, self.nlev)]
        self.nu_pre, self.nu_post, self.nu_coarse = nu_pre, nu_post, nu_coarse
        self.octant_order = tuple(octant_order)

    # ------------------------------------------------------- transfers
    def prolong(self, l, xc):
        """Fine-level (T_l) coefficients of a T_{l-1} function."""
        S = self.grid.S
        return (self.P[l] @ xc.reshape(-1, S)).reshape(-1)

    def restrict(self, l, rf):
        """R = P^T applied to a T_l (weak-form) residual."""
        S = self.grid.S
        return (self.P[l].T @ rf.reshape(-1, S)).reshape(-1)

    # ------------------------------------------------------- coarse GS
    def coarse_gs(self, f, nu=None, adjoint=False):
        """Block Gauss-Seidel on T_0 (Section 5.2), ``nu`` sweeps from zero."""
        nu = self.nu_coarse if nu is None else nu
        lv = self.levels[0]
        g = self.grid
        ns, nd = g.ns, lv.nd
        fb = lv.blocks(f)
        phi = np.zeros_like(fb)
        St = lv.Stilde
        for _ in range(nu):
            for o in self.octant_order:
                Q = [q for q in range(lv.P) if lv.patches[q].octant == o]
                planes = g.sweep_planes(ang.octant_signs(o))
                if adjoint:
                    planes = planes[::-1]
                for J in planes:
                    for q in Q:
                        self_sc = np.kron(St[nd * q:nd * q + nd, nd * q:nd * q + nd], g.N)
                        K = (lv.K_stream[q][None] + lv.sigma_t[J][:, None, None] * lv.K_mass[q][None]
                             - lv.sigma_s[J][:, None, None] * self_sc[None])
                        rhs = fb[q][J].copy()
                        for p in range(lv.P):
                            if p == q:
                                continue
                            blk = np.kron(St[nd * q:nd * q + nd, nd * p:nd * p + nd], g.N)
                            if adjoint:
                                blk = np.kron(St[nd * p:nd * p + nd, nd * q:nd * q + nd], g.N).T
                            rhs += lv.sigma_s[J][:, None] * (phi[p][J] @ blk.T)
                        for xi, side, Cm in lv.couple[q]:
                            if not adjoint:
                                nb = lv.nbr[(xi, side)][J]
                                ok = nb >= 0
                                rhs[ok] -= phi[q][nb[ok]] @ Cm.T
                            else:
                                down = lv.nbr[(xi, 1 - side)][J]
                                ok = down >= 0
                                rhs[ok] -= phi[q][down[ok]] @ Cm
                        if adjoint:
                            K = np.swapaxes(K, 1, 2)
                        phi[q][J] = np.linalg.solve(K, rhs[..., None])[..., 0]
        return lv.flat(phi)

    # ------------------------------------------------------- V-cycle
    def _smooth(self, lv, phi, f, nu, adjoint):
        for _ in range(nu):
            if adjoint:
                phi = lv.sweep_T(lv.apply_ST(phi) + f)
            else:
                phi = lv.sweep(lv.apply_S(phi) + f)
        return phi

    def lmg(self, f, l, adjoint=False):
        """LMG(0, f_l, l) of Fig. lmg; returns phi_l."""
        if l == 0:
            return self.coarse_gs(f, adjoint=adjoint)
        lv = self.levels[l]
        phi = np.zeros_like(f)
        phi = self._smooth(lv, phi, f, self.nu_pre, adjoint)
        r = f - (lv.apply_AT(phi) if adjoint else lv.apply_A(phi))
        fc = self.restrict(l, r)
        phic = self.lmg(fc, l - 1, adjoint)
        phi = phi + self.prolong(l, phic)
        phi = self._smooth(lv, phi, f, self.nu_post, adjoint)
        return phi

    def vcycle(self, r, adjoint=False):
        """Preconditioner M^{-1} r = LMG(0, r, L)."""
        return self.lmg(r, self.nlev - 1, adjoint)
