"""Detector response and its gradient by the adjoint method (oracle; test
infrastructure only).

R(sigma_t, sigma_s) = w . phi with A phi = b, A = L - S at the full scatter
order.  With A^T lambda = w, dR/dp = -lambda^T (dA/dp) phi, and per cell j:
  dA/dsigma_{t,j} = N (x) M_q on every (j, q) block  (removal term, eq. complete)
  dA/dsigma_{s,j} = -N (x) S~ on cell j's blocks      (scatter, Section 5.2)
so
  dR/dsigma_{t,j} = -sum_q lambda_{jq}^T (N (x) M_q) phi_{jq}
  dR/dsigma_{s,j} = +lambda_j^T (N (x) S~) phi_j.
"""
import numpy as np

from .krylov import gmres


def gradients(level, lam, phi):
    """Per-cell contractions of lambda and phi with dA/dsigma_t, dA/dsigma_s."""
    g = level.grid
    lb = level.blocks(lam)
    pb = level.blocks(phi)
    gt = np.zeros(g.C)
    for q in range(level.P):
        gt -= np.einsum('ca,ab,cb->c', lb[q], level.K_mass[q], pb[q])
    x = phi.reshape(level.A, g.C, g.ns)
    z = (level.Stilde @ x.reshape(level.A, g.S)).reshape(level.A, g.C, g.ns)
    z = np.einsum('acj,lj->acl', z, g.N)
    gs = np.einsum('acl,acl->c', lam.reshape(level.A, g.C, g.ns), z)
    return gt, gs


def solve_adjoint(level, mg, w, tol=1e-8, m=10, max_restarts=200):
    """lambda = A^{-T} w with GMRES preconditioned by the adjoint V-cycle."""
    return gmres(level.apply_AT, lambda r: mg.vcycle(r, adjoint=True), w, tol, m, max_restarts)


def response_and_gradient(level, mg, b, w, tol=1e-8, m=10, max_restarts=200):
    fwd = gmres(level.apply_A, mg.vcycle, b, tol, m, max_restarts)
    adj = solve_adjoint(level, mg, w, tol, m, max_restarts)
    gt, gs = gradients(level, adj.x, fwd.x)
    return float(w @ fwd.x), gt, gs, fwd, adj
