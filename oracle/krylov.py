"""Restarted right-preconditioned GMRES(m) (oracle; test infrastructure).

The paper accelerates its preconditioned iteration with BiCGStab (Section 3);
this build's outer solver is GMRES(m): x0 = 0, modified Gram-Schmidt Arnoldi
on A M^{-1}, Givens rotations, inner exit when the implicit residual drops
below tol ||b||, x += M^{-1}(V y) at the end of each cycle, and the explicit
residual ||b - A x|| / ||b|| < tol (the stopping rule of Section 5.1) as the
convergence test at every restart.
"""
import math
import numpy as np


class GmresResult:
    def __init__(self, x, iters, restarts, rel_res, converged, history):
        self.x, self.iters, self.restarts = x, iters, restarts
        self.rel_res, self.converged, self.history = rel_res, converged, history


def gmres(apply_A, apply_M, b, tol=1e-8, m=10, max_restarts=200):
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return GmresResult(x, 0, 0, 0.0, True, [])
    r = b.copy()
    iters = 0
    history = []
    for cycle in range(max_restarts + 1):
        beta = float(np.linalg.norm(r))
        history.append(beta / bnorm)
        if beta / bnorm < tol:
            return GmresResult(x, iters, cycle, beta / bnorm, True, history)
        if cycle == max_restarts:
            break
        V = [r / beta]
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        gvec = np.zeros(m + 1)
        gvec[0] = beta
        k = 0
        for j in range(m):
            w = apply_A(apply_M(V[j]))
            iters += 1
            for i in range(j + 1):
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / rho, H[j + 1, j] / rho
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V.append(w / H[j + 1, j])
            H[j, j] = rho
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            k = j + 1
            if abs(gvec[j + 1]) / bnorm < tol or breakdown:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (gvec[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        upd = np.zeros(n)
        for i in range(k):
            upd += y[i] * V[i]
        x = x + apply_M(upd)
        r = b - apply_A(x)
    rel = float(np.linalg.norm(r)) / bnorm
    return GmresResult(x, iters, max_restarts, rel, False, history)
