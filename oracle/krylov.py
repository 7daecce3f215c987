"""Outer Krylov solvers (oracle; test infrastructure).

The paper accelerates its preconditioned iteration with BiCGStab (Section 3);
the configured workloads' outer solver is GMRES(m): x0 = 0, modified Gram-Schmidt
Arnoldi on A M^{-1}, Givens rotations, inner exit when the implicit residual
drops below tol ||b||, x += M^{-1}(V y) at the end of each cycle, and the
explicit residual ||b - A x|| / ||b|| < tol (the stopping rule of Section
5.1) as the convergence test at every restart.  bicgstab() is the paper's
method, right-preconditioned (van der Vorst's recurrences), with the same
explicit-residual acceptance.
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


class BicgstabResult:
    def __init__(self, x, iters, rel_res, converged, restarts, history):
        self.x, self.iters, self.rel_res, self.converged = x, iters, rel_res, converged
        self.restarts, self.history = restarts, history


def bicgstab(apply_A, apply_M, b, tol=1e-8, max_iters=1000):
    """Right-preconditioned BiCGStab from x0 = 0 for A x = b (Section 3).

    One iteration applies the preconditioner and the operator twice.  The
    recurrence residual r is tested after each half step; when it is below
    tol ||b|| the explicit residual b - A x decides, and a failed test
    restarts the recurrences from the explicit residual (shadow vector =
    that residual).  Returns iterations (full steps; a convergence at the
    half step counts as one)."""
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return BicgstabResult(x, 0, 0.0, True, 0, [])
    r = b.copy()
    iters, restarts, history = 0, 0, []
    while iters < max_iters:
        rhat = r.copy()
        rho_prev = alpha = omega = 1.0
        v = np.zeros(n)
        p = np.zeros(n)
        restart = False
        while iters < max_iters:
            rho = float(rhat @ r)
            if rho == 0.0:
                restart = True
                break
            beta = (rho / rho_prev) * (alpha / omega)
            p = r + beta * (p - omega * v)
            phat = apply_M(p)
            v = apply_A(phat)
            alpha = rho / float(rhat @ v)
            s = r - alpha * v
            iters += 1
            if float(np.linalg.norm(s)) / bnorm < tol:
                x = x + alpha * phat
                r = s
                break
            shat = apply_M(s)
            t = apply_A(shat)
            omega = float(t @ s) / float(t @ t)
            x = x + alpha * phat + omega * shat
            r = s - omega * t
            rho_prev = rho
            history.append(float(np.linalg.norm(r)) / bnorm)
            if history[-1] < tol or omega == 0.0:
                break
        # acceptance by the explicit residual
        r = b - apply_A(x)
        rel = float(np.linalg.norm(r)) / bnorm
        if rel < tol:
            return BicgstabResult(x, iters, rel, True, restarts, history)
        restarts += 1
    rel = float(np.linalg.norm(b - apply_A(x))) / bnorm
    return BicgstabResult(x, iters, rel, False, restarts, history)
