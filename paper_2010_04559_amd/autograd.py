"""Detector response R(sigma_t, sigma_s) = w . A(sigma)^{-1} b as a torch
autograd function.

The forward pass is a GMRES solve of the discrete transport system; the
backward pass is the adjoint solve A^T lambda = w followed by the per-cell
contractions of the derivative of A with respect to each cell's cross
sections (A is affine in sigma_t and sigma_s):

    dR/dsigma_t[j] = -sum_q lambda_jq^T (N (x) M_q) phi_jq
    dR/dsigma_s[j] = +lambda_j^T (N (x) S~) phi_j

both computed by the library (tr_adjoint_grad), and R = w . phi itself
(tr_response).  R is linear in b and in w: dR/db = lambda (the adjoint
solution, A^T lambda = w) and dR/dw = phi, returned when those inputs
require gradients.
"""
import torch

from .transport import Transport


class DetectorResponse(torch.autograd.Function):
    """R = DetectorResponse.apply(tr, sigma_t, sigma_s, b, w, mode, tol).

    tr: a Transport handle (its cross sections are replaced by the inputs);
    sigma_t, sigma_s: [cells] float64 CUDA tensors; b: right-hand side and
    w: detector weights, both canonical float64 CUDA vectors; mode: the
    preconditioner precision ("f64" or "mixed"); tol: GMRES tolerance (the
    gradient is as accurate as the two solves).
    """

    @staticmethod
    def forward(ctx, tr: Transport, sigma_t, sigma_s, b, w, mode="f64", tol=1e-10):
        tr.set_sigma(sigma_t.detach(), sigma_s.detach())
        x, st = tr.solve(b, tol=tol, mode=mode)
        ctx.tr, ctx.mode, ctx.tol = tr, mode, tol
        ctx.save_for_backward(sigma_t, sigma_s, w, x)
        ctx.stats = st
        return torch.tensor(tr.response(w, x), dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, grad_out):
        sigma_t, sigma_s, w, x = ctx.saved_tensors
        tr = ctx.tr
        # another forward call may have replaced the handle's cross sections
        tr.set_sigma(sigma_t.detach(), sigma_s.detach())
        gt, gs, lam, _ = tr.adjoint_grad(w, x, tol=ctx.tol, mode=ctx.mode)
        gb = grad_out * lam if ctx.needs_input_grad[3] else None
        gw = grad_out * x if ctx.needs_input_grad[4] else None
        return None, grad_out * gt, grad_out * gs, gb, gw, None, None


def detector_response(tr: Transport, sigma_t, sigma_s, b, w, mode="f64", tol=1e-10):
    """Functional form of DetectorResponse.apply."""
    return DetectorResponse.apply(tr, sigma_t, sigma_s, b, w, mode, tol)
