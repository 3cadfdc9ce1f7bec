"""Autograd wrappers: differentiate a validation loss through the NysPCG solution.

For the bilevel problem of eq. rlaopt-bilevel with the inner problem the
kernel system (K(sigma) + lambda I) x = b, the solution's sensitivities follow
from the implicit function theorem instead of unrolling the iterations:
with a = (K + lambda I)^{-1} (dL/dx) (the adjoint solve, same preconditioner),

    dL/db = a,   dL/dlambda = -a^T x,   dL/dsigma = -a^T (dK/dsigma) x.

Both the forward solve and the adjoint run in libnys (nyspcg_solve,
nyspcg_backward); the kernel products use kernel_matvec, and the explicit
sigma-term g^T (dK/dsigma) v of a product is one kernel_dot call.  The
preconditioner is held fixed (stop-gradient): the converged solution does not
depend on it.
"""
from __future__ import annotations

import torch

import paper_2609_08136_amd as nys


def _f64_scalar(t) -> float:
    return float(t.detach().cpu()) if isinstance(t, torch.Tensor) else float(t)


class KernelProduct(torch.autograd.Function):
    """y = K(Xr, Xc; sigma) v in float64.
    Backward: dL/dv = K(Xc, Xr) g and dL/dsigma = g^T (dK(Xr, Xc)/dsigma) v."""

    @staticmethod
    def forward(ctx, Xr, Xc, v, sigma, kind: int):
        s = _f64_scalar(sigma)
        out = nys.kernel_matvec(Xr, Xc, v.contiguous(), kind, s, nys.FP64)
        ctx.save_for_backward(Xr, Xc, v)
        ctx.sigma, ctx.kind = s, kind
        ctx.sigma_is_tensor = isinstance(sigma, torch.Tensor)
        return out

    @staticmethod
    def backward(ctx, g):
        Xr, Xc, v = ctx.saved_tensors
        g = g.contiguous()
        gv = gs = None
        if ctx.needs_input_grad[2]:
            gv = nys.kernel_matvec(Xc, Xr, g, ctx.kind, ctx.sigma, nys.FP64)
        if ctx.sigma_is_tensor and ctx.needs_input_grad[3]:
            gs = torch.tensor(nys.kernel_dot(Xr, Xc, g, v.contiguous(), ctx.kind, ctx.sigma, deriv=1),
                              dtype=torch.float64, device=g.device)
        return None, None, gv, gs, None


class NysPCGSolve(torch.autograd.Function):
    """x = (K(X; sigma) + lambda I)^{-1} b by NysPCG (or CG when P is None).
    Backward: the adjoint solve with the same preconditioner (nyspcg_backward)."""

    @staticmethod
    def forward(ctx, X, b, lam, sigma, kind: int, P, opts: dict):
        lam_f, sig_f = _f64_scalar(lam), _f64_scalar(sigma)
        x, info, rc = nys.nyspcg_solve(X, b.contiguous(), [lam_f], kind, sig_f, P, **opts)
        x = x.reshape(-1)
        ctx.save_for_backward(X, x)
        ctx.lam, ctx.sigma, ctx.kind, ctx.P, ctx.opts = lam_f, sig_f, kind, P, opts
        ctx.info = info[0]
        ctx.tensor_lam = isinstance(lam, torch.Tensor)
        ctx.tensor_sigma = isinstance(sigma, torch.Tensor)
        return x

    @staticmethod
    def backward(ctx, gx):
        X, x = ctx.saved_tensors
        adj, dlam, dsig, _ = nys.nyspcg_backward(X, ctx.lam, x, gx.contiguous().reshape(-1), ctx.kind, ctx.sigma,
                                                 ctx.P, **ctx.opts)
        dev = x.device
        gl = torch.tensor(dlam, dtype=torch.float64, device=dev) if ctx.tensor_lam else None
        gs = torch.tensor(dsig, dtype=torch.float64, device=dev) if ctx.tensor_sigma else None
        return None, adj, gl, gs, None, None, None


def validation_loss(X, y, Xv, yv, log_lam, log_sigma, kind: int, P=None, opts: dict | None = None):
    """L(lambda, sigma) = mean((K(Xv, X; sigma) x* - yv)^2) with x* from NysPCGSolve; differentiable
    in (log_lam, log_sigma) through the adjoint."""
    opts = dict(tol=1e-10, prec=nys.FP64) if opts is None else opts
    lam = torch.exp(log_lam)
    sigma = torch.exp(log_sigma)
    x = NysPCGSolve.apply(X, y, lam, sigma, kind, P, opts)
    pred = KernelProduct.apply(Xv, X, x, sigma, kind)
    res = pred - yv
    return torch.mean(res * res)
