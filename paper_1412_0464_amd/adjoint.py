"""Receiver-data misfit and its gradient with respect to the squared slowness
m = 1/c^2, as a ``torch.autograd.Function`` over the GPU library.

forward(m) solves A(m) u_s = b_s for all sources in one batch (one FGMRES
process per source, the preconditioner of the handle; hsp_solve_batch) and
returns the predicted data d_s = u_s[receivers] (complex, shape
(n_sources, n_receivers)).  backward(g_d) solves the adjoint systems
A^H lam_s = R^T g_d,s as one batch with the same handle (conj_transpose = 1,
A being complex symmetric) and accumulates
dL/dm = h^2 omega^2 sum_s Re(conj(lam_s) u_s / (alpha_1 alpha_2)) in a
device kernel (hsp_gradient_accumulate).  ``g_d`` is torch's
conjugate-Wirtinger gradient of a real loss (for L = 1/2 ||d - d_obs||^2 it
is d - d_obs).

Selecting receiver values and placing the adjoint sources are index
operations on device tensors; all arithmetic runs in the library's kernels.
Receiver indices must be distinct: placing the adjoint sources is a plain
assignment, which would keep only one of two entries for a repeated node.
"""
from __future__ import annotations

import torch

from .hsp import Helmholtz


class HelmholtzMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, sources, receivers, omega, h, pml, J, c_pml, tol, opts):
        if not (c_pml and c_pml > 0):
            raise ValueError("an explicit c_pml > 0 is required (with mean(c) the PML would depend on m)")
        receivers = torch.as_tensor(receivers)
        if receivers.dim() != 1 or torch.unique(receivers).numel() != receivers.numel():
            raise ValueError("receivers must be a 1-D set of distinct node indices")
        opts = dict(opts or {})
        opts.setdefault("fine_stencil", 5)
        c = torch.rsqrt(m.detach()).contiguous()
        hs = Helmholtz(c, omega, h, pml, J, c_pml=c_pml, **opts)
        B = torch.stack([hs.rhs(sources[s].contiguous()) for s in range(sources.shape[0])])
        U, its, rrs = hs.solve_batch(B, tol=tol, maxit=500)
        ctx.hs = hs
        ctx.tol = tol
        ctx.receivers = receivers
        ctx.save_for_backward(U)
        return U.reshape(U.shape[0], -1)[:, receivers]

    @staticmethod
    def backward(ctx, grad_d):
        hs = ctx.hs
        (U,) = ctx.saved_tensors
        ns = U.shape[0]
        g = torch.zeros(hs.n_fine, dtype=torch.float64, device=grad_d.device)
        RT = torch.zeros((ns,) + tuple(hs.n_fine), dtype=torch.complex128, device=grad_d.device)
        RT.view(ns, -1)[:, ctx.receivers] = grad_d.to(torch.complex128)
        LAM, its, rrs = hs.solve_batch(RT, tol=ctx.tol, maxit=500, conj_transpose=True)
        for s in range(ns):
            hs.gradient_accumulate(U[s], LAM[s], g)
        return g, None, None, None, None, None, None, None, None, None


def misfit(m, sources, receivers, d_obs, omega, h, pml, J, c_pml, tol=1e-8, **opts):
    """L = 1/2 sum_s ||d_s(m) - d_obs_s||^2, differentiable in m."""
    d = HelmholtzMisfit.apply(m, sources, receivers, omega, h, pml, J, c_pml, tol, opts)
    r = d - d_obs
    return 0.5 * (r.real ** 2 + r.imag ** 2).sum()
