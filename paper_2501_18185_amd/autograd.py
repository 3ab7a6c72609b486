"""Differentiable sigma and energy on top of libmw (torch.autograd).

``Energy.apply(c, h, g, plan)`` returns E = c^H H(h, g) c.  Its backward
runs the library's density-matrix adjoint, which recomputes the determinant
connectivity instead of storing it:

    dE/dh = gamma,   dE/dg = Gamma / 2,   dE/dc = 2 H c  (real c)

with gamma, Gamma the one- and two-particle density matrices (spin-summed
for spin-free problems).  ``Sigma.apply(c, h, g, plan)`` returns sigma = H c;
its backward is sigma applied to the incoming gradient (H is Hermitian) and
the transition density matrices between that gradient and c.

``h`` and ``g`` are CPU tensors laid out as in the problem (spin-free real
n x n and n^4; spinor complex M x M and M^4).  When they differ from the
integrals the plan holds, the plan is updated in place (no regrouping).
Only the argument marshalling happens here; the arithmetic runs in libmw.
"""
from __future__ import annotations

import numpy as np
import torch

from . import mw


def _sync_integrals(plan: mw.Plan, h: torch.Tensor, g: torch.Tensor, ecore: float):
    hn = h.detach().cpu().numpy()
    gn = g.detach().cpu().numpy()
    key = getattr(plan, "_int_key", None)
    if key is not None and key[0] is not None and np.array_equal(key[0], hn) and np.array_equal(key[1], gn) \
            and key[2] == ecore:
        return
    plan.set_integrals(hn, gn, ecore)
    plan._int_key = (hn.copy(), gn.copy(), ecore)


def _to(x, meta):
    dtype, device = meta
    return x.to(device=device, dtype=dtype)


class Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, h, g, plan, ecore=0.0):
        _sync_integrals(plan, h, g, ecore)
        sigma = plan.sigma(c)
        e = torch.sum(c.conj() * sigma).real
        ctx.save_for_backward(c, sigma)
        ctx.plan = plan
        ctx.h_meta = (h.dtype, h.device)
        ctx.g_meta = (g.dtype, g.device)
        return e

    @staticmethod
    def backward(ctx, ge):
        c, sigma = ctx.saved_tensors
        plan = ctx.plan
        grad_c = grad_h = grad_g = None
        if ctx.needs_input_grad[0]:
            # real c: dE/dc = 2 sigma; complex c: torch's convention for a
            # real loss is the conjugate Wirtinger derivative times 2
            grad_c = 2.0 * ge * sigma
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            gam, Gam = plan.rdm(c, c)
            if ctx.needs_input_grad[1]:
                gh = gam if plan.is_complex else gam.real
                grad_h = _to(ge * gh if not plan.is_complex else ge * gh.conj(), ctx.h_meta)
            if ctx.needs_input_grad[2]:
                gg = 0.5 * Gam
                grad_g = _to(ge * gg if not plan.is_complex else ge * gg.conj(), ctx.g_meta)
        return grad_c, grad_h, grad_g, None, None


class Sigma(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, h, g, plan, ecore=0.0):
        _sync_integrals(plan, h, g, ecore)
        sigma = plan.sigma(c)
        ctx.save_for_backward(c)
        ctx.plan = plan
        ctx.h_meta = (h.dtype, h.device)
        ctx.g_meta = (g.dtype, g.device)
        return sigma

    @staticmethod
    def backward(ctx, gs):
        (c,) = ctx.saved_tensors
        plan = ctx.plan
        gs = gs.contiguous()
        grad_c = grad_h = grad_g = None
        if ctx.needs_input_grad[0]:
            grad_c = plan.sigma(gs)
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            if plan.is_complex:
                raise NotImplementedError("integral gradients of Sigma are provided for real problems")
            # L = gs^T H c  ->  dL/dh = gamma(gs, c), dL/dg = Gamma(gs, c) / 2
            gam, Gam = plan.rdm(gs, c)
            if ctx.needs_input_grad[1]:
                grad_h = _to(gam, ctx.h_meta)
            if ctx.needs_input_grad[2]:
                grad_g = _to(0.5 * Gam, ctx.g_meta)
        return grad_c, grad_h, grad_g, None, None
