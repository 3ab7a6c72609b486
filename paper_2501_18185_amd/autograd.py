"""Differentiable sigma and energy on top of libmw (torch.autograd).

``Energy.apply(c, h, g, plan)`` returns the energies E_k = c_k^H H(h, g) c_k
(a scalar for c of shape [ndet], one per root for [ndet, nroots]).  Its
backward runs the library's density-matrix adjoint, which recomputes the
determinant connectivity instead of storing it:

    dE/dh = gamma,   dE/dg = Gamma / 2,   dE/dc = 2 H c  (real c)

with gamma, Gamma the one- and two-particle density matrices (spin-summed
for spin-free problems).  ``Sigma.apply(c, h, g, plan)`` returns sigma = H c;
its backward is sigma applied to the incoming gradient (H is Hermitian) and
the transition density matrices between that gradient and c.

``h`` and ``g`` are CPU tensors laid out as in the problem (spin-free real
n x n and n^4; spinor complex M x M and M^4).  When they differ from the
integrals the plan holds, the plan is updated in place (no regrouping).
``BatchedEnergy.apply(plans, ecores, *cs, *hs, *gs)`` does the same for
several problems at once: the forward runs one batched sigma launch (a
replayed HIP graph) and the batched energies, the backward one captured
graph of every problem's gradient kernels.

Only argument marshalling happens here: the energies, the scaling by the
upstream gradient, the factor 1/2 and the conjugation of complex integral
gradients all run in libmw (mw_energy, mw_energy_backward,
mw_sigma_backward and their batched forms).
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
    if x is None:
        return None
    dtype, device = meta
    return x.to(device=device, dtype=dtype)


class Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, h, g, plan, ecore=0.0):
        _sync_integrals(plan, h, g, ecore)
        sigma = plan.sigma(c)
        e = plan.energy(c, sigma)
        ctx.save_for_backward(c, sigma)
        ctx.plan = plan
        ctx.h_meta = (h.dtype, h.device)
        ctx.g_meta = (g.dtype, g.device)
        return e.reshape(()) if c.dim() == 1 else e

    @staticmethod
    def backward(ctx, ge):
        c, sigma = ctx.saved_tensors
        want_c = ctx.needs_input_grad[0]
        want_int = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        gc, gh, gg = ctx.plan.energy_backward(c, sigma, ge, want_c, want_int)
        return (gc, _to(gh, ctx.h_meta) if ctx.needs_input_grad[1] else None,
                _to(gg, ctx.g_meta) if ctx.needs_input_grad[2] else None, None, None)


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
        want_c = ctx.needs_input_grad[0]
        want_int = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        gc, gh, gg = ctx.plan.sigma_backward(c, gs.contiguous(), want_c, want_int)
        return (gc, _to(gh, ctx.h_meta) if ctx.needs_input_grad[1] else None,
                _to(gg, ctx.g_meta) if ctx.needs_input_grad[2] else None, None, None)


class BatchedEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plans, ecores, *tensors):
        n = len(plans)
        cs, hs, gs = tensors[:n], tensors[n:2 * n], tensors[2 * n:3 * n]
        for pl, h, g, ec in zip(plans, hs, gs, ecores):
            _sync_integrals(pl, h, g, ec)
        cs = [c.contiguous() for c in cs]
        sig = mw.sigma_batched(plans, cs)
        es = mw.energy_batched(plans, cs, sig)
        ctx.save_for_backward(*cs, *sig)
        ctx.plans = plans
        ctx.metas = [((h.dtype, h.device), (g.dtype, g.device)) for h, g in zip(hs, gs)]
        return tuple(e.reshape(()) if c.dim() == 1 else e for e, c in zip(es, cs))

    @staticmethod
    def backward(ctx, *ges):
        plans = ctx.plans
        n = len(plans)
        saved = ctx.saved_tensors
        cs, sig = saved[:n], saved[n:]
        want_c = any(ctx.needs_input_grad[2:2 + n])
        want_int = any(ctx.needs_input_grad[2 + n:2 + 3 * n])
        gc, gh, gg = mw.energy_backward_batched(plans, cs, sig, ges, want_c, want_int)
        grads_c = [x if ctx.needs_input_grad[2 + i] else None for i, x in enumerate(gc)]
        grads_h = [_to(x, m[0]) if ctx.needs_input_grad[2 + n + i] else None
                   for i, (x, m) in enumerate(zip(gh, ctx.metas))]
        grads_g = [_to(x, m[1]) if ctx.needs_input_grad[2 + 2 * n + i] else None
                   for i, (x, m) in enumerate(zip(gg, ctx.metas))]
        return (None, None, *grads_c, *grads_h, *grads_g)
