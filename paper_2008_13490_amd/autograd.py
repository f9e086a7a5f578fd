"""torch.autograd.Function wrappers of the HIP path.

``gst_nll(rho, E, G, target)``   negative log-likelihood of the counts; its
                                 backward is the library's gradient (computed in
                                 the same launch sequence as the objective).
``gst_probs(rho, E, G, target)`` outcome probabilities [S, M]; its backward is
                                 the library's vector-Jacobian product with the
                                 upstream weights dLoss/dp.
``gst_gateset(theta, param)``    (rho, E, G) of a parameter vector of an
                                 estimation mode (``api.Parameterization``: full,
                                 TP or CPTP); its backward is the library's chain
                                 rule ``gst_param_backward``.

``target`` is an ``api.Request`` (resident sequences and counts) or a tuple
``(api.Context, api.DeviceSeqs, counts or None)``.  Every number is computed
on the GPU by ``libgst.so``.
"""
from __future__ import annotations

import torch

from . import api


def _gateset(rho, E, G):
    D = rho.shape[0]
    n = {4: 1, 16: 2, 64: 3}[D]
    return api.DeviceGateSet(n, rho.detach().contiguous(), E.detach().contiguous(), G.detach().contiguous())


def _split(g, rho, E, G):
    D, M, K = rho.shape[0], E.shape[0], G.shape[0]
    return g[:D].view_as(rho), g[D:D + M * D].view_as(E), g[D + M * D:].view_as(G)


class _NLL(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, E, G, target):
        gs = _gateset(rho, E, G)
        if isinstance(target, api.Request):
            obj, _, grad = target.eval(gs, want_probs=False, want_grad=True)
        else:
            c, seqs, counts = target
            obj, _, grad = c.loglik(gs, seqs, counts, want_probs=False, want_grad=True)
        ctx.save_for_backward(grad)
        ctx.shapes = (rho, E, G)
        return obj[0]

    @staticmethod
    def backward(ctx, gout):
        (grad,) = ctx.saved_tensors
        rho, E, G = ctx.shapes
        dr, dE, dG = _split(grad * gout, rho, E, G)
        return dr, dE, dG, None


class _Probs(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, E, G, target):
        gs = _gateset(rho, E, G)
        if isinstance(target, api.Request):
            p = target.probs(gs)
        else:
            c, seqs, _ = target
            p = c.probs(gs, seqs)
        ctx.save_for_backward(rho, E, G)
        ctx.target = target
        return p

    @staticmethod
    def backward(ctx, gout):
        rho, E, G = ctx.saved_tensors
        gs = _gateset(rho, E, G)
        w = gout.detach().to(torch.float64).contiguous()
        if isinstance(ctx.target, api.Request):
            g = ctx.target.vjp(gs, w)
        else:
            c, seqs, _ = ctx.target
            g = c.vjp(gs, seqs, w)
        dr, dE, dG = _split(g, rho, E, G)
        return dr, dE, dG, None


def gst_nll(rho, E, G, target):
    return _NLL.apply(rho, E, G, target)


def gst_probs(rho, E, G, target):
    return _Probs.apply(rho, E, G, target)


class _GateSet(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, param):
        th = theta.detach().contiguous()
        gs = param.forward(th)
        ctx.save_for_backward(th)
        ctx.param = param
        return gs.rho, gs.effects, gs.gates

    @staticmethod
    def backward(ctx, grho, gE, gG):
        (th,) = ctx.saved_tensors
        par = ctx.param
        D, M, K = par.D, par.M, par.K
        parts = []
        for g, shape in ((grho, (D,)), (gE, (M, D)), (gG, (K, D, D))):
            if g is None:
                g = torch.zeros(shape, dtype=torch.float64, device=th.device)
            parts.append(g.detach().to(torch.float64).reshape(-1))
        return par.backward(th, torch.cat(parts).contiguous()), None


def gst_gateset(theta, param):
    return _GateSet.apply(theta, param)
