"""Gradients of K unrolled steps of Algorithm 1 behind ``torch.autograd.Function``.

Forward: A_s = P(H A_{s-1}), s = 1..K, with H = e^{tau Delta} (Section 5.1) and P
the pointwise closest orthogonal matrix (Lemma 1.1), run by ``mbo_iterate`` in
segments of ``checkpoint`` steps; only the segment starts are kept.

Backward (the paper has no adjoint; this is the chain rule): for each segment,
last first, the iterates are recomputed from its start (``mbo_diffuse`` and
``mbo_project``), then for s from the segment's end down to its start

    Gtil_s      = VJP of P at H A_{s-1} applied to Gbar_s   (mbo_project_vjp)
    dL/dtau    += <Gtil_s, d/dtau H A_{s-1}>                 (mbo_diffuse_dtau)
    Gbar_{s-1}  = H Gtil_s                                   (mbo_diffuse; H is self-adjoint)

and dL/dA_0 = Gbar_0.  Every step runs in the HIP kernels of libmbo; this module
only orders the calls and keeps the checkpoints (torch tensors on the device).
"""
from __future__ import annotations

import torch

from . import mbo


class UnrolledMBO(torch.autograd.Function):
    """A_K = (P o H)^K (A_0) with gradients in A_0 and tau."""

    @staticmethod
    def forward(ctx, A0, tau, plan: "mbo.Plan", K: int, checkpoint: int):
        if K < 0 or checkpoint < 1:
            raise ValueError("K must be >= 0 and checkpoint >= 1")
        tau_f = float(tau)
        plan.set_tau(tau_f)
        A = A0.detach().contiguous().clone()
        ckpts = [A.clone()]
        s = 0
        while s < K:
            m = min(checkpoint, K - s)
            plan.iterate(A, m, logs=False)
            s += m
            if s < K:
                ckpts.append(A.clone())
        ctx.plan, ctx.K, ctx.checkpoint, ctx.tau = plan, int(K), int(checkpoint), tau_f
        ctx.ckpts = ckpts
        ctx.tau_is_tensor = isinstance(tau, torch.Tensor)
        if ctx.tau_is_tensor:
            ctx.tau_meta = (tau.dtype, tau.device)
        return A

    @staticmethod
    def backward(ctx, grad_out):
        plan, K, c = ctx.plan, ctx.K, ctx.checkpoint
        plan.set_tau(ctx.tau)
        G = grad_out.detach().to(plan.dtype).contiguous().clone()
        dtau = 0.0
        for j in reversed(range(len(ctx.ckpts))):
            s0, s1 = j * c, min(j * c + c, K)
            prev = [ctx.ckpts[j]]      # A_{s-1} for s = s0+1..s1
            tilde = []                 # H A_{s-1}
            X = ctx.ckpts[j]
            for s in range(s0 + 1, s1 + 1):
                At = plan.diffuse(X)
                tilde.append(At)
                if s < s1:
                    X = plan.project(At)
                    prev.append(X)
            for i in reversed(range(len(tilde))):
                Gt = plan.project_vjp(tilde[i], G)
                d = plan.diffuse_dtau(prev[i], G=Gt)
                dtau += float(d.sum()) if hasattr(d, "sum") else float(d)
                G = plan.diffuse(Gt)
        ctx.ckpts = None
        gtau = None
        if ctx.tau_is_tensor and ctx.needs_input_grad[1]:
            dt, dev = ctx.tau_meta
            gtau = torch.tensor(dtau, dtype=dt, device=dev)
        gA0 = G if ctx.needs_input_grad[0] else None
        return gA0, gtau, None, None, None


def unrolled_mbo(A0, tau, plan: "mbo.Plan", K: int, checkpoint: int = 10):
    """A_K after K steps of Algorithm 1 from A0, differentiable in A0 and tau.

    ``plan`` fixes n, grid, batch and precision (its tau is overwritten by
    ``tau``); A0 has the plan's dtype and layout.  ``tau`` may be a float or a
    0-dim tensor with ``requires_grad``.
    """
    return UnrolledMBO.apply(A0, tau, plan, K, checkpoint)
