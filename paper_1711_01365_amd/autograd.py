"""Gradients of K unrolled steps of Algorithm 1 behind ``torch.autograd.Function``.

Forward: A_s = P(H A_{s-1}), s = 1..K, with H = e^{tau Delta} (Section 5.1) and P
the pointwise closest orthogonal matrix (Lemma 1.1), run by ``mbo_iterate`` in
segments of ``checkpoint`` steps; only the segment starts are kept.

Backward (the paper has no adjoint; this is the chain rule): for each segment,
last first, the iterates are recomputed from its start (``mbo_step``), then for
s from the segment's end down to its start one ``mbo_step_vjp`` computes

    Gtil_s      = VJP of P at H A_{s-1} applied to Gbar_s
    dL/dtau    += <Gtil_s, d/dtau H A_{s-1}>      (accumulated on the device)
    Gbar_{s-1}  = H Gtil_s                        (H is self-adjoint)

and dL/dA_0 = Gbar_0.  Nothing in the backward pass waits for the host until
the tau-gradient is read at the end.  Every step runs in the HIP kernels of
libmbo; this module only orders the calls and keeps the checkpoints (torch
tensors on the device).
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
        # dL/dtau accumulates on the device; one read at the end
        dtau = torch.zeros(plan.batch, dtype=torch.float64, device=G.device)
        # K = 0: A_K = A_0, so dL/dA_0 = G and dL/dtau = 0 (no step to pull back through)
        for j in reversed(range(len(ctx.ckpts) if K > 0 else 0)):
            s0, s1 = j * c, min(j * c + c, K)
            prev = [ctx.ckpts[j]]  # A_{s-1} for s = s0+1 .. s1, recomputed
            for _ in range(s0 + 1, s1):
                prev.append(plan.step(prev[-1]))
            for X in reversed(prev):
                plan.step_vjp(X, G, dtau)  # G: Gbar_s -> Gbar_{s-1}
        ctx.ckpts = None
        gtau = None
        if ctx.tau_is_tensor and ctx.needs_input_grad[1]:
            dt, dev = ctx.tau_meta
            gtau = dtau.sum().to(device=dev, dtype=dt)
        gA0 = G if ctx.needs_input_grad[0] else None
        return gA0, gtau, None, None, None


def unrolled_mbo(A0, tau, plan: "mbo.Plan", K: int, checkpoint: int = 10):
    """A_K after K steps of Algorithm 1 from A0, differentiable in A0 and tau.

    ``plan`` fixes n, grid, batch and precision (its tau is overwritten by
    ``tau``); A0 has the plan's dtype and layout.  ``tau`` may be a float or a
    0-dim tensor with ``requires_grad``.
    """
    return UnrolledMBO.apply(A0, tau, plan, K, checkpoint)
