"""ln psi as a differentiable PyTorch function whose backward pass is the
library's hand-written vector-Jacobian-product kernel.

``log_psi(params, samples, state)`` returns ln psi(s) for every row of
``samples`` with the RBM parameters ``params`` (float64 tensor in the packed
layout [a | b | W]); its gradient with respect to ``params`` is
sum_n g_n O(s_n), O = d ln psi / d p (paper, log-derivative equation and the
appendix on vector-Jacobian products), computed by ``nqs_log_psi_vjp``.
"""
from __future__ import annotations

import torch


class _LogPsi(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, samples: torch.Tensor, state):
        state.set_params(params.detach().to(torch.float64))
        out = state.log_psi(samples)
        ctx.state = state
        ctx.save_for_backward(samples)
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (samples,) = ctx.saved_tensors
        g = ctx.state.log_psi_vjp(samples, grad_out.contiguous())
        return g.to(torch.float64), None, None


def log_psi(params: torch.Tensor, samples: torch.Tensor, state) -> torch.Tensor:
    """Differentiable ln psi(samples) under ``params`` (see module docstring)."""
    return _LogPsi.apply(params, samples, state)
