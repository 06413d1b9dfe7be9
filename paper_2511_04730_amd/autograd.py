"""torch.autograd entry to the bank gradient.

SnrReconstructionLoss wraps lloid_grad: its forward loads the given bases
U^s and mixing matrices W^s into the plan (lloid_set_slice), runs the
filter over the strain segment on the GPU and returns the loss
sum (rho - target)^2 over every real SNR row, template, detector and sample
of the segment; its backward returns the gradients that the same library
call produced (dW = 2 G Y^T and dU = the correlation of W^T G, upsampled back
through every rate, with the strain), scaled by the incoming gradient.

Gradients flow to the bank parameters only; strain and target are treated
as constants.  The plan must be FP32 with normalize = False (the loss is
defined for the bank as given), and its stream state is used and advanced
as lloid_grad describes (the segment is filtered from a zero history).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple


def _torch():
    import torch
    return torch


class SnrReconstructionLoss(_torch().autograd.Function):
    """loss = SnrReconstructionLoss.apply(plan, strain, target, *U, *W)

    U: one [L, N] tensor per slice (plan slice order), W: one [2M, L] per
    slice; float32 or float64 cuda tensors.  Returns a 0-d float64 tensor."""

    @staticmethod
    def forward(ctx, plan, strain, target, *params):
        torch = _torch()
        n = len(params) // 2
        if len(params) != 2 * n or n != len(plan.slice_shapes()):
            raise ValueError("expected one U and one W per plan slice")
        Us, Ws = params[:n], params[n:]
        for i in range(n):
            plan.set_slice(i, Us[i].detach().to(torch.float64).contiguous(),
                           Ws[i].detach().to(torch.float64).contiguous())
        loss, dW, dU = plan.grad(strain, target)
        ctx.save_for_backward(*dU, *dW)
        ctx.dtypes = [p.dtype for p in params]
        return torch.tensor(loss, dtype=torch.float64, device=strain.device)

    @staticmethod
    def backward(ctx, gout):
        saved = ctx.saved_tensors
        grads = [(gout * g.to(gout.dtype)).to(dt) for g, dt in zip(saved, ctx.dtypes)]
        return (None, None, None, *grads)


def bank_loss(plan, strain, target, U: Sequence, W: Sequence):
    """Differentiable loss of the bank (U, W) on the segment; see module doc."""
    return SnrReconstructionLoss.apply(plan, strain, target, *U, *W)


def bank_parameters(banks, requires_grad: bool = True) -> Tuple[List, List]:
    """float64 cuda copies of every slice's (U, W), in plan slice order."""
    torch = _torch()
    U = [torch.tensor(s.basis, dtype=torch.float64, device="cuda", requires_grad=requires_grad)
         for b in banks for s in b.slices]
    W = [torch.tensor(s.mixing, dtype=torch.float64, device="cuda", requires_grad=requires_grad)
         for b in banks for s in b.slices]
    return U, W
