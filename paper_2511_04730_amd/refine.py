"""Bank refinement by gradient descent on the SNR-reconstruction loss.

Each step: loss and gradient through SnrReconstructionLoss (the library's
lloid_grad behind torch.autograd, which also writes the current slices into
the plan), a plain gradient step on float64 master copies, and FP64
re-orthonormalisation of the bases on the device (lloid_orthonormalize).  The plan must be FP32 with
normalize = False.

The loss curvature grows with the number of samples in the segment, so the
step is eta / (T F) for a segment of T strides of F samples.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

from .autograd import bank_loss, bank_parameters
from .plan import LloidPlan, orthonormalize, quantize_fp8_rows


def refine(plan: LloidPlan, banks: Sequence, strain, target, steps: int, eta: float, log=None,
           quantize: Optional[str] = None, eta_u: Optional[float] = None):
    """Returns the loss before every step and after the last one, and the
    refined float64 (U, W) per slice (cuda tensors).

    eta_u: step of the bases (default eta).  The curvature of the loss in U
    scales with the squared singular values folded into W, in W with the
    basis outputs' variance, so a bank with large singular values needs a
    much smaller basis step (about eta / sigma_max^2) than mixing step.

    quantize="fp8": refinement for the FP8 form.  Every basis is held at
    its FP8 values (quantize_fp8_rows; the FP8 form converts them exactly)
    and only the mixing rows are refined, which compensates the rounding:
    for a fixed basis the loss is quadratic in W.  (Moving the unrounded
    basis with the gradient taken at its FP8 values, straight through the
    rounding, raises the FP8 loss: each step and re-orthonormalisation
    re-rounds every value.)"""
    import torch
    lr = eta / strain.shape[1]
    lr_u = (eta if eta_u is None else eta_u) / strain.shape[1]
    U, W = bank_parameters(banks)
    if quantize is not None:
        assert quantize == "fp8"
        U = [quantize_fp8_rows(u.detach()) for u in U]          # fixed, no gradient
    losses: List[float] = []
    for step in range(steps):
        loss = bank_loss(plan, strain, target, U, W)
        loss.backward()
        losses.append(float(loss.detach()))
        if log:
            log(step, losses[-1])
        with torch.no_grad():
            for i in range(len(U)):
                W[i] -= lr * W[i].grad
                W[i].grad = None
                if quantize is None:
                    U[i] -= lr_u * U[i].grad
                    U[i].grad = None
                    orthonormalize(U[i].detach(), W[i].detach())
    with torch.no_grad():
        losses.append(float(bank_loss(plan, strain, target, U, W)))
    return losses, [u.detach() for u in U], [w.detach() for w in W]
