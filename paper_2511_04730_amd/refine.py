"""Bank refinement by gradient descent on the SNR-reconstruction loss.

Each step: loss and gradient from the library (lloid_grad), a plain
gradient step on float64 master copies, FP64 re-orthonormalisation of the
bases on the device (lloid_orthonormalize), and the refined slices written
back into the plan (lloid_set_slice).  The plan must be FP32 with
normalize = False.

The loss curvature grows with the number of samples in the segment, so the
step is eta / (T F) for a segment of T strides of F samples.
"""
from __future__ import annotations

from typing import List, Sequence

from .plan import LloidPlan, orthonormalize


def refine(plan: LloidPlan, banks: Sequence, strain, target, steps: int, eta: float, log=None):
    """Returns the loss before every step and after the last one, and the
    refined float64 (U, W) per slice (cuda tensors)."""
    import torch
    lr = eta / strain.shape[1]
    U = [torch.tensor(s.basis, dtype=torch.float64, device="cuda") for b in banks for s in b.slices]
    W = [torch.tensor(s.mixing, dtype=torch.float64, device="cuda") for b in banks for s in b.slices]
    losses: List[float] = []
    for step in range(steps):
        loss, dW, dU = plan.grad(strain, target)
        losses.append(loss)
        if log:
            log(step, loss)
        for i in range(len(U)):
            W[i] -= lr * dW[i].double()
            U[i] -= lr * dU[i].double()
            orthonormalize(U[i], W[i])
            plan.set_slice(i, U[i], W[i])
    loss, _, _ = plan.grad(strain, target)
    losses.append(loss)
    return losses, U, W
