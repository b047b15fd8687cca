"""torch.autograd binding of the multislice loss (Sec. 3.2: the gradient of the
noise-model loss with respect to every reconstruction variable).

``MultisliceLoss`` is a ``torch.autograd.Function``: its forward runs the
library's forward pass with the per-slice entry waves checkpointed on the
device (every slice, or every k-th slice when the HBM budget of the context
asks for it, the others then being recomputed segment by segment in the
backward pass) and returns the group loss; its backward runs the adjoint
kernels from that tape and returns the object, probe and position gradients
scaled by the incoming gradient. Complex gradients follow PyTorch's
convention (dL/dRe + i dL/dIm), so the result can be fed to any torch
optimiser.
"""
from __future__ import annotations

import torch

from .api import Problem


class MultisliceLoss(torch.autograd.Function):
    """loss = MultisliceLoss.apply(obj, probe, positions, problem, patterns, batch_idx)"""

    @staticmethod
    def forward(ctx, obj, probe, positions, problem: Problem, patterns, batch_idx):
        loss, _ = problem.forward_save(probe.detach(), obj.detach(), positions.detach(), patterns, batch_idx)
        ctx.problem = problem
        ctx.tape = problem.tape_id
        # the tape refers to these buffers: autograd's version check rejects in-place edits
        ctx.save_for_backward(obj, probe, positions)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad_loss):
        obj, probe, positions = ctx.saved_tensors
        if ctx.problem.tape_id != ctx.tape:
            raise RuntimeError("another forward pass ran on this Problem before this backward; "
                               "use one Problem per pending graph")
        need_o, need_p, need_x = ctx.needs_input_grad[:3]
        g_o = torch.empty_like(obj) if need_o else None
        g_p = torch.empty_like(probe) if need_p else None
        g_x = torch.empty_like(positions) if need_x else None
        # the adjoint is linear in the incoming gradient: the kernels scale every
        # output by it, reading it on the device (no host synchronisation)
        scale = grad_loss.detach().reshape(1).to(device=obj.device, dtype=torch.float64).contiguous()
        ctx.problem.backward(scale, g_o, g_p, g_x, dense_pos=True)
        return g_o, g_p, g_x, None, None, None


def multislice_loss(obj, probe, positions, problem: Problem, patterns, batch_idx):
    """Differentiable group loss of one batch of positions."""
    return MultisliceLoss.apply(obj, probe, positions, problem, patterns, batch_idx)
