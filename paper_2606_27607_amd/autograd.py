"""The log-likelihood as a differentiable function of branch lengths (torch.autograd).

    lnL = BranchLengthLnL.apply(t, inst, mode)

``t`` is a CUDA float64 tensor of the 2N-2 branch lengths (indexed by node) of the tree the
instance was given with ``set_tree``.  The forward pass runs transition matrices, post-order
partials and root integration; the backward pass is the pre-order traversal with the fused
edge integration (the paper's linear-time branch gradient), scaled by the incoming
gradient.  Modes:

* ``"store"``     - backward reuses the post-order partials the forward pass left in the
                    instance's workspace (no recomputation).  If the instance was used for
                    anything else between forward and backward, backward recomputes them.
* ``"recompute"`` - backward recomputes the post-order partials together with the pre-order
                    pass in one launch; nothing has to survive from forward to backward, so
                    one workspace can serve several likelihood terms in between.
* ``"fused"``     - forward already computes the gradient (one launch for both passes);
                    backward only scales it.  Fastest when every forward is differentiated
                    (gradient-based MCMC and optimisers).
* ``"checkpoint"`` - ``inst`` is a :class:`~.checkpoint.Checkpointed` instance: forward keeps
                    the post-order partials of every m-th level only, and backward
                    recomputes the rest segment by segment (far fewer partial buffers, about
                    one more post-order pass; the calls block on the host).  A backward pass
                    whose forward state was overwritten (a later forward call, or a first
                    backward pass) runs that forward pass again from its saved branch
                    lengths.
"""
from __future__ import annotations

import torch

MODES = ("store", "recompute", "fused", "checkpoint")


class BranchLengthLnL(torch.autograd.Function):
    @staticmethod
    def forward(ctx, t, inst, mode="store"):
        if mode not in MODES:
            raise ValueError(f"mode must be one of {MODES}")
        t = t.detach().contiguous()
        ctx.mode = mode
        ctx.inst = inst
        if mode == "checkpoint":
            lnl = inst.lnl(t.cpu().numpy())
            # the backward pass runs the forward pass again unless this token is still live
            ctx.token = inst.forward_token
            ctx.t_host = inst.last_t
            return torch.tensor(lnl, dtype=torch.float64, device=t.device)
        if mode == "fused":
            out = inst.evaluate_device(t, want_grad=True)
            ctx.save_for_backward(out[1:])
            return out[0].clone()
        out = inst.evaluate_device(t, want_grad=False)
        ctx.generation = inst.generation
        ctx.save_for_backward(t)
        return out[0].clone()

    @staticmethod
    def backward(ctx, grad_out):
        inst = ctx.inst
        if ctx.mode == "checkpoint":
            g = torch.as_tensor(inst.gradients(ctx.t_host, ctx.token), dtype=torch.float64,
                                device=grad_out.device)
            return grad_out * g, None, None
        if ctx.mode == "fused":
            (g,) = ctx.saved_tensors
        else:
            (t,) = ctx.saved_tensors
            if ctx.mode == "store" and inst.generation == ctx.generation:
                g = inst.gradients_device()
            else:
                g = inst.evaluate_device(t, want_grad=True)[1:]
        return grad_out * g, None, None


def lnl(t: torch.Tensor, inst, mode: str = "store") -> torch.Tensor:
    return BranchLengthLnL.apply(t, inst, mode)


__all__ = ["BranchLengthLnL", "lnl", "MODES"]
