"""torch.autograd wrapper of the library's discrete adjoint (adscl_adjoint).

``drift_loss(batch, c, eps, J, T)`` returns the per-instance drift objective
L_b = sum_{j<J} (E_j(T) - E_j(0))^2 of mode-sum initial data
Pi(x,0) = eps_b sum_k c_bk e_k(x) (arXiv:1706.07413, Sec. II); its backward
hands out dL/dc computed by the library's reverse kernels together with L in
the forward call (one forward evolution and one reverse sweep per call).
Instances that collapse before T have valid = 0 and a zero gradient.
"""
import torch


class DriftLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, eps, batch, J, T, ckpt_every):
        c_d = c.detach().to(torch.float64).contiguous()
        e_d = eps.detach().to(device=c_d.device, dtype=torch.float64).contiguous()
        L, g, valid = batch.adjoint(e_d, c_d, J, T, ckpt_every)
        ctx.save_for_backward(g)
        ctx.mark_non_differentiable(valid)
        return L, valid

    @staticmethod
    def backward(ctx, gL, gvalid):
        (g,) = ctx.saved_tensors
        return gL.to(g.dtype)[:, None] * g, None, None, None, None, None


def drift_loss(batch, c, eps, J, T, ckpt_every=512):
    """(L [n_inst], valid [n_inst]) with dL/dc available through autograd."""
    return DriftLoss.apply(c, eps, batch, int(J), float(T), int(ckpt_every))
