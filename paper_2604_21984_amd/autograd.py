"""torch.autograd wrappers around the hand-derived kernels (Sec. 5: the paper derives
every gradient by hand instead of using automatic differentiation; here the
hand-derived backward kernel is exposed to torch's autograd).

``SADRender``: sites [10, cap] (differentiable) + top-K list field (not
differentiable) -> image [3, H, W].  The forward stores nothing but the derived
records and the lists; the backward recomputes the blend weights.
``SADMSELoss``: L = (1/P) sum_x ||c(x) - I(x)||^2 (Sec. 6.1) with its gradient formed
by the loss kernel in the forward call.
"""
import torch

from . import _lib as S


class SADRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sites, topk, img, rec):
        S.prepare_sites(img, sites.detach(), rec)
        out = torch.empty((3, img.H, img.W), dtype=torch.float32, device=sites.device)
        S.render_fwd(img, rec, topk, out)
        ctx.img = img
        ctx.cap = sites.shape[1]
        ctx.save_for_backward(rec, topk)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        rec, topk = ctx.saved_tensors
        g = torch.zeros((10, ctx.cap), dtype=torch.float32, device=grad_out.device)
        S.render_bwd(ctx.img, rec, topk, grad_out.contiguous(), g)
        return g, None, None, None


class SADMSELoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rendered, target, img):
        loss = S.loss_acc(rendered.device)
        grad = torch.empty_like(rendered)
        S.loss_grad(img, rendered.detach().contiguous(), target.contiguous(), grad, loss)
        ctx.save_for_backward(grad)
        return loss[0].clone()

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return grad * g, None, None


def render(sites, topk, img, rec=None):
    """Differentiable render of ``sites`` with the given list field."""
    if rec is None:
        rec = torch.empty(max(img.n_slots, 1) * S.REC_FLOATS, dtype=torch.float32,
                          device=sites.device)
    return SADRender.apply(sites, topk, img, rec)


def mse_loss(rendered, target, img):
    return SADMSELoss.apply(rendered, target, img)
