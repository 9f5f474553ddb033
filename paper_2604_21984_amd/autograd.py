"""torch.autograd wrappers around the hand-derived kernels (Sec. 5: the paper derives
every gradient by hand instead of using automatic differentiation; here the
hand-derived backward kernel is exposed to torch's autograd).

``SADRender``: sites [10, cap] (differentiable) + top-K list field (not
differentiable) -> image [3, H, W].  The forward stores nothing but the derived
records and the lists; the backward recomputes the blend weights.
``SADMSELoss``: L = (1/P) sum_x ||c(x) - I(x)||^2 (Sec. 6.1) with its gradient formed
by the loss kernel in the forward call.
``SADTrainPass``: sites -> L for one whole pass (propagation, blend, loss, backward in
the fused kernel); the gradient is formed in the forward launch and handed out by the
backward.
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


class SADTrainPass(torch.autograd.Function):
    """One propagation pass, blend, MSE loss and backward in a single kernel (the fused
    training pass, ``sad_train_image_pass``): the forward returns L and forms dL/dsites
    in the same launch (site-major accumulator, nothing else stored); the backward
    returns grad_output * dL/dsites in the layout of the sites (``sad_grad_to_params``,
    which also clears the accumulator for the next call).  The lists are not
    differentiable; the pass index comes from the device step state."""

    @staticmethod
    def forward(ctx, sites, target, img, cfg, rec, topk_in, topk_out, gacc, state, prepare):
        if prepare:
            S.prepare_sites(img, sites.detach(), rec)
        if not (cfg.flags & S.TRAIN_LOSS_SET) or img.n_slots == 0:
            S.state_loss(state).zero_()   # the pass adds L (with no sites it forms none)
        S.train_image_pass(img, cfg, target, rec, topk_in, topk_out, gacc, None, None, state)
        ctx.img, ctx.cap = img, sites.shape[1]
        ctx.gacc = gacc
        return S.state_loss(state).clone()

    @staticmethod
    def backward(ctx, g):
        grad = torch.empty((10, ctx.cap), dtype=torch.float32, device=g.device)
        S.grad_to_params(ctx.img, ctx.gacc, grad, scale=g.detach().reshape(1).contiguous(),
                         clear=True)
        return grad, None, None, None, None, None, None, None, None, None


def render(sites, topk, img, rec=None):
    """Differentiable render of ``sites`` with the given list field."""
    if rec is None:
        rec = torch.empty(max(img.n_slots, 1) * S.REC_FLOATS, dtype=torch.float32,
                          device=sites.device)
    return SADRender.apply(sites, topk, img, rec)


def mse_loss(rendered, target, img):
    return SADMSELoss.apply(rendered, target, img)


class AutogradTrainer:
    """Training iterations through the autograd wrappers: a propagation pass (the lists
    are not differentiable), ``SADRender``, ``SADMSELoss``, ``backward()`` and Adam on
    ``sites.grad``.  The pass index (jump schedule, injection stream) and the Adam step
    live in a device step state, so an iteration issues no host-side counter and the
    iterations can be recorded once as a HIP graph (``capture``) and replayed.

    sites: float32 [10, cap] device tensor (copied); topk: the current list field
    (copied); target: float32 [3, H, W]; adam: a ``SadAdamParams``."""

    def __init__(self, img, sites, topk, target, adam, n_inject=4, seed=0):
        self.img, self.adam, self.J, self.seed = img, adam, int(n_inject), int(seed)
        dev = sites.device
        self.sites = sites.detach().clone().requires_grad_(True)
        self.rec = torch.empty(max(img.n_slots, 1) * S.REC_FLOATS, dtype=torch.float32,
                               device=dev)
        S.prepare_sites(img, self.sites.detach(), self.rec)
        self.m = torch.zeros_like(self.sites.detach())
        self.v = torch.zeros_like(self.sites.detach())
        self.lists = [topk.clone(), torch.empty_like(topk)]
        self.cur = 0
        self.target = target
        self.state = S.step_state(dev)
        self.loss = None
        self.graph = None
        self._one = torch.ones((), dtype=torch.float32, device=dev)  # dL/dL, allocated once

    def step(self):
        a, b = self.lists[self.cur], self.lists[1 - self.cur]
        S.propagate_topk_state(self.img, self.rec, a, b, self.J, self.seed, self.state)
        # with no .grad the backward's gradient tensor becomes sites.grad as it is (no
        # accumulate kernel, no clearing after Adam); dL/dL is a preallocated one
        self.sites.grad = None
        out = render(self.sites, b, self.img, self.rec)
        loss = mse_loss(out, self.target, self.img)
        loss.backward(self._one)
        self.loss = loss.detach()  # keep no autograd graph alive across iterations
        S.adam_step_state(self.img, self.sites.data, self.sites.grad, self.m, self.v,
                          self.adam, self.rec, self.state)
        self.cur = 1 - self.cur

    def capture(self, pairs=1, warmup=2):
        """Record 2 * pairs iterations as one graph (the list field ping-pongs, so the
        graph starts and ends on the same buffer), after `warmup` eager iteration pairs
        on a side stream."""
        side = torch.cuda.Stream(device=self.sites.device)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(2 * warmup):
                self.step()
        torch.cuda.current_stream().wait_stream(side)
        assert self.cur == 0
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            for _ in range(2 * pairs):
                self.step()

    def replay(self, n=1):
        for _ in range(n):
            self.graph.replay()

    def counters(self):
        """(pass, adam_step) on the host (synchronises)."""
        return tuple(int(x) for x in S.state_counters(self.state).cpu())


class FusedAutogradTrainer(AutogradTrainer):
    """Training iterations through ``SADTrainPass``: the pass, blend, loss and backward of
    an iteration are one kernel behind the autograd Function; ``backward()`` lays the
    gradient out as ``sites.grad`` and Adam (which also refreshes the derived records and
    advances the device counters) follows.  Recordable as a HIP graph like the parent."""

    def __init__(self, img, sites, topk, target, adam, n_inject=4, seed=0):
        super().__init__(img, sites, topk, target, adam, n_inject, seed)
        self.cfg = S.train_config(self.J, self.seed, adam, loss_set=True)
        self.gacc = torch.zeros((img.cap, 10), dtype=torch.float32, device=sites.device)

    def step(self):
        a, b = self.lists[self.cur], self.lists[1 - self.cur]
        self.sites.grad = None
        loss = SADTrainPass.apply(self.sites, self.target, self.img, self.cfg, self.rec, a, b,
                                  self.gacc, self.state, False)
        loss.backward(self._one)
        self.loss = loss.detach()
        S.adam_step_state(self.img, self.sites.data, self.sites.grad, self.m, self.v,
                          self.adam, self.rec, self.state)
        self.cur = 1 - self.cur
