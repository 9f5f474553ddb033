"""Single-image encoder: gradient-weighted initialisation, seed pass, then one
propagation pass + forward + backward + Adam per iteration (Sec. 4.3-4.4, Sec. 5,
Sec. 6.1), every step on the GPU.

The iteration is one ``sad_train_step`` call whose counters live in device memory, so a
pair of iterations (the list field ping-pongs between two buffers) can be recorded as
a HIP graph once and replayed.

With a ``BudgetSchedule`` the encoder also densifies and prunes (Sec. 4.5, App. B.5):
after the iterations the schedule names, a statistics pass and one
``sad_densify_prune`` call; the new high-water mark of active slots is read back (one
synchronisation per budget event) and becomes the slot range of later iterations.
"""
import math
from dataclasses import dataclass, field

import torch

from . import _lib as S

# Per-parameter learning-rate multipliers over the base rate, order
# (x, y, log_tau, r, c_r, c_g, c_b, u_x, u_y, a).  The paper states per-parameter base
# rates without values; positions and radius move in pixels, the rest in their units.
LR_MULT = (100.0, 100.0, 10.0, 100.0, 1.0, 1.0, 1.0, 10.0, 10.0, 10.0)


@dataclass
class BudgetSchedule:
    """Densify every densify_every iterations within [densify_start, densify_end], prune
    every prune_every iterations within [prune_start, prune_end) (Sec. 4.5); defaults
    are the base schedule of Sec. 6.1."""
    densify_every: int = 20
    densify_start: int = 20
    densify_end: int = 3000
    p_split: float = 0.01
    prune_every: int = 40
    prune_start: int = 100
    prune_end: int = 3000
    p_prune: float = 0.033
    alpha: float = 0.7
    eps: float = 1e-8
    min_mass: float = 1.0
    seed_lists: bool = True

    def events(self, it):
        """(densify, prune) due after iteration it (1-based)."""
        d = self.densify_start <= it <= self.densify_end and it % self.densify_every == 0
        p = self.prune_start <= it < self.prune_end and it % self.prune_every == 0
        return d, p


@dataclass
class EncodeConfig:
    K: int = 8
    n_inject: int = 4              # J (Sec. 6.1)
    lr: float = 1e-3               # base learning rate
    lr_mult: tuple = LR_MULT
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    lam_init: float = 0.3          # lambda_init of Sec. 4.4
    r0: float = 1.0                # initial radius (the clamp minimum)
    log_tau0: float = None         # None: clamp(ln(2 max(H,W) / sqrt(HW/N)), 2, 20)
    seed: int = 0
    score_scale: float = 0.0       # 0: 1 / max(H, W)
    budget: BudgetSchedule = None  # adaptive budget (None: fixed site count)
    prop_every: int = 1            # candidate update period f_cand (App. B.3)
    deterministic: bool = False    # bit-reproducible gradient and statistics sums (integer)


def default_log_tau(H, W, N):
    """Initial log tau giving an adjacent-site logit gap of about 2 (kappa * spacing)."""
    spacing = math.sqrt(H * W / max(N, 1))
    return float(min(max(math.log(2.0 * max(H, W) / spacing), 2.0), 20.0))


class Encoder:
    """Device state of one image: sites, derived records, two list fields, Adam
    moments, gradient, step counters."""

    def __init__(self, target, n_sites, cfg=None, cap=None, device=None):
        cfg = cfg or EncodeConfig()
        self.cfg = cfg
        self.device = device or target.device
        self.target = target.contiguous().to(self.device, torch.float32)
        _, H, W = self.target.shape
        self.H, self.W = H, W
        cap = int(cap or n_sites)
        self.img = S.image(H, W, cfg.K, n_sites, cap, cfg.score_scale)
        dev = self.device
        f32 = dict(dtype=torch.float32, device=dev)
        self.sites = torch.empty((S.NPARAM, cap), **f32)
        self.rec = torch.empty(max(cap if cfg.budget else n_sites, 1) * S.REC_FLOATS, **f32)
        self.lists = [torch.empty((cfg.K // 4, H, W, 4), dtype=torch.int32, device=dev)
                      for _ in range(2)]
        self.cur = 0
        # site-major gradient accumulator (int64 fixed point in the deterministic mode)
        self.grad = torch.zeros((cap, S.NPARAM), device=dev,
                                dtype=torch.int64 if cfg.deterministic else torch.float32)
        self.m = torch.zeros((S.NPARAM, cap), **f32)
        self.v = torch.zeros((S.NPARAM, cap), **f32)
        self.rendered = torch.empty((3, H, W), **f32)
        self.grad_img = torch.empty((3, H, W), **f32)
        self.state = S.step_state(dev)
        lt0 = cfg.log_tau0 if cfg.log_tau0 is not None else default_log_tau(H, W, n_sites)
        ws = torch.empty(S.init_workspace_bytes(self.img), dtype=torch.uint8, device=dev)
        S.init_sites(self.img, self.target, n_sites, cfg.lam_init, cfg.seed, lt0, cfg.r0,
                     self.sites, ws)
        del ws
        S.prepare_sites(self.img, self.sites, self.rec)
        S.seed_topk(self.img, self.rec, self.lists[0], self.lists[1])
        lr = [cfg.lr * mlt for mlt in cfg.lr_mult]
        self.adam = S.adam_params(lr, cfg.beta1, cfg.beta2, cfg.eps)
        self.train_cfg = S.train_config(cfg.n_inject, cfg.seed ^ 0x5AD5AD, self.adam,
                                        prop_every=cfg.prop_every,
                                        deterministic=cfg.deterministic)
        self.graph = None
        self.steps = 0
        self.budget_log = []
        if cfg.budget:
            self.stats = torch.zeros((S.NSTAT, cap), **f32)
            if cfg.deterministic:
                self.stats_acc = torch.empty(2 * S.NSTAT * cap, dtype=torch.int64, device=dev)
            self.counts = torch.zeros(6, dtype=torch.int64, device=dev)
            self.dp_ws = torch.empty(S.densify_workspace_bytes(self.img), dtype=torch.uint8,
                                     device=dev)

    def loss_value(self):
        """L of the last iteration (synchronises)."""
        return float(S.state_loss(self.state).item())

    def counters(self):
        """(pass, adam_step) device counters (synchronises)."""
        return [int(v) for v in S.state_counters(self.state).tolist()]

    @property
    def topk(self):
        return self.lists[self.cur]

    def step(self):
        """One training iteration, enqueued on the current stream (no host sync unless a
        budget event follows it)."""
        a, b = self.lists[self.cur], self.lists[1 - self.cur]
        S.train_step(self.img, self.train_cfg, self.target, self.sites, self.rec, a, b, self.grad,
                     self.m, self.v, None, None, self.state)
        self.cur = 1 - self.cur
        self.steps += 1
        if self.cfg.budget:
            d, p = self.cfg.budget.events(self.steps)
            if d or p:
                self.budget_step(densify=d, prune=p)

    def budget_step(self, densify=True, prune=True):
        """Statistics pass, one prune / split step, record refresh (Sec. 4.5)."""
        bs = self.cfg.budget
        flags = (S.DP_SPLIT if densify else 0) | (S.DP_PRUNE if prune else 0)
        if bs.seed_lists and densify:
            flags |= S.DP_SEED
        if self.cfg.deterministic:  # integer sums: the budget step is reproducible too
            S.site_stats_fixed(self.img, self.rec, self.topk, self.target, self.stats_acc,
                               self.stats)
        else:
            self.stats.zero_()
            S.site_stats(self.img, self.rec, self.topk, self.target, self.stats)
        prm = S.budget_params(bs.p_prune, bs.p_split, flags, bs.alpha, bs.eps, bs.min_mass)
        S.densify_prune(self.img, self.target, self.sites, self.m, self.v, self.stats, prm,
                        self.topk, self.counts, self.dp_ws)
        c = [int(x) for x in self.counts.tolist()]
        self.img.n_slots = max(c[4], 1)
        S.prepare_sites(self.img, self.sites, self.rec)
        self.budget_log.append({"iteration": self.steps, "densify": densify, "prune": prune,
                                "counts": c})
        self.graph = None  # a recorded graph holds the old slot range

    def capture(self, pairs=1):
        """Record 2 * pairs iterations (the list field ping-pongs A -> B -> A) as one HIP
        graph; more pairs per graph amortise the graph launch."""
        assert self.cur == 0, "capture from the first list buffer"
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(2 * pairs):
                self.step()
        self.steps -= 2 * pairs  # recording does not execute
        self.graph = g
        self.graph_steps = 2 * pairs
        return g

    def replay(self, n=1):
        """Replay the recorded graph n times."""
        for _ in range(n):
            self.graph.replay()
        self.steps += self.graph_steps * n

    def render(self, out=None):
        out = out if out is not None else torch.empty((3, self.H, self.W), dtype=torch.float32,
                                                      device=self.device)
        S.render_fwd(self.img, self.rec, self.topk, out)
        return out

    def psnr(self):
        img = self.render().clamp(0, 1)
        mse = torch.mean((img - self.target) ** 2).item()
        return 10.0 * math.log10(1.0 / max(mse, 1e-20))
