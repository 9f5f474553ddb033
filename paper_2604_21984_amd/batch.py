"""Batched encoder: many images of uneven size and site budget trained together, one
persistent launch over all (image, tile) work items per iteration (plus one loss fold,
one Adam and one counter update for the whole batch), recordable as a HIP graph.

Every image follows exactly the single-image iteration of ``encode.Encoder`` (same
initialisation, seeds and counters), so its lists are bit-identical to a per-image run
with the same settings and its parameters agree up to the order of float additions.
"""
import ctypes as C
import math

import torch

from . import _lib as S
from .encode import EncodeConfig, default_log_tau


def tiles_of(H, W, tile_w=16):
    """Work items of an H x W image with tiles tile_w pixels wide, 256 / tile_w tall."""
    th = 256 // tile_w
    return ((H + th - 1) // th) * ((W + tile_w - 1) // tile_w)


class BatchEncoder:
    def __init__(self, targets, n_sites, cfg=None, device=None, grid=0, chunked=1, tile_w=16):
        cfg = cfg or EncodeConfig()
        self.cfg = cfg
        self.device = device or targets[0].device
        dev = self.device
        K = cfg.K
        self.K = K
        self.shapes = [(int(t.shape[1]), int(t.shape[2])) for t in targets]
        self.n_sites = [int(n) for n in n_sites]
        B = len(targets)
        self.B = B
        px0, site0 = [], []
        P_tot = S_tot = 0
        for (H, W), n in zip(self.shapes, self.n_sites):
            px0.append(P_tot)
            site0.append(S_tot)
            P_tot += H * W
            S_tot += n
        self.px0, self.site0 = px0, site0
        self.P_tot, self.S_tot = P_tot, S_tot
        f32 = dict(dtype=torch.float32, device=dev)
        self.target = torch.empty(3 * P_tot, **f32)
        for b, t in enumerate(targets):
            H, W = self.shapes[b]
            self.target[3 * px0[b]:3 * (px0[b] + H * W)].copy_(t.reshape(-1))
        self.sites = torch.empty(10 * S_tot, **f32)
        self.rec = torch.empty(max(S_tot, 1) * S.REC_FLOATS, **f32)
        self.grad = torch.zeros(10 * S_tot, device=dev,
                                dtype=torch.int64 if cfg.deterministic else torch.float32)
        self.m = torch.zeros(10 * S_tot, **f32)
        self.v = torch.zeros(10 * S_tot, **f32)
        self.lists = [torch.empty(K * P_tot, dtype=torch.int32, device=dev) for _ in range(2)]
        self.cur = 0
        self.states = torch.zeros(B * S.STEP_STATE_INT64, dtype=torch.int64, device=dev)
        self.tile_w = None
        self._set_tiles(int(tile_w), int(grid), int(chunked))
        # per-image initialisation through the single-image entry points on views
        for b in range(B):
            img = self.img(b)
            H, W = self.shapes[b]
            n = self.n_sites[b]
            lt0 = cfg.log_tau0 if cfg.log_tau0 is not None else default_log_tau(H, W, n)
            ws = torch.empty(S.init_workspace_bytes(img), dtype=torch.uint8, device=dev)
            S.init_sites(img, self.view_target(b), n, cfg.lam_init, cfg.seed, lt0, cfg.r0,
                         self.view_sites(b), ws)
            S.prepare_sites(img, self.view_sites(b), self.view_rec(b))
            S.seed_topk(img, self.view_rec(b), self.view_list(0, b), self.view_list(1, b))
        lr = [cfg.lr * mlt for mlt in cfg.lr_mult]
        self.adam = S.adam_params(lr, cfg.beta1, cfg.beta2, cfg.eps)
        self.train_cfg = S.train_config(cfg.n_inject, cfg.seed ^ 0x5AD5AD, self.adam,
                                        prop_every=cfg.prop_every,
                                        deterministic=cfg.deterministic)
        self.graph = None
        self.steps = 0

    # ---- views of one image's blocks ------------------------------------------------
    def img(self, b):
        H, W = self.shapes[b]
        return S.image(H, W, self.K, self.n_sites[b], self.n_sites[b], self.cfg.score_scale)

    def view_target(self, b):
        H, W = self.shapes[b]
        return self.target[3 * self.px0[b]:3 * (self.px0[b] + H * W)].view(3, H, W)

    def view_list(self, which, b):
        H, W = self.shapes[b]
        K = self.K
        return self.lists[which][K * self.px0[b]:K * (self.px0[b] + H * W)].view(K // 4, H, W, 4)

    def view_sites(self, b, buf=None):
        n = self.n_sites[b]
        buf = self.sites if buf is None else buf
        return buf[10 * self.site0[b]:10 * (self.site0[b] + n)].view(10, n)

    def view_rec(self, b):
        n = self.n_sites[b]
        return self.rec[S.REC_FLOATS * self.site0[b]:S.REC_FLOATS * (self.site0[b] + max(n, 1))]

    def state(self, b):
        k = S.STEP_STATE_INT64
        return self.states[k * b:k * (b + 1)]

    def _set_tiles(self, tile_w, grid, chunked):
        """Number the work items for tiles tile_w pixels wide (16: 16 x 16, 32: 32 x 8)
        and upload the image descriptors."""
        assert tile_w in (16, 32), tile_w
        tile0, T_tot = [], 0
        for H, W in self.shapes:
            tile0.append(T_tot)
            T_tot += tiles_of(H, W, tile_w)
        self.tile0, self.T_tot, self.tile_w = tile0, T_tot, tile_w
        arr = (S.SadBatchImage * self.B)()
        for b, ((H, W), n) in enumerate(zip(self.shapes, self.n_sites)):
            s = float(self.cfg.score_scale) or float(
                torch.tensor(1.0, dtype=torch.float32) /
                torch.tensor(float(max(H, W)), dtype=torch.float32))
            arr[b] = S.SadBatchImage(H, W, n, tile0[b], n, self.px0[b], self.site0[b], s, 0)
        self.images_dev = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).to(self.device)
        self.batch = S.SadBatch(self.B, self.K, T_tot, grid, chunked, tile_w, self.S_tot,
                                self.images_dev.data_ptr())
        self.graph = None

    # ---- iteration ------------------------------------------------------------------
    def set_launch(self, grid, chunked, tile_w=None):
        """Persistent grid (0: one workgroup per tile), work assignment and, if given, the
        tile shape of the work items."""
        if tile_w is not None and int(tile_w) != self.tile_w:
            self._set_tiles(int(tile_w), int(grid), int(chunked))
        self.batch.grid = int(grid)
        self.batch.chunked = int(chunked)
        self.graph = None

    def set_prop_every(self, f):
        """Candidate update period (propagate on every f-th iteration)."""
        self.train_cfg.prop_every = int(f)
        self.graph = None

    def step(self):
        a, b = self.lists[self.cur], self.lists[1 - self.cur]
        S.batch_train_step(self.batch, self.train_cfg, self.target, self.sites, self.rec, a, b,
                           self.grad, self.m, self.v, None, None, self.states)
        self.cur = 1 - self.cur
        self.steps += 1

    def capture(self):
        """Record one pair of iterations as a HIP graph (the list field ping-pongs, so the
        graph starts and ends on the first buffer: capture after an even number of
        iterations)."""
        if self.cur != 0:
            raise RuntimeError("capture after an even number of iterations (the list "
                               "field must be on its first buffer)")
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
            self.step()
        self.steps -= 2
        self.graph = g
        return g

    def replay(self, pairs=1):
        for _ in range(pairs):
            self.graph.replay()
        self.steps += 2 * pairs

    # ---- snapshots (the autotuner restores the state after its trials) ---------------
    def snapshot(self):
        return [t.clone() for t in (self.sites, self.rec, self.grad, self.m, self.v,
                                    self.lists[0], self.lists[1], self.states)], self.cur, self.steps

    def restore(self, snap):
        bufs, cur, steps = snap
        for dst, src in zip((self.sites, self.rec, self.grad, self.m, self.v, self.lists[0],
                             self.lists[1], self.states), bufs):
            dst.copy_(src)
        self.cur, self.steps = cur, steps

    # ---- reporting ------------------------------------------------------------------
    def losses(self):
        k = S.STEP_STATE_INT64
        return self.states.view(torch.float32).view(self.B, 2 * k)[:, 4].tolist()

    def render(self, b):
        H, W = self.shapes[b]
        out = torch.empty((3, H, W), dtype=torch.float32, device=self.device)
        S.render_fwd(self.img(b), self.view_rec(b), self.view_list(self.cur, b), out)
        return out

    def psnr(self, b):
        img = self.render(b).clamp(0, 1)
        mse = torch.mean((img - self.view_target(b)) ** 2).item()
        return 10.0 * math.log10(1.0 / max(mse, 1e-20))

    def pixels(self):
        return self.P_tot
