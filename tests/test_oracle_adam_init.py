"""Pins of the oracle's Adam step (Sec. 5, clamps of Sec. 6.1) against
torch.optim.Adam, and of the gradient-weighted initialisation (Sec. 4.4)."""
import math

import numpy as np
import torch

import oracle as O
import synth

LR = np.array([0.1, 0.1, 0.01, 0.1, 1e-3, 1e-3, 1e-3, 0.01, 0.01, 0.01])
LO = [0, 0, 2, 1, 0, 0, 0, -math.inf, -math.inf, -2]


def test_adam_matches_torch_with_clamps():
    H, W, N, cap = 20, 30, 16, 18
    rng = np.random.default_rng(3)
    s32 = synth.random_sites(2, H, W, N, cap=cap, anisotropic=True, log_tau=5.0, r=2.0)
    # start some sites at the bounds so that every clamp is exercised
    s32[0, 0], s32[1, 1], s32[0, 2], s32[1, 3] = 0.02, 0.01, W - 1.01, H - 1.02
    s32[2, 4], s32[2, 5], s32[3, 6], s32[3, 7] = 2.001, 19.99, 1.01, 511.99
    s32[4, 8], s32[5, 9], s32[6, 10], s32[9, 11], s32[9, 12] = 0.001, 0.999, 0.0, 1.99, -1.99
    sites = s32.astype(np.float64)
    m = np.zeros_like(sites)
    v = np.zeros_like(sites)
    params = [torch.tensor(sites[p, :N].copy(), dtype=torch.float64, requires_grad=True)
              for p in range(10)]
    opt = torch.optim.Adam([{"params": [params[p]], "lr": float(LR[p])} for p in range(10)],
                           betas=(0.9, 0.999), eps=1e-8)
    hi = [W - 1, H - 1, 20, 512, 1, 1, 1, math.inf, math.inf, 2]
    for t in range(1, 6):
        g = rng.normal(0, 1, (10, cap)) * np.array([1, 1, 0.1, 1, 0.5, 0.5, 0.5, 2, 2, 1])[:, None]
        # push the boundary sites outwards
        g[0, 0], g[1, 1], g[0, 2], g[1, 3] = 1, 1, -1, -1
        g[2, 4], g[2, 5], g[3, 6], g[3, 7] = 1, -1, 1, -1
        g[4, 8], g[5, 9], g[6, 10], g[9, 11], g[9, 12] = 1, -1, 1, -1, 1
        O.adam(H, W, sites, g, m, v, N, LR, 0.9, 0.999, 1e-8, t)
        for p in range(10):
            params[p].grad = torch.tensor(g[p, :N])
        opt.step()
        with torch.no_grad():
            for p in range(10):
                params[p].clamp_(LO[p], hi[p])
            nu = torch.sqrt(params[7] ** 2 + params[8] ** 2)
            params[7].div_(nu)
            params[8].div_(nu)
        ref = np.stack([q.detach().numpy() for q in params])
        np.testing.assert_allclose(sites[:, :N], ref, rtol=1e-12, atol=1e-12)
    assert sites[0, 0] == 0 and sites[1, 1] == 0 and sites[0, 2] == W - 1 and sites[1, 3] == H - 1
    assert sites[2, 4] == 2 and sites[2, 5] == 20 and sites[3, 6] == 1 and sites[3, 7] == 512
    assert sites[4, 8] == 0 and sites[5, 9] == 1 and sites[9, 11] == 2 and sites[9, 12] == -2
    assert np.all(sites[:, N:] == s32[:, N:])            # inactive slots untouched


def test_init_keys_follow_mixture_density():
    H, W, N, lam, seed = 12, 15, 30, 0.3, 5
    img = synth.image_small(9, H, W, n_shapes=4)
    sites, k, keys = O.init_sites(img, N, lam, seed, 3.0, 1.0, 40, return_keys=True)
    pad = np.pad(img.astype(np.float64), ((0, 0), (1, 1), (1, 1)), mode="edge")
    gx = 0.5 * (pad[:, 1:-1, 2:] - pad[:, 1:-1, :-2])
    gy = 0.5 * (pad[:, 2:, 1:-1] - pad[:, :-2, 1:-1])
    gm = np.sqrt((gx * gx + gy * gy).sum(0)).ravel()
    pinit = (1 - lam) * gm / gm.sum() + lam / (H * W)
    u = np.array([((O.splitmix64(seed, p) >> 32) + 0.5) / 2 ** 32 for p in range(H * W)])
    np.testing.assert_allclose(keys, np.log(u) / pinit, rtol=1e-12)
    assert k == N
    win = np.sort(np.argsort(-keys, kind="stable")[:N])
    np.testing.assert_array_equal(sites[0, :N], (win % W).astype(np.float32))
    np.testing.assert_array_equal(sites[1, :N], (win // W).astype(np.float32))
    np.testing.assert_array_equal(sites[4:7, :N], img.reshape(3, -1)[:, win])
    assert np.all(sites[2, :N] == 3.0) and np.all(sites[3, :N] == 1.0)
    assert np.all(sites[7, :N] == 1.0) and np.all(sites[8:, :N] == 0.0)
    assert np.all(sites[0, N:] == -1.0)


def test_init_every_pixel_when_n_equals_p():
    H, W = 5, 7
    img = synth.image_small(1, H, W, n_shapes=1)
    sites, k = O.init_sites(img, H * W, 0.3, 1, 3.0, 1.0, H * W)
    assert k == H * W
    np.testing.assert_array_equal(sites[0], np.tile(np.arange(W), H).astype(np.float32))
    np.testing.assert_array_equal(sites[1], np.repeat(np.arange(H), W).astype(np.float32))


def test_init_single_draw_is_categorical():
    """Efraimidis-Spirakis with N = 1 selects pixel p with probability P_init(p)."""
    H, W = 2, 3
    img = np.zeros((3, H, W), np.float32)
    img[:, :, 2] = 1.0
    pad = np.pad(img.astype(np.float64), ((0, 0), (1, 1), (1, 1)), mode="edge")
    gx = 0.5 * (pad[:, 1:-1, 2:] - pad[:, 1:-1, :-2])
    gy = 0.5 * (pad[:, 2:, 1:-1] - pad[:, :-2, 1:-1])
    gm = np.sqrt((gx * gx + gy * gy).sum(0)).ravel()
    pinit = 0.7 * gm / gm.sum() + 0.3 / 6
    T = 6000
    counts = np.zeros(6)
    for seed in range(T):
        s, _ = O.init_sites(img, 1, 0.3, seed, 3.0, 1.0, 1)
        counts[int(s[1, 0]) * W + int(s[0, 0])] += 1
    sd = np.sqrt(T * pinit * (1 - pinit))
    assert np.all(np.abs(counts - T * pinit) < 5 * sd + 1)
