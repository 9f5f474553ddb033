"""Pins of the oracle's variants: tau diffusion (App. B.6)."""
import numpy as np
import pytest

import oracle as O
import synth

INV = 0xFFFFFFFF


def _case(seed=0, H=30, W=40, K=8, N=300):
    s = synth.random_sites(seed, H, W, N, anisotropic=True, log_tau_range=(2, 5),
                           r_range=(1, 3))
    s[0:2, 4] = -1.0
    sc = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, sc, s, N)
    g = np.random.default_rng(seed).normal(0, 1, N)
    return H, W, K, sc, s, N, lists, g


def test_tau_diffusion_lambda_zero_is_identity():
    H, W, K, sc, s, N, lists, g = _case()
    assert np.array_equal(O.tau_diffusion(H, W, K, sc, s, N, lists, g, 0.0), g)


def test_tau_diffusion_constant_field_is_fixed():
    H, W, K, sc, s, N, lists, _ = _case(1)
    g = np.full(N, 0.375)
    assert np.allclose(O.tau_diffusion(H, W, K, sc, s, N, lists, g, 0.7), g, rtol=0, atol=1e-15)


def test_tau_diffusion_hand_example():
    """Three sites on a 1 x 5 strip, K = 4.  Lists (exact top 4): every pixel holds all
    three.  Site 0 sits at pixel 0, site 1 at pixel 2, site 2 at pixel 4; with
    g = (1, 2, 6) and lambda = 1/2: g0' = 1/2 + 1/2 (2 + 6)/2 = 2.5, g1' = 1 + (1 + 6)/4
    = 2.75, g2' = 3 + (1 + 2)/4 = 3.75."""
    H, W, K = 1, 5, 4
    s = np.zeros((10, 3), np.float32)
    s[0] = [0, 2, 4]
    s[2] = 3.0
    s[3] = 1.0
    s[7] = 1.0
    sc = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, sc, s, 3)
    assert (np.sort(lists[:, :3], axis=1) == [0, 1, 2]).all() and (lists[:, 3] == INV).all()
    out = O.tau_diffusion(H, W, K, sc, s, 3, lists, np.array([1.0, 2.0, 6.0]), 0.5)
    assert np.array_equal(out, [2.5, 2.75, 3.75])


def test_tau_diffusion_lambda_one_is_neighbour_mean_and_edge_cases():
    H, W, K, sc, s, N, lists, g = _case(2)
    out = O.tau_diffusion(H, W, K, sc, s, N, lists, g, 1.0)
    for i in range(N):
        if s[0, i] < 0:
            assert out[i] == g[i]          # inactive: untouched
            continue
        p = int(min(max(np.rint(s[1, i]), 0), H - 1)) * W + int(min(max(np.rint(s[0, i]), 0), W - 1))
        nb = [int(j) for j in lists[p] if j != INV and j != i and s[0, j] >= 0]
        want = np.mean(g[nb]) if nb else g[i]
        assert abs(out[i] - want) <= 1e-12 * (1 + abs(want)), i
    # a site alone in its pixel's list keeps its gradient
    lone = lists.copy()
    lone[:] = INV
    assert np.array_equal(O.tau_diffusion(H, W, K, sc, s, N, lone, g, 0.9), g)


# ---- one-dimensional SAD (Sec. 7 "1D Signal Fitting") ------------------------------------

import math  # noqa: E402

import torch  # noqa: E402


def _sites1d(seed, M, n, log_tau=None, r=None, cap=None):
    rng = np.random.default_rng(seed)
    cap = n if cap is None else cap
    s = np.zeros((4, cap), np.float32)
    s[0, :] = -1.0
    s[0, :n] = rng.uniform(0, M - 1, n)
    s[1, :n] = rng.uniform(-1, 1, n)
    s[2, :n] = rng.uniform(2, 5, n) if log_tau is None else log_tau
    s[3, :n] = rng.uniform(1, 4, n) if r is None else r
    return s


def test_1d_brute_topk_is_sorted_distance():
    """Equal temperature and radius: the top K of a sample are its K nearest sites
    (numpy argsort of the float64 distance, ties to the lower ID)."""
    M, n, K = 200, 60, 8
    s = _sites1d(1, M, n, log_tau=3.0, r=1.0)
    s[0, 7] = -1.0
    sc = O.scale1d(M)
    got = O.brute_topk1d(M, K, sc, s, n)
    act = np.flatnonzero(s[0, :n] >= 0)
    for m in range(M):
        d = np.abs(m - s[0, act].astype(np.float64))
        order = act[np.lexsort((act, d))][:K]
        assert list(got[m]) == list(order), m


def test_1d_full_softmax_and_hard_limit():
    M, n = 64, 8
    s = _sites1d(2, M, n)
    sc = O.scale1d(M)
    lists = O.brute_topk1d(M, n, sc, s, n)
    col, _, _, _ = O.render1d(M, n, sc, s, n, lists, mode=O.SCORE_F64)
    for m in range(M):     # K = N: the softmax over every site (independent numpy)
        l = np.exp(s[2].astype(np.float64)) * sc * (s[3] - np.abs(m - s[0].astype(np.float64)))
        w = np.exp(l - l.max())
        assert abs(col[m] - (w / w.sum()) @ s[1].astype(np.float64)) < 1e-12
    # common log tau = 20 and equal r: each sample takes its nearest site's value
    h = _sites1d(3, M, n, log_tau=20.0, r=1.0)
    lists = O.brute_topk1d(M, 4, sc, h, n)
    col, _, _, _ = O.render1d(M, 4, sc, h, n, lists)
    for m in range(M):
        d = np.abs(m - h[0].astype(np.float64))
        o = np.argsort(d)
        if d[o[1]] - d[o[0]] > 0.02:
            assert abs(col[m] - h[1, o[0]]) < 1e-9, m


def test_1d_gradients_match_central_differences():
    M, n, K = 40, 10, 4
    s = _sites1d(4, M, n)
    sc = O.scale1d(M)
    lists = O.brute_topk1d(M, K, sc, s, n)
    tgt = np.sin(np.arange(M) / 5.0).astype(np.float32)
    _, L, g, _ = O.render1d(M, K, sc, s, n, lists, target=tgt, mode=O.SCORE_F64, grad=True)
    rng = np.random.default_rng(5)
    for _ in range(40):
        q, i = int(rng.integers(4)), int(rng.integers(n))
        h = 1e-4 if q == 0 else 1e-3 * max(1.0, abs(float(s[q, i])))
        if q == 0 and np.any(np.abs(s[0, i] - np.arange(M)) < 2 * h):
            continue   # the step would cross the kink of |x - p| at a sample
        sp, sm = s.copy(), s.copy()
        sp[q, i] += np.float32(h)
        sm[q, i] -= np.float32(h)
        hh = (float(sp[q, i]) - float(sm[q, i])) / 2
        Lp = O.render1d(M, K, sc, sp, n, lists, target=tgt, mode=O.SCORE_F64)[1]
        Lm = O.render1d(M, K, sc, sm, n, lists, target=tgt, mode=O.SCORE_F64)[1]
        fd = (Lp - Lm) / (2 * hh)
        assert abs(fd - g[q, i]) <= 2e-5 * max(abs(fd), 1e-4), (q, i, fd, g[q, i])


def test_1d_gradient_identities():
    M, n, K = 80, 30, 8
    s = _sites1d(6, M, n, log_tau=3.0, r=2.0)
    sc = O.scale1d(M)
    lists = O.brute_topk1d(M, K, sc, s, n)
    tgt = (np.arange(M) > 40).astype(np.float32)
    col, L, g, _ = O.render1d(M, K, sc, s, n, lists, target=tgt, grad=True)
    gimg = 2 * (col - tgt) / M
    assert abs(g[1].sum() - gimg.sum()) < 1e-12           # sum of dL/dc = sum of dL/dc(x)
    assert abs(g[3].sum()) < 1e-12 * np.abs(g[3]).sum() + 1e-15   # equal tau: sum dL/dr = 0
    assert abs(L - np.mean((col - tgt) ** 2)) < 1e-15


def test_1d_propagation_converges_and_dilates():
    M, n, K = 300, 6, 8
    s = _sites1d(7, M, n)
    s[0, 2] = -1.0
    sc = O.scale1d(M)
    lists = O.seed1d(M, K, sc, s, n)
    exact = O.brute_topk1d(M, K, sc, s, n)
    for t in range(14):
        lists = O.prop_pass1d(M, K, sc, s, n, lists, O.jump(t, 1, M), 2, 3, t)
    assert np.array_equal(lists, exact)
    # one site, no injections: the set of samples holding it dilates by {0, +-s_t}
    one = _sites1d(8, M, 1)
    one[0, 0] = 17.0
    cur = O.seed1d(M, 4, sc, one, 1)
    have = {17}
    for t in range(10):
        st = O.jump(t, 1, M)
        cur = O.prop_pass1d(M, 4, sc, one, 1, cur, st, 0, 0, t)
        have = {x + d for x in have for d in (0, st, -st) if 0 <= x + d < M}
        assert set(np.flatnonzero(cur[:, 0] == 0).tolist()) == have


def test_1d_adam_matches_torch_with_clamps():
    M, n, cap = 50, 6, 7
    s = _sites1d(9, M, n, cap=cap).astype(np.float64)
    s[0, 0], s[2, 1], s[3, 2] = 0.01, 19.995, 1.001
    m = np.zeros_like(s)
    v = np.zeros_like(s)
    lr = np.array([0.1, 0.01, 0.05, 0.1])
    params = [torch.tensor(s[q, :n].copy(), requires_grad=True) for q in range(4)]
    opt = torch.optim.Adam([{"params": [params[q]], "lr": float(lr[q])} for q in range(4)],
                           betas=(0.9, 0.999), eps=1e-8)
    lo, hi = [0, -math.inf, 2, 1], [M - 1, math.inf, 20, 512]
    rng = np.random.default_rng(10)
    for t in range(1, 6):
        g = rng.normal(0, 1, (4, cap))
        g[0, 0], g[2, 1], g[3, 2] = 1.0, -1.0, 1.0
        O.adam1d(M, s, g, m, v, n, lr, 0.9, 0.999, 1e-8, t)
        for q in range(4):
            params[q].grad = torch.tensor(g[q, :n])
        opt.step()
        with torch.no_grad():
            for q in range(4):
                params[q].clamp_(lo[q], hi[q])
        np.testing.assert_allclose(s[:, :n], np.stack([p.detach().numpy() for p in params]),
                                   rtol=1e-12, atol=1e-12)
    assert s[0, 0] == 0 and s[2, 1] == 20 and s[3, 2] == 1
    assert s[0, n] == -1       # the free slot is untouched
