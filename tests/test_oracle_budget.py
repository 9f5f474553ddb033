"""Pins of the oracle's adaptive-budget functions (Sec. 4.5, App. B.5): the statistics
pass against the partition of unity, the loss, a library weighted covariance and the
removal delta of the backward; prune / split selections against numpy sorts; the split
geometry against closed forms; slot assignment, Adam reset and list seeding."""
import math

import numpy as np
import pytest

import oracle as O
import synth

ALPHA = 0.7


def _setup(seed=0, H=20, W=28, N=30, K=4):
    tg = synth.image_small(seed, H, W, n_shapes=6)
    sites = synth.random_sites(seed, H, W, N, anisotropic=True, log_tau_range=(2.5, 4.0),
                               r_range=(1.0, 8.0))
    s = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, s, sites, N)
    return tg, sites, s, lists


# ---- statistics ----------------------------------------------------------------------
def test_stats_mass_is_partition_of_unity_and_energy_sums_to_loss():
    H, W, K, N = 20, 28, 4, 30
    tg, sites, s, lists = _setup(H=H, W=W, N=N, K=K)
    st = O.site_stats(H, W, K, s, sites, N, lists, tg)
    assert st[0].sum() == pytest.approx(H * W, rel=1e-12)           # sum_i w_i(x) = 1
    img = O.render(H, W, K, s, sites, N, lists)
    L, _ = O.loss_grad(img, tg)                                      # (1/P) sum ||c - I||^2
    assert st[1].sum() == pytest.approx(L * H * W, rel=1e-12)
    assert (st[0] >= 0).all() and (st[1] >= 0).all()
    # second moments are sums of omega d^2 >= 0, and Cauchy-Schwarz per site
    assert (st[4] >= 0).all() and (st[6] >= 0).all()
    assert (st[5] ** 2 <= st[4] * st[6] * (1 + 1e-12) + 1e-300).all()
    st2, sa, ss = O.site_stats(H, W, K, s, sites, N, lists, tg, scales=True)
    np.testing.assert_array_equal(st2, st)
    for q in (0, 1, 4, 6):                                           # terms >= 0
        np.testing.assert_allclose(sa[q], st[q], rtol=1e-12)
    assert (sa >= np.abs(st) * (1 - 1e-12)).all() and (ss >= 0).all()
    np.testing.assert_allclose(ss[0], st[0], rtol=1e-12)             # mass: w per term


def test_stats_one_site_moments_equal_weighted_covariance():
    H, W, K = 18, 25, 4
    tg = synth.image_small(3, H, W, n_shapes=5)
    sites = synth.random_sites(3, H, W, 1, anisotropic=True, log_tau=3.0, r=4.0)
    lists = np.full((H * W, K), O.INVALID, np.uint32)
    lists[:, 0] = 0                                                  # w = 1 everywhere
    st = O.site_stats(H, W, K, O.default_scale(H, W), sites, 1, lists, tg)
    c = sites[4:7, 0].astype(np.float64)
    e = ((c[:, None, None] - tg.astype(np.float64)) ** 2).sum(0).ravel()
    yy, xx = np.mgrid[0:H, 0:W]
    X, Y = xx.ravel().astype(np.float64), yy.ravel().astype(np.float64)
    assert st[0, 0] == pytest.approx(H * W, rel=1e-12)
    assert st[1, 0] == pytest.approx(e.sum(), rel=1e-12)
    mu = np.array([np.average(X, weights=e), np.average(Y, weights=e)])
    cov = np.cov(np.stack([X, Y]), aweights=e, bias=True)
    p = sites[:2, 0].astype(np.float64)
    E = st[1, 0]
    np.testing.assert_allclose(st[2:4, 0] / E, mu - p, rtol=1e-10, atol=1e-10)
    m = st[2:4, 0] / E
    got = np.array([[st[4, 0] / E - m[0] ** 2, st[5, 0] / E - m[0] * m[1]],
                    [st[5, 0] / E - m[0] * m[1], st[6, 0] / E - m[1] ** 2]])
    np.testing.assert_allclose(got, cov, rtol=1e-9, atol=1e-9)


def test_stats_removal_delta_equals_backward_channel():
    H, W, K, N = 16, 22, 4, 25
    tg, sites, s, lists = _setup(seed=5, H=H, W=W, N=N, K=K)
    st = O.site_stats(H, W, K, s, sites, N, lists, tg)
    g = np.zeros((3, H, W))
    _, rd = O.render_bwd(H, W, K, s, sites, N, lists, g, target=tg, removal_delta=True)
    # the same Sec. 4.5 sums, in another order (the backward splits pixels over threads)
    np.testing.assert_allclose(st[7], rd, rtol=1e-12, atol=1e-18)


# ---- selections ----------------------------------------------------------------------
def _blank(H, W, cap, n_active, seed=0):
    sites = synth.random_sites(seed, H, W, cap, anisotropic=True, log_tau=4.0, r=6.0)
    rng = np.random.default_rng(seed)
    inactive = rng.choice(cap, cap - n_active, replace=False)
    sites[0, inactive] = -1.0
    sites[1, inactive] = -1.0
    return sites, np.sort(inactive)


def test_prune_removes_smallest_removal_delta_with_id_ties():
    H, W, cap = 20, 20, 60
    sites, inactive = _blank(H, W, cap, 45)
    rng = np.random.default_rng(1)
    st = np.zeros((8, cap), np.float32)
    st[7] = rng.choice([-0.5, 0.0, 0.25, 1.0, 2.0], cap).astype(np.float32)   # many ties
    st[7, inactive] = -9.0                           # inactive slots are never candidates
    before = sites.copy()
    counts = O.densify_prune(synth.image_small(0, H, W), sites, st, 0.3, 0.0, O.DP_PRUNE)
    active = np.setdiff1d(np.arange(cap), inactive)
    n_p = math.floor(0.3 * 45)                       # 13 (not 14: floor)
    order = active[np.lexsort((active, st[7, active]))]
    pruned = np.sort(order[:n_p])
    assert counts == [45, n_p, 0, 45 - n_p, int(np.max(np.setdiff1d(active, pruned))) + 1, 0]
    now_inactive = np.where(sites[0] < 0)[0]
    np.testing.assert_array_equal(now_inactive, np.union1d(inactive, pruned))
    np.testing.assert_array_equal(sites[1, pruned], -1.0)
    keep = np.setdiff1d(np.arange(cap), pruned)
    np.testing.assert_array_equal(sites[:, keep], before[:, keep])


def test_split_selects_top_error_density_and_fills_lowest_free_slots():
    H, W, cap = 24, 30, 40
    sites, inactive = _blank(H, W, cap, 30, seed=2)
    tg = synth.image_small(2, H, W)
    st = np.zeros((8, cap), np.float32)
    # E / m^0.7 ranks differently from E and from E / m
    st[0] = np.linspace(0.5, 40.0, cap).astype(np.float32)[np.random.default_rng(3).permutation(cap)]
    st[1] = np.random.default_rng(4).uniform(0.1, 5.0, cap).astype(np.float32)
    am = np.ones((10, cap), np.float32)
    av = np.full((10, cap), 2.0, np.float32)
    counts = O.densify_prune(tg, sites, st, 0.0, 0.25, O.DP_SPLIT, adam_m=am, adam_v=av)
    active = np.setdiff1d(np.arange(cap), inactive)
    cand = active[st[0, active] > 1.0]
    score = (st[1, cand].astype(np.float64) / np.maximum(st[0, cand].astype(np.float64), 1e-8)
             ** ALPHA).astype(np.float32)
    n_s = min(math.floor(0.25 * 30), len(cand), len(inactive))
    parents = np.sort(cand[np.lexsort((cand, -score))][:n_s])
    assert counts[:3] == [30, 0, n_s] and counts[3] == 30 + n_s and counts[5] == len(cand)
    kids = inactive[:n_s]                                  # lowest free slots, in order
    assert (sites[0, kids] >= 0).all() and (sites[0, inactive[n_s:]] < 0).all()
    touched = np.union1d(parents, kids)
    assert (am[:, touched] == 0).all() and (av[:, touched] == 0).all()
    rest = np.setdiff1d(np.arange(cap), touched)
    assert (am[:, rest] == 1).all() and (av[:, rest] == 2).all()
    # the wrong exponents pick different parents on these statistics
    for wrong in (0.0, 1.0):
        sw = st[1, cand] / np.maximum(st[0, cand], 1e-8) ** wrong
        assert set(np.sort(cand[np.lexsort((cand, -sw))][:n_s])) != set(parents)


def test_split_count_limited_by_candidates_and_free_slots():
    H, W, cap = 16, 16, 20
    sites, inactive = _blank(H, W, cap, 18, seed=6)
    st = np.zeros((8, cap), np.float32)
    st[0] = 5.0
    st[1] = np.arange(cap, dtype=np.float32) + 1
    c = O.densify_prune(synth.image_small(6, H, W), sites, st, 0.0, 0.5, O.DP_SPLIT)
    assert c[2] == 2 and c[3] == 20                        # only two free slots
    sites, inactive = _blank(H, W, 40, 20, seed=7)
    st = np.zeros((8, 40), np.float32)
    st[0] = 1.0                                            # m <= 1: never a candidate
    st[0, :5] = 1.5
    st[1] = 1.0
    c = O.densify_prune(synth.image_small(7, H, W), sites, st, 0.0, 0.5, O.DP_SPLIT)
    act5 = 5 - int(np.isin(np.arange(5), inactive).sum())
    assert c[5] == act5 and c[2] == act5


def test_prune_then_split_reuses_pruned_slot():
    H, W, cap = 16, 16, 10
    sites, _ = _blank(H, W, cap, 10, seed=8)               # full: no free slot
    st = np.zeros((8, cap), np.float32)
    st[7] = np.arange(cap, dtype=np.float32)               # slot 0 has the smallest delta
    st[0] = 4.0
    st[1] = np.arange(cap, dtype=np.float32)               # slot 9 has the largest score
    c = O.densify_prune(synth.image_small(8, H, W), sites, st, 0.1, 0.1, O.DP_PRUNE | O.DP_SPLIT)
    assert c == [10, 1, 1, 10, 10, 9]
    assert sites[0, 0] >= 0                                # pruned, then refilled by the child


# ---- split geometry ----------------------------------------------------------------------
def _one(H, W, x, y, log_tau=5.0, r=10.0, ux=1.0, uy=0.0, a=0.5):
    sites = np.zeros((10, 2), np.float32)
    sites[:, 0] = [x, y, log_tau, r, 0.1, 0.2, 0.3, ux, uy, a]
    sites[:, 1] = [-1, -1, 0, 0, 0, 0, 0, 1, 0, 0]
    return sites


def _stats_for(E, m, mu, lam1, lam2, th):
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    C = R @ np.diag([lam1, lam2]) @ R.T
    S2 = E * (C + np.outer(mu, mu))
    st = np.zeros((8, 2), np.float32)
    st[:, 0] = [m, E, E * mu[0], E * mu[1], S2[0, 0], S2[0, 1], S2[1, 1], 0.0]
    return st


def _split(tg, sites, st):
    return O.densify_prune(tg, sites, st, 0.0, 1.0, O.DP_SPLIT)


@pytest.mark.parametrize("th", [math.pi / 6, 2.0, -1.1])
def test_split_along_residual_covariance_axis(th):
    H, W = 32, 40
    tg = synth.image_small(9, H, W)
    sites = _one(H, W, 20.0, 15.0)
    mu = np.array([1.5, -0.5])
    st = _stats_for(2.0, 16.0, mu, 9.0, 1.0, th)
    c = _split(tg, sites, st)
    assert c[2] == 1
    e1 = np.array([math.cos(th), math.sin(th)])
    e1 = e1 if (e1[0] > 0 or (e1[0] == 0 and e1[1] > 0)) else -e1
    centre = np.array([20.0, 15.0]) + mu
    delta = 0.5 * math.sqrt(16.0)                           # = 2 px
    np.testing.assert_allclose(sites[:2, 0], centre + delta * e1, atol=2e-5)
    np.testing.assert_allclose(sites[:2, 1], centre - delta * e1, atol=2e-5)
    for k in (0, 1):
        np.testing.assert_allclose(sites[7:9, k], e1, atol=1e-6)       # u along the axis
        assert sites[9, k] == pytest.approx(-math.log(3.0), abs=1e-6)  # 0.5 ln(1/9)
        assert sites[2, k] == pytest.approx(4.75) and sites[3, k] == pytest.approx(8.5)
        j, i = int(np.rint(sites[0, k])), int(np.rint(sites[1, k]))
        np.testing.assert_array_equal(sites[4:7, k], tg[:, i, j])


def test_split_offset_clamps_and_parameter_clamps():
    H, W = 32, 40
    tg = synth.image_small(10, H, W)
    for m, d in [(4.0, 1.5), (1e4, 48.0), (36.0, 3.0)]:
        sites = _one(H, W, 20.0, 16.0, log_tau=2.1, r=1.1)
        st = _stats_for(1.0, m, np.zeros(2), 4.0, 1.0, 0.0)
        _split(tg, sites, st)
        exp_x = [min(20.0 + d, W - 1), max(20.0 - d, 0.0)]
        np.testing.assert_allclose(sites[0, :2], exp_x, atol=1e-5)
        assert (sites[2, :2] == 2.0).all() and (sites[3, :2] == 1.0).all()
    # image-boundary clamp and the degenerate (line) covariance: a = -2
    sites = _one(H, W, 0.5, 31.0)
    st = _stats_for(1.0, 16.0, np.zeros(2), 5.0, 0.0, math.pi / 2)
    _split(tg, sites, st)
    np.testing.assert_allclose(sites[:2, 0], [0.5, 31.0], atol=1e-5)   # +2 in y, clamped
    np.testing.assert_allclose(sites[:2, 1], [0.5, 29.0], atol=1e-5)
    assert (sites[9, :2] == -2.0).all()


@pytest.mark.parametrize("ramp,axis", [("x", (1.0, 0.0)), ("y", (0.0, 1.0)),
                                       ("xy", (math.sqrt(0.5), math.sqrt(0.5))),
                                       ("flat", (0.6, 0.8))])
def test_split_fallback_axis_is_image_gradient(ramp, axis):
    H, W = 24, 24
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float32)
    f = {"x": xx, "y": yy, "xy": xx + yy, "flat": np.zeros_like(xx)}[ramp] / 48.0
    tg = np.stack([f, 0.5 * f, 0.25 + 0 * f]).astype(np.float32)
    sites = _one(H, W, 11.0, 12.0, ux=0.6, uy=0.8, a=1.5)
    st = np.zeros((8, 2), np.float32)
    st[0, 0] = 16.0                                         # E = 0: no statistics
    _split(tg, sites, st)
    e = np.array(axis)
    np.testing.assert_allclose(sites[:2, 0], [11.0, 12.0] + 2.0 * e, atol=1e-5)
    np.testing.assert_allclose(sites[:2, 1], [11.0, 12.0] - 2.0 * e, atol=1e-5)
    np.testing.assert_allclose(sites[7:9, :2].T, [[0.6, 0.8]] * 2, atol=1e-7)  # u kept
    assert sites[9, 0] == pytest.approx(1.2) and sites[9, 1] == pytest.approx(1.2)


def test_isotropic_residual_falls_back():
    H, W = 24, 24
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float32)
    tg = np.stack([yy / 48.0] * 3).astype(np.float32)
    sites = _one(H, W, 11.0, 12.0, a=1.0)
    st = _stats_for(1.0, 16.0, np.array([0.5, 0.5]), 3.0, 3.0, 0.3)
    _split(tg, sites, st)
    np.testing.assert_allclose(sites[:2, 0], [11.0, 14.0], atol=1e-5)   # centre p, y axis
    assert sites[9, 0] == pytest.approx(0.8)


# ---- list seeding -------------------------------------------------------------------------
def test_children_seeded_into_lists_smallest_id_wins():
    H, W, K, cap = 16, 16, 4, 8
    tg = synth.image_small(11, H, W)
    sites = np.zeros((10, cap), np.float32)
    for i, (x, y) in enumerate([(4.0, 4.0), (10.0, 4.0), (4.0, 12.0)]):
        sites[:, i] = [x, y, 4.0, 6.0, 0.5, 0.5, 0.5, 1.0, 0.0, 0.0]
    sites[0, 3:] = -1.0
    sites[1, 3:] = -1.0
    st = np.zeros((8, cap), np.float32)
    st[0, :3] = 16.0          # delta 2, E = 0, flat target -> axis u = (1, 0)
    tg[:] = 0.3
    lists = np.arange(H * W * K, dtype=np.uint32).reshape(H * W, K) % 3
    before = lists.copy()
    c = O.densify_prune(tg, sites, st, 0.0, 1.0, O.DP_SPLIT | O.DP_SEED, K=K, lists=lists)
    assert c[2] == 3
    # parents 0, 1, 2 -> children in slots 3, 4, 5 at x - 2
    spots = {(4, 2): 3, (4, 8): 4, (12, 2): 5}
    for (i, j), cid in spots.items():
        assert lists[i * W + j, K - 1] == cid
    changed = np.where((lists != before).any(1))[0]
    assert set(changed) <= {i * W + j for (i, j) in spots}
    # two children on one pixel: the smaller ID wins
    sites2 = np.zeros((10, cap), np.float32)
    sites2[:, 0] = [6.0, 6.0, 4.0, 6.0, 0.5, 0.5, 0.5, 1.0, 0.0, 0.0]
    sites2[:, 1] = [2.0, 6.0, 4.0, 6.0, 0.5, 0.5, 0.5, -1.0, 0.0, 0.0]  # u = (-1, 0)
    sites2[0, 2:] = -1.0
    sites2[1, 2:] = -1.0
    st2 = np.zeros((8, cap), np.float32)
    st2[0, :2] = 16.0
    lists2 = np.zeros((H * W, K), np.uint32)
    O.densify_prune(tg, sites2, st2, 0.0, 1.0, O.DP_SPLIT | O.DP_SEED, K=K, lists=lists2)
    # child of 0 at (4, 6) in slot 2; child of 1 at (4, 6) too (p - 2 u) in slot 3
    np.testing.assert_allclose(sites2[:2, 2], [4.0, 6.0])
    np.testing.assert_allclose(sites2[:2, 3], [4.0, 6.0])
    assert lists2[6 * W + 4, K - 1] == 2
