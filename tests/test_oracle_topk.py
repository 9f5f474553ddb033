"""Pins of the oracle's exact top-K and seed pass (Sec. 4.3, App. B.3)."""
import math

import numpy as np
from scipy.spatial import cKDTree

import oracle as O
import synth


def test_brute_topk_isotropic_equals_kdtree_knn():
    """a = 0, r = 0, equal tau: the score ranks by Euclidean distance, so the exact
    top-K is the K nearest neighbours (Voronoi / k-th order Voronoi, Eq. vor_cell)."""
    H, W, N, K = 24, 31, 50, 8
    sites = synth.random_sites(11, H, W, N, log_tau=2.0, r=0.0)
    lists = O.brute_topk(H, W, K, O.default_scale(H, W), sites, N)
    tree = cKDTree(np.stack([sites[0, :N], sites[1, :N]], 1).astype(np.float64))
    yy, xx = np.mgrid[0:H, 0:W]
    pts = np.stack([xx.ravel(), yy.ravel()], 1).astype(np.float64)
    d, idx = tree.query(pts, k=K)
    # compare where the K-th and (K+1)-th distances are well separated
    d2, _ = tree.query(pts, k=K + 1)
    gaps = np.min(np.diff(d2, axis=1), axis=1)
    ok = gaps > 1e-4
    assert ok.mean() > 0.95
    assert np.array_equal(lists[ok].astype(np.int64), idx[ok])


def _score64(sites, i, s, X, Y):
    x, y, lt, r, _, _, _, ux, uy, a = [float(v) for v in sites[:, i]]
    dx, dy = X - x, Y - y
    al, be = ux * dx + uy * dy, -uy * dx + ux * dy
    return math.exp(lt) * s * (r - math.sqrt(math.exp(a) * al * al + math.exp(-a) * be * be))


def test_brute_topk_anisotropic_weighted_by_definition():
    H, W, N, K = 12, 14, 30, 4
    sites = synth.random_sites(4, H, W, N, anisotropic=True, log_tau_range=(1, 5),
                               r_range=(0, 4))
    s = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, s, sites, N)
    checked = 0
    for p in range(H * W):
        X, Y = float(p % W), float(p // W)
        sc = np.array([_score64(sites, i, s, X, Y) for i in range(N)])
        order = np.argsort(-sc, kind="stable")
        srt = sc[order]
        if np.min(np.abs(np.diff(srt[:K + 1]))) < 1e-4 * max(1, np.abs(srt[:K + 1]).max()):
            continue
        assert list(lists[p]) == list(order[:K])
        checked += 1
    assert checked > 0.9 * H * W


def test_brute_topk_k_exceeds_active_and_skips_inactive():
    H, W, N, K = 6, 7, 5, 8
    sites = synth.random_sites(8, H, W, N, cap=9)
    sites[0, 2] = -1.0                    # inactive
    sites[3, 4] = np.inf                  # non-finite
    lists = O.brute_topk(H, W, K, 0.125, sites, N)
    for p in range(H * W):
        row = list(lists[p])
        assert sorted(row[:3]) == [0, 1, 3]
        assert row[3:] == [O.INVALID] * 5
        sc = [O.score(sites, i, 0.125, float(p % W), float(p // W)) for i in row[:3]]
        assert sc == sorted(sc, reverse=True)


def test_brute_topk_tie_breaks_by_lower_id():
    sites = synth.random_sites(1, 4, 4, 3)
    sites[:, 1] = sites[:, 0]            # two identical sites
    lists = O.brute_topk(4, 4, 3, 0.25, sites, 3)
    for p in range(16):
        row = list(lists[p])
        assert row.index(0) < row.index(1)


def test_seed_pass_buckets_by_nearest_pixel():
    H, W, K, N = 9, 11, 4, 40
    sites = synth.random_sites(21, H, W, N, cap=44)
    sites[0, 5] = -1.0
    s = 0.1
    lists = O.seed_lists(H, W, K, s, sites, N)
    buckets = {}
    for i in range(N):
        if sites[0, i] < 0:
            continue
        ii = min(max(int(np.rint(sites[1, i])), 0), H - 1)
        jj = min(max(int(np.rint(sites[0, i])), 0), W - 1)
        buckets.setdefault(ii * W + jj, []).append(i)
    for p in range(H * W):
        mine = buckets.get(p, [])
        X, Y = float(p % W), float(p // W)
        mine = sorted(mine, key=lambda i: (-O.score(sites, i, s, X, Y), i))[:K]
        assert list(lists[p]) == mine + [O.INVALID] * (K - len(mine))
