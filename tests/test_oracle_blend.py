"""Pins of the oracle's soft blend (Sec. 4.2) and point query (Sec. 6.6)."""
import math

import numpy as np

import oracle as O
import synth


def _lists_random(rng, H, W, K, N, fill=0.8):
    lists = np.full((H * W, K), O.INVALID, np.uint32)
    for p in range(H * W):
        m = int(rng.integers(0, K + 1)) if rng.uniform() > fill else K
        lists[p, :m] = rng.choice(N, size=m, replace=False)
    return lists


def test_partition_of_unity_and_convex_output():
    """The blend is a convex combination of the list colours (Sec. 4.2; a convex
    output is listed among the representation's properties in Sec. 6)."""
    rng = np.random.default_rng(1)
    H, W, K, N = 10, 13, 8, 40
    sites = synth.random_sites(3, H, W, N, anisotropic=True, log_tau_range=(0, 8),
                               r_range=(0, 6))
    lists = _lists_random(rng, H, W, K, N)
    img = O.render(H, W, K, O.default_scale(H, W), sites, N, lists)
    # a constant colour renders exactly to itself (weights sum to one)
    flat = sites.copy()
    flat[4:7] = np.array([0.25, 0.5, 0.75], np.float32)[:, None]
    img1 = O.render(H, W, K, O.default_scale(H, W), flat, N, lists)
    for p in range(H * W):
        ids = [i for i in lists[p] if i != O.INVALID]
        i, j = divmod(p, W)
        if not ids:
            assert np.all(img[:, i, j] == 0)                     # empty list -> 0
            continue
        cols = sites[4:7, ids].astype(np.float64)
        assert np.all(img[:, i, j] >= cols.min(1) - 1e-12)
        assert np.all(img[:, i, j] <= cols.max(1) + 1e-12)
        np.testing.assert_allclose(img1[:, i, j], [0.25, 0.5, 0.75], atol=1e-12)


def _full_softmax(sites, N, s, H, W):
    out = np.zeros((3, H, W))
    for i in range(H):
        for j in range(W):
            l = []
            for k in range(N):
                x, y, lt, r, _, _, _, ux, uy, a = [float(v) for v in sites[:, k]]
                dx, dy = j - x, i - y
                al, be = ux * dx + uy * dy, -uy * dx + ux * dy
                n = math.sqrt(math.exp(a) * al * al + math.exp(-a) * be * be)
                l.append(math.exp(lt) * s * (r - n))
            l = np.array(l)
            w = np.exp(l - l.max())
            w /= w.sum()
            out[:, i, j] = sites[4:7, :N].astype(np.float64) @ w
    return out


def test_k_equals_n_is_full_softmax():
    H, W, N = 9, 8, 8
    sites = synth.random_sites(7, H, W, N, anisotropic=True, log_tau_range=(0, 5),
                               r_range=(0, 3))
    s = O.default_scale(H, W)
    lists = O.brute_topk(H, W, N, s, sites, N)
    ref = _full_softmax(sites, N, s, H, W)
    np.testing.assert_allclose(O.render(H, W, N, s, sites, N, lists, O.SCORE_F64), ref,
                               atol=1e-12)
    np.testing.assert_allclose(O.render(H, W, N, s, sites, N, lists, O.SCORE_F32), ref,
                               atol=1e-5)


def test_hard_limit_is_apollonius_owner():
    """A large common tau turns the blend into hard ownership by the anisotropic
    Apollonius cell argmin_i ||x - p_i||_G - r_i (Sec. 3 Eq. our_score_hard)."""
    H, W, N, K = 16, 16, 24, 4
    sites = synth.random_sites(12, H, W, N, anisotropic=True, r_range=(0, 3), log_tau=20.0)
    s = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, s, sites, N)
    img = O.render(H, W, K, s, sites, N, lists)
    tested = 0
    for p in range(H * W):
        X, Y = p % W, p // W
        d = []
        for k in range(N):
            x, y, lt, r, _, _, _, ux, uy, a = [float(v) for v in sites[:, k]]
            dx, dy = X - x, Y - y
            al, be = ux * dx + uy * dy, -uy * dx + ux * dy
            d.append(math.sqrt(math.exp(a) * al * al + math.exp(-a) * be * be) - r)
        d = np.array(d)
        o = np.argsort(d)
        if d[o[1]] - d[o[0]] < 1e-3:
            continue
        np.testing.assert_allclose(img[:, Y, X], sites[4:7, o[0]], atol=1e-9)
        tested += 1
    assert tested > 0.95 * H * W


def test_query_at_pixel_centres_equals_render_and_uses_nearest_list():
    rng = np.random.default_rng(5)
    H, W, K, N = 11, 9, 4, 20
    sites = synth.random_sites(13, H, W, N, anisotropic=True, log_tau_range=(1, 4))
    s = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, s, sites, N)
    img = O.render(H, W, K, s, sites, N, lists)
    yy, xx = np.mgrid[0:H, 0:W]
    xy = np.stack([xx.ravel(), yy.ravel()], 1).astype(np.float32)
    q = O.query(H, W, K, s, sites, N, lists, xy)
    np.testing.assert_array_equal(q, img.reshape(3, -1).T)
    # off-centre points: the list of the nearest pixel (clamped), blended at the point
    pts = np.stack([rng.uniform(-2, W + 1, 50), rng.uniform(-2, H + 1, 50)], 1).astype(np.float32)
    q2 = O.query(H, W, K, s, sites, N, lists, pts)
    for m, (x, y) in enumerate(pts):
        i = min(max(int(np.rint(y)), 0), H - 1)
        j = min(max(int(np.rint(x)), 0), W - 1)
        ids = [k for k in lists[i * W + j] if k != O.INVALID]
        l = np.array([O.score(sites, k, s, float(x), float(y)) for k in ids], np.float64)
        w = np.exp(l - l.max())
        w /= w.sum()
        np.testing.assert_allclose(q2[m], sites[4:7, ids].astype(np.float64) @ w, atol=1e-12)
