"""Pins of the oracle's loss, gradients and removal delta (Sec. 4.5, Sec. 6.1,
App. B.4) against finite differences of an independent numpy forward, exact identities
and brute-force re-rendering."""
import math

import numpy as np
import pytest

import oracle as O
import synth


def _forward_loss(sites, lists, target, s, H, W):
    """Independent float64 forward + loss: logits from the rotated quadratic form,
    max-subtracted softmax over the list, L = (1/P) sum ||c - I||^2."""
    P = H * W
    L = 0.0
    for p in range(P):
        X, Y = p % W, p // W
        ids = [int(i) for i in lists[p] if i != O.INVALID]
        if not ids:
            c = np.zeros(3)
        else:
            l = []
            for k in ids:
                x, y, lt, r, _, _, _, ux, uy, a = [float(v) for v in sites[:, k]]
                dx, dy = X - x, Y - y
                al, be = ux * dx + uy * dy, -uy * dx + ux * dy
                l.append(math.exp(lt) * s * (r - math.sqrt(math.exp(a) * al * al +
                                                           math.exp(-a) * be * be)))
            l = np.array(l)
            w = np.exp(l - l.max())
            w /= w.sum()
            c = sites[4:7, ids].astype(np.float64) @ w
        d = c - target[:, Y, X].astype(np.float64)
        L += float(d @ d)
    return L / P


@pytest.fixture(scope="module")
def case():
    H, W, N, K = 9, 11, 14, 4
    sites = synth.random_sites(31, H, W, N, anisotropic=True, log_tau_range=(1.5, 3.5),
                               r_range=(0.5, 3.0), a_range=(-1.5, 1.5))
    s = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, s, sites, N)
    target = synth.image_small(4, H, W, n_shapes=3)
    return H, W, N, K, s, sites, lists, target


def test_loss_and_grad_image(case):
    H, W, N, K, s, sites, lists, target = case
    img = O.render(H, W, K, s, sites, N, lists, O.SCORE_F64)
    L, g = O.loss_grad(img, target)
    assert abs(L - _forward_loss(sites, lists, target, s, H, W)) < 1e-12
    np.testing.assert_allclose(g, 2 * (img - target) / (H * W), atol=1e-15)


def test_gradients_match_central_differences(case):
    H, W, N, K, s, sites, lists, target = case
    img = O.render(H, W, K, s, sites, N, lists, O.SCORE_F64)
    _, g = O.loss_grad(img, target)
    grad = O.render_bwd(H, W, K, s, sites, N, lists, g, mode=O.SCORE_F64)
    rng = np.random.default_rng(0)
    # float64 copies so finite differences see the perturbation exactly
    for trial in range(60):
        i = int(rng.integers(0, N))
        prm = int(rng.integers(0, 10))
        x0 = float(sites[prm, i])
        h = 1e-5 * max(1.0, abs(x0))
        sp, sm = sites.astype(np.float64), sites.astype(np.float64)
        sp[prm, i] += h
        sm[prm, i] -= h
        fd = (_forward_loss(sp, lists, target, s, H, W) -
              _forward_loss(sm, lists, target, s, H, W)) / (2 * h)
        an = grad[prm, i]
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-10, (i, prm, fd, an)


def test_radius_shift_and_colour_sum_identities():
    """Equal tau: adding a constant to every r leaves the weights unchanged, so the r
    gradients sum to zero; the colour gradients sum to sum_x dL/dc(x) (the weights
    form a partition of unity)."""
    H, W, N, K = 10, 10, 20, 8
    sites = synth.random_sites(41, H, W, N, anisotropic=True, log_tau=3.0, r_range=(0, 3))
    s = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, s, sites, N)
    target = synth.image_small(5, H, W, n_shapes=2)
    img = O.render(H, W, K, s, sites, N, lists)
    _, g = O.loss_grad(img, target)
    grad = O.render_bwd(H, W, K, s, sites, N, lists, g)
    assert abs(grad[3].sum()) < 1e-12 * max(1, np.abs(grad[3]).sum()) + 1e-15
    np.testing.assert_allclose(grad[4:7].sum(1), g.reshape(3, -1).sum(1), atol=1e-13)


def test_removal_delta_against_rerender():
    H, W, N, K = 8, 9, 12, 4
    sites = synth.random_sites(51, H, W, N, anisotropic=True, log_tau_range=(1, 6),
                               r_range=(0, 3))
    s = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, s, sites, N)
    target = synth.image_small(6, H, W, n_shapes=3)
    img = O.render(H, W, K, s, sites, N, lists)
    _, g = O.loss_grad(img, target)
    _, rd = O.render_bwd(H, W, K, s, sites, N, lists, g, target=target, removal_delta=True)
    ref = np.zeros(N)
    P = H * W
    for p in range(P):
        ids = [int(i) for i in lists[p] if i != O.INVALID]
        i, j = divmod(p, W)
        base = img[:, i, j] - target[:, i, j]
        for k in ids:
            sub = np.array([[x if x != k else O.INVALID for x in lists[p]]], np.uint32)
            # re-render this single pixel with site k removed from its list
            one = np.full((H * W, K), O.INVALID, np.uint32)
            one[p] = sub
            c2 = O.render(H, W, K, s, sites, N, one)[:, i, j]
            d2 = c2 - target[:, i, j]
            ref[k] += (d2 @ d2 - base @ base) / P
    np.testing.assert_allclose(rd[:N], ref, atol=1e-13)


def test_removal_delta_equals_paper_closed_form_when_well_conditioned():
    """Sec. 4.5: c' = (c - w_k c_k) / (1 - w_k)."""
    H, W, N, K = 6, 6, 10, 4
    sites = synth.random_sites(61, H, W, N, log_tau=1.0)
    s = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, s, sites, N)
    target = np.zeros((3, H, W), np.float32)
    img = O.render(H, W, K, s, sites, N, lists)
    _, g = O.loss_grad(img, target)
    _, rd = O.render_bwd(H, W, K, s, sites, N, lists, g, target=target, removal_delta=True)
    ref = np.zeros(N)
    for p in range(H * W):
        i, j = divmod(p, W)
        ids = [int(x) for x in lists[p]]
        l = np.array([O.score(sites, k, s, float(j), float(i)) for k in ids], np.float64)
        w = np.exp(l - l.max())
        w /= w.sum()
        c = img[:, i, j]
        assert w.max() < 0.999
        for k, wk in zip(ids, w):
            cp = (c - wk * sites[4:7, k].astype(np.float64)) / (1 - wk)
            ref[k] += (cp @ cp - c @ c) / (H * W)
    np.testing.assert_allclose(rd[:N], ref, atol=1e-12)


def test_gradient_skips_coincident_pixel():
    """n = 0 (a site exactly on a pixel centre): the position / metric gradients of
    that entry are taken as zero; everything stays finite."""
    H, W, N, K = 5, 5, 3, 3
    sites = synth.random_sites(71, H, W, N, log_tau=2.0, r=1.0)
    sites[0, 0], sites[1, 0] = 2.0, 2.0
    s = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, s, sites, N)
    img = O.render(H, W, K, s, sites, N, lists)
    _, g = O.loss_grad(img, np.zeros((3, H, W), np.float32))
    grad = O.render_bwd(H, W, K, s, sites, N, lists, g)
    assert np.all(np.isfinite(grad))


def test_removal_delta_when_one_weight_is_one():
    """Removing a site whose weight is 1 to double precision leaves the softmax of the
    others (here: the single other site's colour), not 0/0."""
    H, W, N, K = 1, 3, 2, 2
    sites = synth.random_sites(81, H, W, N, log_tau=20.0, r=0.0)
    sites[0, 0], sites[1, 0] = 0.0, 0.0
    sites[0, 1], sites[1, 1] = 2.0, 0.0
    s = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, s, sites, N)
    target = np.zeros((3, H, W), np.float32)
    img = O.render(H, W, K, s, sites, N, lists)
    _, g = O.loss_grad(img, target)
    _, rd = O.render_bwd(H, W, K, s, sites, N, lists, g, target=target, removal_delta=True)
    c0, c1 = sites[4:7, 0].astype(np.float64), sites[4:7, 1].astype(np.float64)
    # pixel 0 is owned by site 0 (w = 1): removing it shows site 1; pixel 2 the reverse
    want0 = (c1 @ c1 - c0 @ c0) / 3
    want1 = (c0 @ c0 - c1 @ c1) / 3
    assert np.all(np.isfinite(rd))
    # pixel 1 (x = 1) is equidistant: exact halves; removing either shows the other
    cm = 0.5 * (c0 + c1)
    want0 += (c1 @ c1 - cm @ cm) / 3
    want1 += (c0 @ c0 - cm @ cm) / 3
    np.testing.assert_allclose(rd[:2], [want0, want1], atol=1e-12)
