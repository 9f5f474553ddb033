"""GPU parity of the fused training pass and the batched training step against the CPU
oracle (rows a3-a6 as one kernel: propagation pass, blend, loss gradient, backward).

Each case builds a site set and a list field on the CPU (oracle initialisation, seed
pass and propagation passes of the oracle, never the GPU), runs one pass through the
C ABI from that field at a given pass index, and compares:
  lists      bit-exact over the whole field (the oracle's pass at the same index);
  colours    max-abs <= 1e-5 against the oracle's blend of the oracle's new lists;
  dL/dc      |d| <= 2/P * 2e-5 (float32 c - I);
  loss       relative 1e-5;
  gradients  the per-group rule of the parity tests (conditioning term included), with
             the worst ratio under the plain rule printed beside it.
The batched step runs Adam after the pass; its learning rates are zero and its moments
start at zero, so after one step m = (1 - beta1) g gives the summed gradient g.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth
from _helpers import grad_check, planar_to_rows, rows_to_planar

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def S():
    import paper_2604_21984_amd._lib as S
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return S


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _encode_sites(seed, H, W, N, cap=None):
    """Target, sites (oracle initialisation moved to a mid-encode-like state), scale."""
    target = synth.image_encode(seed, H, W, n_polygons=200 if H * W > 100_000 else 20,
                                patch=128 if H * W > 100_000 else 16)
    lt0 = float(np.clip(math.log(2 * max(H, W) / math.sqrt(H * W / N)), 2, 20))
    sites, n = O.init_sites(target, N, 0.3, seed, lt0, 1.0, cap or N)
    assert n == N
    sites = synth.perturb_sites(seed + 1, sites, N, H, W)
    return target, sites, O.default_scale(H, W)


def _fields(H, W, K, s, sites, N, J, seed, upto):
    """Oracle list fields: F[0] = seed pass, F[t + 1] = pass t of the schedule."""
    F = [O.seed_lists(H, W, K, s, sites, N)]
    for t in range(upto):
        F.append(O.prop_pass(H, W, K, s, sites, N, F[-1], O.jump(t, H, W), J, seed, t))
    return F


def _oracle_pass(H, W, K, s, sites, N, lists_in, J, seed, t, target):
    out = O.prop_pass(H, W, K, s, sites, N, lists_in, O.jump(t, H, W), J, seed, t)
    col = O.render(H, W, K, s, sites, N, out)
    L, g = O.loss_grad(col, target)
    grad, ab = O.render_bwd(H, W, K, s, sites, N, out, g, abs_sum=True)
    return out, col, L, g, grad, ab


def _fused(S, H, W, K, s, sites, N, lists_in, J, seed, t, target, deterministic=False):
    """One sad_train_image_pass from lists_in at pass index t; returns host arrays
    (lists, rendered, dL/dc, loss, gradient [10][cap])."""
    cap = sites.shape[1]
    img = S.image(H, W, K, N, cap, s)
    dsites = _t(sites)
    rec = torch.empty(max(N, 1) * 16, dtype=torch.float32, device=DEV)
    S.prepare_sites(img, dsites, rec)
    lin = _t(rows_to_planar(lists_in, H, W, K))
    lout = torch.empty_like(lin)
    adam = S.adam_params([0.0] * 10)
    cfg = S.train_config(J, seed, adam, deterministic=deterministic)
    grad = torch.zeros((cap, 10), device=DEV,
                       dtype=torch.int64 if deterministic else torch.float32)
    rendered = torch.empty((3, H, W), dtype=torch.float32, device=DEV)
    gimg = torch.empty_like(rendered)
    state = S.step_state()
    state[0] = t
    S.train_image_pass(img, cfg, _t(target), rec, lin, lout, grad, rendered, gimg, state)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().astype(np.float64)
    if deterministic:
        e = 0
        while (1 << (e + 1)) < H * W:
            e += 1
        g = g * 2.0 ** -(20 + e)
    return (planar_to_rows(lout.cpu().numpy(), H, W, K), rendered.cpu().numpy(),
            gimg.cpu().numpy(), float(S.state_loss(state).item()), g.T.copy())


def _det_quantum(H, W, lists, cap):
    """Rounding bound of the deterministic mode per site: every gradient term is rounded
    once to the unit 2^-(20 + e) (2^e the power of two just below P, 2^(e+1) >= P), an
    error of at most half a unit per term, and a site receives one term per parameter
    from every pixel whose list holds it."""
    e = 0
    while (1 << (e + 1)) < H * W:
        e += 1
    ids = lists[lists != 0xFFFFFFFF].astype(np.int64)
    n_terms = np.bincount(ids, minlength=cap)[:cap].astype(np.float64)
    return n_terms * 2.0 ** -(21 + e)


def _compare(label, H, W, got, ref, det=False):
    lists, col, gimg, loss, grad = got
    rlists, rcol, rL, rg, rgrad, ab = ref
    if det:  # the deterministic mode's documented per-term rounding, added to the rule
        ab = ab + _det_quantum(H, W, rlists, ab.shape[1])[None, :] / 1e-5
    bad = np.argwhere(np.any(lists != rlists, axis=1)).ravel()
    assert bad.size == 0, f"{label}: {bad.size} pixels differ, first {bad[:5]}"
    err = np.abs(col - rcol).max()
    assert err <= 1e-5, f"{label}: colour error {err}"
    P = H * W
    gerr = np.abs(gimg - rg).max()
    assert gerr <= 2.0 / P * 2e-5, f"{label}: dL/dc error {gerr} (2/P = {2.0 / P})"
    assert abs(loss - rL) <= 1e-5 * rL, f"{label}: loss {loss} vs {rL}"
    w, plain, rep = grad_check(grad, rgrad, ab, label)
    assert w <= 1.0, f"{label}: gradient mismatch ratio {w}\n{rep}"


@pytest.mark.parametrize("K", [4, 8, 16, 32])
def test_fused_pass_whole_field_768x512(S, K):
    """768x512, N = 20 000, J = 4: the fused pass at pass 2 (jump 256) and pass 10 (jump
    1, the steady state where most candidates repeat) from the oracle's fields."""
    H, W, N, J, seed = 512, 768, 20000, 4, 21
    target, sites, s = _encode_sites(K, H, W, N)
    F = _fields(H, W, K, s, sites, N, J, seed, 10)
    for t in (2, 10):
        got = _fused(S, H, W, K, s, sites, N, F[t], J, seed, t, target)
        ref = _oracle_pass(H, W, K, s, sites, N, F[t], J, seed, t, target)
        _compare(f"fused K={K} 768x512 pass {t}", H, W, got, ref)


def test_fused_pass_deterministic_768x512(S):
    """The deterministic (integer-sum) form of the fused pass against the oracle."""
    H, W, N, J, seed, K = 512, 768, 20000, 4, 22, 8
    target, sites, s = _encode_sites(5, H, W, N)
    F = _fields(H, W, K, s, sites, N, J, seed, 10)
    got = _fused(S, H, W, K, s, sites, N, F[10], J, seed, 10, target, deterministic=True)
    ref = _oracle_pass(H, W, K, s, sites, N, F[10], J, seed, 10, target)
    _compare("fused deterministic K=8 768x512 pass 10", H, W, got, ref, det=True)


def _edge_case(name):
    if name == "hard_limit":
        # half the sites at log tau = 20 (the clamp maximum: nearly hard ownership)
        H, W, N, K = 48, 80, 300, 8
        target = synth.image_encode(31, H, W, n_polygons=10, patch=16)
        sites = synth.random_sites(32, H, W, N, anisotropic=True, log_tau_range=(3.0, 7.0),
                                   r_range=(1.0, 3.0))
        sites[2, ::2] = 20.0
        return target, sites, H, W, K, N, O.default_scale(H, W)
    if name == "all_hard":
        H, W, N, K = 40, 56, 200, 4
        target = synth.image_encode(33, H, W, n_polygons=10, patch=16)
        sites = synth.random_sites(34, H, W, N, anisotropic=True, log_tau=20.0,
                                   r_range=(1.0, 3.0))
        return target, sites, H, W, K, N, O.default_scale(H, W)
    if name == "k_ge_active":
        # 6 active sites of 10 slots (two inactive, one non-finite, one free), K = 8
        H, W, N, K = 37, 53, 10, 8
        target = synth.image_encode(35, H, W, n_polygons=5, patch=8)
        sites = synth.random_sites(36, H, W, N, anisotropic=True, log_tau_range=(2.0, 4.0),
                                   r_range=(1.0, 3.0))
        sites[0:2, [1, 4]] = -1.0
        sites[3, 7] = np.inf
        sites[0:2, 9] = -1.0
        return target, sites, H, W, K, N, O.default_scale(H, W)
    if name == "k_eq_n":
        H, W, N, K = 29, 31, 8, 8
        target = synth.image_encode(37, H, W, n_polygons=5, patch=8)
        sites = synth.random_sites(38, H, W, N, anisotropic=True, log_tau_range=(2.0, 4.0),
                                   r_range=(1.0, 3.0))
        return target, sites, H, W, K, N, O.default_scale(H, W)
    if name in ("ragged_k12", "ragged_k20", "ragged_k28"):
        K = int(name[-2:])
        H, W, N = 33, 47, 150 + 10 * K
        target = synth.image_encode(39 + K, H, W, n_polygons=8, patch=8)
        sites = synth.random_sites(40 + K, H, W, N, anisotropic=True, log_tau_range=(2.0, 7.0),
                                   r_range=(1.0, 4.0))
        return target, sites, H, W, K, N, O.default_scale(H, W)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["hard_limit", "all_hard", "k_ge_active", "k_eq_n",
                                  "ragged_k12", "ragged_k20", "ragged_k28"])
def test_fused_pass_edge_cases(S, name):
    """Free-running fused passes (each from the oracle's previous field) over the whole
    schedule and beyond; with K >= the active count the lists end equal to brute force."""
    target, sites, H, W, K, N, s = _edge_case(name)
    J, seed = 2, 41
    lists = O.seed_lists(H, W, K, s, sites, N)
    for t in range(12):
        got = _fused(S, H, W, K, s, sites, N, lists, J, seed, t, target)
        ref = _oracle_pass(H, W, K, s, sites, N, lists, J, seed, t, target)
        _compare(f"fused {name} pass {t}", H, W, got, ref)
        lists = ref[0]
    if name in ("k_ge_active", "k_eq_n"):
        assert np.array_equal(lists, O.brute_topk(H, W, K, s, sites, N))


@pytest.mark.parametrize("K", [4, 12, 16, 32])
def test_fused_pass_deterministic_small(S, K):
    """The deterministic fused pass at the other list lengths (each its own kernel
    instance; K = 16 carries its own register cap) against the oracle, over the first
    passes of the schedule from the seed pass."""
    H, W, N, J, seed = 41, 67, 260, 3, 23
    target = synth.image_encode(60 + K, H, W, n_polygons=9, patch=12)
    sites = synth.random_sites(61 + K, H, W, N, anisotropic=True, log_tau_range=(2.0, 6.0),
                               r_range=(1.0, 3.0))
    s = O.default_scale(H, W)
    lists = O.seed_lists(H, W, K, s, sites, N)
    for t in range(5):
        got = _fused(S, H, W, K, s, sites, N, lists, J, seed, t, target, deterministic=True)
        ref = _oracle_pass(H, W, K, s, sites, N, lists, J, seed, t, target)
        _compare(f"fused deterministic K={K} pass {t}", H, W, got, ref, det=True)
        lists = ref[0]


@pytest.mark.parametrize("N", [100_000, 400_000])
def test_fused_pass_2048_k16(S, N):
    """2048x2048, N = 100 000 and 400 000 (the start and the capacity of the large
    budget-controlled encode; oracle initialisation, moved), K = 16, J = 4: the fused
    pass at pass 2 from the oracle's field after the seed pass and two passes, whole
    field (the K = 16 kernel carries its own register cap)."""
    H = W = 2048
    K, J, seed = 16, 4, 9
    target = synth.image_large(0, H, W)
    lt0 = float(np.clip(math.log(2 * max(H, W) / math.sqrt(H * W / N)), 2, 20))
    sites, _ = O.init_sites(target, N, 0.3, 3, lt0, 1.0, N)
    sites = synth.perturb_sites(4, sites, N, H, W)
    s = O.default_scale(H, W)
    F = _fields(H, W, K, s, sites, N, J, seed, 2)
    got = _fused(S, H, W, K, s, sites, N, F[2], J, seed, 2, target)
    ref = _oracle_pass(H, W, K, s, sites, N, F[2], J, seed, 2, target)
    _compare(f"fused K=16 2048x2048 N={N} pass 2", H, W, got, ref)


BATCH_SHAPES = [(64, 80, 300), (96, 50, 250), (130, 77, 520), (33, 47, 60), (16, 16, 12),
                (70, 200, 700)]


@pytest.mark.parametrize("grid,chunked,det,tile_w,K", [(0, 0, False, 16, 8), (5, 1, False, 16, 8),
                                                       (0, 0, True, 16, 8), (7, 0, True, 16, 8),
                                                       (0, 0, False, 32, 8), (5, 1, True, 32, 8),
                                                       (0, 0, False, 16, 16), (5, 1, True, 32, 16),
                                                       (0, 0, True, 16, 4)])
def test_batch_step_matches_oracle_per_image(S, grid, chunked, det, tile_w, K):
    """sad_batch_train_step, image by image, against the oracle: every image starts from
    its own oracle field at its own pass index; lists, loss and gradient per image."""
    from paper_2604_21984_amd import batch as B
    from paper_2604_21984_amd import encode as E
    J = 4
    targets = [synth.image_encode(50 + i, H, W, n_polygons=15, patch=16)
               for i, (H, W, _) in enumerate(BATCH_SHAPES)]
    cfg = E.EncodeConfig(K=K, n_inject=J, seed=6, deterministic=det)
    be = B.BatchEncoder([_t(x) for x in targets], [n for _, _, n in BATCH_SHAPES], cfg,
                        grid=grid, chunked=chunked, tile_w=tile_w)
    be.adam = S.adam_params([0.0] * 10, cfg.beta1, cfg.beta2, cfg.eps)
    be.train_cfg = S.train_config(J, be.train_cfg.seed, be.adam, deterministic=det)
    seed = be.train_cfg.seed
    refs = []
    for b, (H, W, N) in enumerate(BATCH_SHAPES):
        s = O.default_scale(H, W)
        sites = synth.perturb_sites(60 + b, synth.random_sites(70 + b, H, W, N, log_tau=4.0,
                                                               r=1.0), N, H, W)
        t = 3 * b                           # each image at its own pass index
        F = _fields(H, W, K, s, sites, N, J, seed, t)
        be.view_sites(b).copy_(_t(sites))
        S.prepare_sites(be.img(b), be.view_sites(b), be.view_rec(b))
        be.view_list(be.cur, b).copy_(_t(rows_to_planar(F[t], H, W, K)))
        be.state(b).zero_()
        be.state(b)[0] = t
        refs.append(_oracle_pass(H, W, K, s, sites, N, F[t], J, seed, t, targets[b]))
    be.m.zero_()
    be.v.zero_()
    be.grad.zero_()
    be.step()
    torch.cuda.synchronize()
    losses = be.losses()
    b1 = np.float64(np.float32(1.0) - np.float32(cfg.beta1))
    for b, (H, W, N) in enumerate(BATCH_SHAPES):
        rlists, rcol, rL, rg, rgrad, ab = refs[b]
        lists = planar_to_rows(be.view_list(be.cur, b).cpu().numpy(), H, W, K)
        assert np.array_equal(lists, rlists), f"image {b}: lists differ"
        assert abs(losses[b] - rL) <= 1e-5 * rL, (b, losses[b], rL)
        m = be.view_sites(b, be.m).cpu().numpy().astype(np.float64)
        if det:  # the deterministic mode's per-term rounding at this image's own P
            ab = ab + _det_quantum(H, W, rlists, ab.shape[1])[None, :] / 1e-5
        w, plain, rep = grad_check(m / b1, rgrad, ab,
                                   f"batch grid={grid} chunked={chunked} det={det} tile={tile_w} "
                                   f"K={K} image {b}")
        assert w <= 1.0, f"image {b}: gradient mismatch ratio {w}\n{rep}"
