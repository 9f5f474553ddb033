"""GPU: the training iteration (sad_train_step), its HIP-graph replay, and the
autograd wrapper, against direct C-ABI calls and the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _helpers import grad_close, planar_to_rows, rows_to_planar

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def mods():
    from paper_2604_21984_amd import _lib as S
    from paper_2604_21984_amd import autograd as A
    from paper_2604_21984_amd import encode as E
    return S, A, E


def _enc(E, H=96, W=130, N=600, seed=0):
    target = torch.from_numpy(synth.image_encode(seed, H, W, n_polygons=25, patch=24)).to(DEV)
    return E.Encoder(target, N, E.EncodeConfig(K=8, n_inject=4, seed=seed))


def test_train_step_equals_individual_calls(mods):
    S, A, E = mods
    enc = _enc(E)
    # replica of the state, driven through the individual entry points
    sites = enc.sites.clone()
    rec = enc.rec.clone()
    la, lb = enc.lists[0].clone(), enc.lists[1].clone()
    m, v = enc.m.clone(), enc.v.clone()
    grad = torch.zeros_like(enc.grad)
    out = torch.empty_like(enc.rendered)
    gimg = torch.empty_like(enc.grad_img)
    loss = S.loss_acc(DEV)
    img = enc.img
    for t in range(4):
        enc.step()
        S.propagate_topk(img, rec, la, lb, S.jump_step(t, enc.H, enc.W), 4,
                         enc.train_cfg.seed, t)
        S.render_fwd(img, rec, lb, out)
        loss.zero_()
        S.loss_grad(img, out, enc.target, gimg, loss)
        gimg2 = torch.empty_like(gimg)
        loss2 = S.loss_acc(DEV)
        out2 = torch.empty_like(out)
        S.render_fwd_loss(img, rec, lb, enc.target, gimg2, out2, loss2)
        assert torch.equal(out2, out) and torch.equal(gimg2, gimg)
        assert abs(loss2[0].item() - loss[0].item()) <= 1e-6 * loss[0].item()
        grad.zero_()
        S.render_bwd(img, rec, lb, gimg, grad)
        S.adam_step(img, sites, grad, m, v, enc.adam, t + 1, rec)
        la, lb = lb, la
        torch.cuda.synchronize()
        if t == 0:
            assert torch.equal(enc.topk, la)
        assert abs(enc.loss_value() - loss[0].item()) <= 1e-6 * loss[0].item()
    assert enc.counters() == [4, 4]
    torch.testing.assert_close(enc.sites, sites, rtol=1e-5, atol=1e-5)
    agree = (enc.topk == la).float().mean().item()
    assert agree > 0.999


def test_candidate_update_period(mods):
    """prop_every = 2: even iterations are passes t/2 of the schedule and injection
    stream, odd ones re-score and sort each pixel's own list (lr = 0 keeps the sites
    fixed, so every list is a deterministic function of the previous one)."""
    S, A, E = mods
    H, W, N = 80, 112, 500
    target = torch.from_numpy(synth.image_encode(6, H, W, n_polygons=20, patch=16)).to(DEV)
    enc = E.Encoder(target, N, E.EncodeConfig(K=8, n_inject=4, seed=2, lr=0.0, prop_every=2))
    rec = enc.rec.clone()
    la, lb = enc.lists[0].clone(), enc.lists[1].clone()
    img, seed = enc.img, enc.train_cfg.seed
    for t in range(7):
        enc.step()
        if t % 2 == 0:
            S.propagate_topk(img, rec, la, lb, S.jump_step(t // 2, H, W), 4, seed, t // 2)
        else:
            S.propagate_topk(img, rec, la, lb, max(H, W), 0, seed, 0)
        la, lb = lb, la
        torch.cuda.synchronize()
        assert torch.equal(enc.topk, la), t
    assert torch.equal(enc.rec, rec)


def test_graph_replay_matches_eager(mods):
    S, A, E = mods
    eager, graphed = _enc(E, seed=3), _enc(E, seed=3)
    graphed.capture()
    losses_e, losses_g = [], []
    for r in range(4):
        eager.step()
        eager.step()
        graphed.replay(1)
        torch.cuda.synchronize()
        losses_e.append(eager.loss_value())
        losses_g.append(graphed.loss_value())
        # eager host work and a synchronisation between replays
        _ = graphed.render().sum().item()
    np.testing.assert_allclose(losses_g, losses_e, rtol=1e-4)
    assert graphed.counters() == [8, 8]
    torch.testing.assert_close(graphed.sites, eager.sites, rtol=1e-4, atol=1e-4)
    assert (graphed.topk == eager.topk).float().mean().item() > 0.999


def test_autograd_render_matches_oracle(mods):
    S, A, E = mods
    H, W, N, K = 40, 52, 150, 8
    sites_np = synth.random_sites(4, H, W, N, cap=160, anisotropic=True,
                                  log_tau_range=(3, 6), r_range=(1, 3))
    s = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, s, sites_np, N)
    target_np = synth.image_encode(2, H, W, n_polygons=8, patch=16)
    img = S.image(H, W, K, N, 160)
    sites = torch.from_numpy(sites_np).to(DEV).requires_grad_(True)
    topk = torch.from_numpy(rows_to_planar(lists, H, W, K)).to(DEV)
    target = torch.from_numpy(target_np).to(DEV)
    out = A.render(sites, topk, img)
    loss = A.mse_loss(out, target, img)
    loss.backward()
    ref_img = O.render(H, W, K, s, sites_np, N, lists)
    L, g = O.loss_grad(ref_img, target_np)
    ref, ab = O.render_bwd(H, W, K, s, sites_np, N, lists, g, abs_sum=True)
    assert abs(loss.item() - L) <= 1e-5 * L
    assert np.abs(out.detach().cpu().numpy() - ref_img).max() <= 1e-5
    assert grad_close(sites.grad.cpu().numpy(), ref, ab) <= 1.0
    # torch's own MSE (scaled to the paper's normalisation) drives the same backward
    sites.grad = None
    out = A.render(sites, topk, img)
    ((out - target) ** 2).sum(0).mean().backward()
    assert grad_close(sites.grad.cpu().numpy(), ref, ab) <= 1.0


def test_fused_autograd_pass_matches_oracle(mods):
    """SADTrainPass: one fused pass behind the autograd Function; the loss, the new lists
    and the gradient (handed out by backward, scaled by the incoming gradient) against
    the oracle's pass, blend, loss and backward; the accumulator is cleared for the next
    call."""
    S, A, E = mods
    H, W, N, K, J, seed = 40, 52, 150, 8, 3, 17
    sites_np = synth.random_sites(4, H, W, N, cap=160, anisotropic=True,
                                  log_tau_range=(3, 6), r_range=(1, 3))
    s = O.default_scale(H, W)
    lists = O.seed_lists(H, W, K, s, sites_np, N)
    for t in range(5):
        lists = O.prop_pass(H, W, K, s, sites_np, N, lists, O.jump(t, H, W), J, seed, t)
    target_np = synth.image_encode(2, H, W, n_polygons=8, patch=16)
    img = S.image(H, W, K, N, 160)
    sites = torch.from_numpy(sites_np).to(DEV).requires_grad_(True)
    topk_in = torch.from_numpy(rows_to_planar(lists, H, W, K)).to(DEV)
    topk_out = torch.empty_like(topk_in)
    target = torch.from_numpy(target_np).to(DEV)
    rec = torch.empty(N * S.REC_FLOATS, dtype=torch.float32, device=DEV)
    gacc = torch.zeros((160, 10), dtype=torch.float32, device=DEV)
    state = S.step_state(DEV)
    state[0] = 5
    cfg = S.train_config(J, seed, S.adam_params([0.0] * 10))
    loss = A.SADTrainPass.apply(sites, target, img, cfg, rec, topk_in, topk_out, gacc, state, True)
    (3.0 * loss).backward()
    new = O.prop_pass(H, W, K, s, sites_np, N, lists, O.jump(5, H, W), J, seed, 5)
    ref_img = O.render(H, W, K, s, sites_np, N, new)
    L, g = O.loss_grad(ref_img, target_np)
    ref, ab = O.render_bwd(H, W, K, s, sites_np, N, new, g, abs_sum=True)
    assert np.array_equal(planar_to_rows(topk_out.cpu().numpy(), H, W, K), new)
    assert abs(loss.item() - L) <= 1e-5 * L
    assert grad_close(sites.grad.cpu().numpy() / 3.0, ref, ab) <= 1.0
    assert float(gacc.abs().max()) == 0.0
    # with SAD_TRAIN_LOSS_SET the pass stores L: a stale value in the state does not leak
    cfg2 = S.train_config(J, seed, S.adam_params([0.0] * 10), loss_set=True)
    S.state_loss(state).fill_(123.0)
    loss2 = A.SADTrainPass.apply(sites.detach(), target, img, cfg2, rec, topk_in, topk_out,
                                 gacc, state, False)
    assert abs(loss2.item() - L) <= 1e-5 * L


def test_fused_autograd_trainer_graph_matches_eager(mods):
    """FusedAutogradTrainer recorded as a HIP graph against the same iterations eagerly;
    its trajectory also follows the separate-kernel autograd trainer."""
    S, A, E = mods
    enc = _enc(E, seed=6)
    for _ in range(4):
        enc.step()
    torch.cuda.synchronize()
    mk = lambda cls: cls(enc.img, enc.sites, enc.topk, enc.target, enc.adam, n_inject=4,
                         seed=11)
    eager, graphed = mk(A.FusedAutogradTrainer), mk(A.FusedAutogradTrainer)
    plain = mk(A.AutogradTrainer)
    graphed.capture(pairs=1, warmup=2)
    for _ in range(4):
        eager.step()
        plain.step()
    torch.cuda.synchronize()
    assert graphed.counters() == eager.counters() == plain.counters() == (4, 4)
    for r in range(4):
        graphed.replay(1)
        for _ in range(2):
            eager.step()
            plain.step()
        torch.cuda.synchronize()
        assert graphed.counters() == eager.counters() == (6 + 2 * r, 6 + 2 * r)
        np.testing.assert_allclose(graphed.loss.item(), eager.loss.item(), rtol=1e-4)
        np.testing.assert_allclose(plain.loss.item(), eager.loss.item(), rtol=1e-3)
        torch.testing.assert_close(graphed.sites.detach(), eager.sites.detach(),
                                   rtol=1e-4, atol=1e-4)
        torch.testing.assert_close(plain.sites.detach(), eager.sites.detach(),
                                   rtol=1e-3, atol=1e-3)


def test_encode_improves_psnr(mods):
    S, A, E = mods
    enc = _enc(E, H=128, W=192, N=1500, seed=5)
    p0 = enc.psnr()
    for _ in range(100):
        enc.step()
    p1 = enc.psnr()
    assert p1 > p0 + 3.0, (p0, p1)


def test_fused_image_pass_equals_separate_kernels(mods):
    S, A, E = mods
    enc = _enc(E, H=100, W=150, N=900, seed=7)
    for _ in range(12):
        enc.step()
    torch.cuda.synchronize()
    img = enc.img
    a = enc.topk
    t = enc.counters()[0]
    # fused pass (pass index from the device state; the state is not advanced)
    lf = torch.empty_like(a)
    gf = torch.zeros_like(enc.grad)
    gif = torch.empty_like(enc.grad_img)
    S.train_image_pass(img, enc.train_cfg, enc.target, enc.rec, a, lf, gf, None, gif, enc.state)
    # the same work through the separate entry points
    ls = torch.empty_like(a)
    S.propagate_topk(img, enc.rec, a, ls, S.jump_step(t, enc.H, enc.W), 4, enc.train_cfg.seed, t)
    gis = torch.empty_like(enc.grad_img)
    S.render_fwd_loss(img, enc.rec, ls, enc.target, gis)
    gs = torch.zeros_like(enc.grad)
    S.render_bwd(img, enc.rec, ls, gis, gs)
    torch.cuda.synchronize()
    assert torch.equal(lf, ls)
    assert torch.equal(gif, gis)
    gf = gf.reshape(-1, 10).t()          # the fused pass accumulates site-major [cap][10]
    gs = gs.reshape(10, -1)
    scale = gs.abs().amax(dim=1, keepdim=True) + 1e-30
    assert ((gf - gs).abs() / scale).max().item() < 1e-5


def test_state_entry_points_match_host_counter_forms(mods):
    """sad_propagate_topk_state / sad_adam_step_state against the host-counter calls at
    the same pass index and Adam step: lists, sites, moments and records bit-identical;
    the Adam form advances the counters."""
    S, A, E = mods
    enc = _enc(E, seed=5)
    for _ in range(3):
        enc.step()
    torch.cuda.synchronize()
    img, H, W = enc.img, enc.H, enc.W
    state = S.step_state()
    for t in (0, 1, 5, 40):
        state[0] = t
        a = enc.topk.clone()
        b1, b2 = torch.empty_like(a), torch.empty_like(a)
        S.propagate_topk(img, enc.rec, a, b1, S.jump_step(t, H, W), 4, 99, t)
        S.propagate_topk_state(img, enc.rec, a, b2, 4, 99, state)
        torch.cuda.synchronize()
        assert torch.equal(b1, b2), t
    state.zero_()
    state[1] = 6
    g = torch.randn(10, img.cap, device=DEV) * 1e-3
    s1, s2 = enc.sites.clone(), enc.sites.clone()
    m1, m2 = torch.full_like(s1, 0.01), torch.full_like(s1, 0.01)
    v1, v2 = torch.full_like(s1, 0.02), torch.full_like(s1, 0.02)
    r1, r2 = enc.rec.clone(), enc.rec.clone()
    g1, g2 = g.clone(), g.clone()
    S.adam_step(img, s1, g1, m1, v1, enc.adam, 7, r1, zero_grad=True)
    S.adam_step_state(img, s2, g2, m2, v2, enc.adam, r2, state, zero_grad=True)
    torch.cuda.synchronize()
    for x, y in ((s1, s2), (m1, m2), (v1, v2), (r1, r2), (g1, g2)):
        assert torch.equal(x, y)
    assert S.state_counters(state).tolist() == [1, 7]


def test_autograd_trainer_graph_matches_eager(mods):
    """The autograd iteration recorded as a HIP graph against the same iterations run
    eagerly from the same state; eager work and a synchronisation between replays."""
    S, A, E = mods
    enc = _enc(E, seed=6)
    for _ in range(4):
        enc.step()
    torch.cuda.synchronize()
    mk = lambda: A.AutogradTrainer(enc.img, enc.sites, enc.topk, enc.target, enc.adam,
                                   n_inject=4, seed=11)
    eager, graphed = mk(), mk()
    graphed.capture(pairs=1, warmup=2)   # four eager iterations run, two recorded
    for _ in range(4):
        eager.step()
    torch.cuda.synchronize()
    assert graphed.counters() == eager.counters() == (4, 4)
    for r in range(4):
        graphed.replay(1)
        eager.step()
        eager.step()
        torch.cuda.synchronize()
        assert graphed.counters() == eager.counters() == (6 + 2 * r, 6 + 2 * r)
        np.testing.assert_allclose(graphed.loss.item(), eager.loss.item(), rtol=1e-4)
        _ = graphed.sites.detach().sum().item()
        torch.testing.assert_close(graphed.sites.detach(), eager.sites.detach(),
                                   rtol=1e-4, atol=1e-4)
        same = (graphed.lists[0] == eager.lists[0]).float().mean().item()
        assert same > 0.999, (r, same)


@pytest.mark.parametrize("K,every", [(8, 1), (16, 2)])
def test_deterministic_training_is_reproducible(mods, K, every):
    """Deterministic gradient sums: two encodes from the same seed are bit-identical after
    many iterations (graph replay included); one pass's int64 sums agree with the float
    sums of the default mode within the rounding of the units."""
    S, A, E = mods
    target = torch.from_numpy(synth.image_encode(8, 96, 130, n_polygons=25, patch=24)).to(DEV)
    cfg = E.EncodeConfig(K=K, n_inject=4, seed=8, deterministic=True, prop_every=every)
    a, b = E.Encoder(target, 600, cfg), E.Encoder(target, 600, cfg)
    for _ in range(10):
        a.step()
        b.step()
    b.capture(5)
    for _ in range(10):
        a.step()
    b.replay(1)
    torch.cuda.synchronize()
    assert a.counters() == b.counters()
    for x, y in ((a.sites, b.sites), (a.m, b.m), (a.v, b.v), (a.topk, b.topk), (a.rec, b.rec)):
        assert torch.equal(x, y)
    assert a.grad.dtype == torch.int64 and (a.grad == 0).all()
    # one image pass from a's state in both modes
    fcfg = S.train_config(4, 99, a.adam)
    dcfg = S.train_config(4, 99, a.adam, deterministic=True)
    gf = torch.zeros((a.img.cap, 10), dtype=torch.float32, device=DEV)
    gd = torch.zeros((a.img.cap, 10), dtype=torch.int64, device=DEV)
    outs = [torch.empty_like(a.topk) for _ in range(2)]
    for cfg_, g_, o_ in ((fcfg, gf, outs[0]), (dcfg, gd, outs[1])):
        st = S.step_state()
        S.train_image_pass(a.img, cfg_, a.target, a.rec, a.topk, o_, g_, None, None, st)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    H, W = a.H, a.W
    e = 0
    while (1 << (e + 1)) < H * W:
        e += 1
    unit = 2.0 ** -(20 + e)
    got = gd.cpu().numpy().astype(np.float64) * unit
    ref = gf.cpu().numpy().astype(np.float64)
    # each (pixel, entry) term of a site is rounded once to the unit (<= unit / 2 each);
    # the float sums of the default mode are exact per tile, rounded per tile sum
    ids = outs[0].cpu().numpy().astype(np.int64).reshape(-1) & 0xFFFFFFFF
    terms = np.bincount(ids[ids < a.img.n_slots], minlength=a.img.cap)[:, None]
    scale = np.abs(ref).max(axis=0, keepdims=True)
    assert (np.abs(got - ref) <= 0.5 * terms * unit + 1e-6 * scale).all()
