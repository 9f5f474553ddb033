"""GPU: the batched persistent launch against per-image encoders with the same
settings, its HIP-graph replay, and the autotuner."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
SHAPES = [(64, 80, 300), (96, 50, 250), (130, 77, 520), (33, 47, 60), (16, 16, 12), (70, 200, 700)]


@pytest.fixture(scope="module")
def mods():
    from paper_2604_21984_amd import _lib as S
    from paper_2604_21984_amd import autotune as T
    from paper_2604_21984_amd import batch as B
    from paper_2604_21984_amd import encode as E
    return S, B, E, T


def _targets():
    return [torch.from_numpy(synth.image_encode(10 + i, H, W, n_polygons=15, patch=16)).to(DEV)
            for i, (H, W, _) in enumerate(SHAPES)]


def test_batch_equals_per_image_encoders(mods):
    S, B, E, T = mods
    cfg = E.EncodeConfig(K=8, n_inject=4, seed=3)
    tg = _targets()
    be = B.BatchEncoder(tg, [n for _, _, n in SHAPES], cfg, grid=0, chunked=0)
    singles = [E.Encoder(t, n, cfg) for t, (_, _, n) in zip(tg, SHAPES)]
    for b, enc in enumerate(singles):  # identical initial state
        assert torch.equal(be.view_sites(b), enc.sites)
        assert torch.equal(be.view_list(0, b), enc.topk)
    be.step()
    for enc in singles:
        enc.step()
    torch.cuda.synchronize()
    for b, enc in enumerate(singles):
        assert torch.equal(be.view_list(be.cur, b), enc.topk), b
        torch.testing.assert_close(be.view_sites(b), enc.sites, rtol=1e-5, atol=1e-5)
    for _ in range(5):
        be.step()
        for enc in singles:
            enc.step()
    torch.cuda.synchronize()
    lb = be.losses()
    for b, enc in enumerate(singles):
        assert abs(lb[b] - enc.loss_value()) <= 1e-4 * enc.loss_value(), b
        agree = (be.view_list(be.cur, b) == enc.topk).float().mean().item()
        assert agree > 0.999, (b, agree)
    assert [int(x) for x in be.state(2)[:2].tolist()] == [6, 6]


@pytest.mark.parametrize("grid,chunked,tile_w", [(0, 0, 16), (7, 1, 16), (5, 0, 16), (3, 1, 16),
                                                 (0, 0, 32), (7, 1, 32), (5, 0, 32)])
def test_batch_launch_shapes_agree(mods, grid, chunked, tile_w):
    """Every launch form and tile shape gives the same lists (bit for bit) and the same
    parameters up to the order of the float sums."""
    S, B, E, T = mods
    cfg = E.EncodeConfig(K=8, n_inject=4, seed=5)
    tg = _targets()
    ref = B.BatchEncoder(tg, [n for _, _, n in SHAPES], cfg, grid=0, chunked=0)
    alt = B.BatchEncoder(tg, [n for _, _, n in SHAPES], cfg, grid=grid, chunked=chunked,
                         tile_w=tile_w)
    ref.step()
    alt.step()
    torch.cuda.synchronize()
    assert torch.equal(ref.lists[1], alt.lists[1])
    torch.testing.assert_close(ref.sites, alt.sites, rtol=1e-5, atol=1e-5)


def test_batch_graph_replay_and_autotune(mods):
    S, B, E, T = mods
    cfg = E.EncodeConfig(K=8, n_inject=4, seed=9)
    tg = _targets()
    eager = B.BatchEncoder(tg, [n for _, _, n in SHAPES], cfg)
    graphed = B.BatchEncoder(tg, [n for _, _, n in SHAPES], cfg)
    before = graphed.sites.clone()
    grid, chunked, timings = T.Autotuner().tune(graphed, pairs=1, reps=1)
    assert len(timings) >= 2 and graphed.tile_w in (16, 32)
    assert any(k.endswith("/32") for k in timings) and any(k.endswith("/16") for k in timings)
    assert torch.equal(graphed.sites, before)          # tuning leaves the encode untouched
    graphed.capture()
    for _ in range(3):
        eager.step()
        eager.step()
        graphed.replay(1)
        torch.cuda.synchronize()
        np.testing.assert_allclose(graphed.losses(), eager.losses(), rtol=1e-4)
    torch.testing.assert_close(graphed.sites, eager.sites, rtol=1e-4, atol=1e-4)


def test_autotune_update_period_at_equal_wall_time(mods):
    """The schedule trials: the first period runs the window, every other period stops
    before it would run longer than that; the chosen period is applied, the encode's
    state is left as it was, and a second call returns the cached choice."""
    S, B, E, T = mods
    cfg = E.EncodeConfig(K=8, n_inject=4, seed=11)
    tg = _targets()
    be = B.BatchEncoder(tg, [n for _, _, n in SHAPES], cfg)
    before = (be.sites.clone(), be.lists[be.cur].clone())
    tuner = T.Autotuner()
    _, _, timings = tuner.tune(be, pairs=1, reps=1, schedules=(1, 2), window=16,
                               tile_widths=(16,))
    pe = timings["prop_every"]
    assert set(pe) == {"1", "2"} and pe["1"]["iterations"] == 16
    assert pe["2"]["iterations"] >= 2 and pe["2"]["iterations"] % 2 == 0
    assert pe["2"]["iterations"] == 2 or pe["2"]["ms"] <= pe["1"]["ms"] * 1.0001
    best = timings["prop_every_best"]
    assert best == min((1, 2), key=lambda f: (pe[str(f)]["loss"], f))
    assert be.train_cfg.prop_every == best
    assert torch.equal(be.sites, before[0]) and torch.equal(be.lists[be.cur], before[1])
    be.set_prop_every(1)
    tuner.tune(be, pairs=1, reps=1, schedules=(1, 2), window=16, tile_widths=(16,))
    assert be.train_cfg.prop_every == best


def test_deterministic_batch_equals_per_image_bitwise(mods):
    """With deterministic gradient sums every image of the batch follows its per-image
    encoder bit for bit (same tiles, exact tile sums, one rounding each, integer sums),
    over several iterations, for both batched launch forms; and two batched runs agree."""
    S, B, E, T = mods
    cfg = E.EncodeConfig(K=8, n_inject=4, seed=4, deterministic=True)
    tg = _targets()
    ns = [n for _, _, n in SHAPES]
    singles = [E.Encoder(t, n, cfg) for t, n in zip(tg, ns)]
    runs = [B.BatchEncoder(tg, ns, cfg, grid=0, chunked=0),
            B.BatchEncoder(tg, ns, cfg, grid=5, chunked=1),
            B.BatchEncoder(tg, ns, cfg, grid=0, chunked=0, tile_w=32)]
    for _ in range(6):
        for enc in singles:
            enc.step()
        for be in runs:
            be.step()
    torch.cuda.synchronize()
    for be in runs:
        for b, enc in enumerate(singles):
            assert torch.equal(be.view_sites(b), enc.sites), b
            assert torch.equal(be.view_list(be.cur, b), enc.topk), b
    assert torch.equal(runs[0].sites, runs[1].sites)
    assert torch.equal(runs[0].sites, runs[2].sites)
    assert (runs[0].grad == 0).all()


def test_deterministic_batch_full_size_equals_per_image(mods):
    """The batched-encode workload at its full size (64 images of 256^2 to 1024^2 pixels,
    26.2 Mpx, 0.05 sites per pixel, K = 8): in the deterministic mode every image of the
    batch, in the launch the benchmark times (one workgroup per 16 x 16 tile) and in the
    persistent form with contiguous runs of tiles, equals its per-image encoder bit for
    bit after four iterations (the per-image encoder is checked against the oracle at
    768 x 512 in test_gpu_train_oracle)."""
    from concurrent.futures import ThreadPoolExecutor
    S, B, E, T = mods
    shapes = synth.batch_shapes(0)
    print(f"full-size batch: {len(shapes)} images, "
          f"{sum(h * w for h, w, _ in shapes)} px", flush=True)
    with ThreadPoolExecutor(8) as ex:
        imgs = list(ex.map(lambda a: synth.image_encode(100 + a[0], a[1][0], a[1][1],
                                                        n_polygons=20), enumerate(shapes)))
    tg = [torch.from_numpy(im).to(DEV) for im in imgs]
    ns = [n for _, _, n in shapes]
    cfg = E.EncodeConfig(K=8, n_inject=4, seed=2, deterministic=True)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    runs = [B.BatchEncoder(tg, ns, cfg, grid=0, chunked=0),
            B.BatchEncoder(tg, ns, cfg, grid=4 * n_cu, chunked=1)]
    for _ in range(4):
        for be in runs:
            be.step()
    torch.cuda.synchronize()
    assert torch.equal(runs[0].sites, runs[1].sites)
    assert torch.equal(runs[0].lists[runs[0].cur], runs[1].lists[runs[1].cur])
    be = runs[0]
    for b, (t, n) in enumerate(zip(tg, ns)):
        enc = E.Encoder(t, n, cfg)
        for _ in range(4):
            enc.step()
        torch.cuda.synchronize()
        assert torch.equal(be.view_sites(b), enc.sites), b
        assert torch.equal(be.view_list(be.cur, b), enc.topk), b
        del enc
