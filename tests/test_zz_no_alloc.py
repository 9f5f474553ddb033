"""The seed pass without allocation (sad_seed_topk_noalloc) against sad_seed_topk, through
the C ABI: two calls in a row on the device's shared static scratch, the second with a
smaller image, each bit-exact against the scratch-argument entry point; an image beyond
the static size is rejected before anything is enqueued."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def S():
    import paper_2604_21984_amd._lib as S
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return S


def _seeded_pair(S, H, W, K, n, seed):
    sites = synth.random_sites(seed, H, W, n, anisotropic=True, log_tau_range=(2.0, 6.0),
                               r_range=(1.0, 3.0))
    sites[0:2, 7] = -1.0
    img = S.image(H, W, K, n, n)
    sd = torch.from_numpy(sites).to(DEV)
    rec = torch.empty(n * 16, dtype=torch.float32, device=DEV)
    S.prepare_sites(img, sd, rec)
    want = torch.empty((K // 4, H, W, 4), dtype=torch.int32, device=DEV)
    scratch = torch.empty(H * W, dtype=torch.int64, device=DEV)
    S.seed_topk(img, rec, want, scratch)
    got = torch.full_like(want, 3)
    S.seed_topk_noalloc(img, rec, got)
    return img, rec, want, got


def test_noalloc_seed_matches_scratch_argument_form(S):
    # the first call is large (most sites crowd few pixels: many bid rounds per pixel),
    # the second smaller, so it starts on the first call's leftover scratch words
    cases = [(1024, 1536, 16, 200_000, 1), (37, 53, 8, 400, 2)]
    for H, W, K, n, seed in cases:
        _, _, want, got = _seeded_pair(S, H, W, K, n, seed)
        torch.cuda.synchronize()
        assert torch.equal(got, want), f"{H}x{W} K={K}: lists differ"
        assert int((got != -1).sum()) > 0


def test_noalloc_seed_limits(S):
    H, W, K, n = 2048, 2048, 4, 1000           # exactly the static size: accepted
    _, _, want, got = _seeded_pair(S, H, W, K, n, 5)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    assert H * W == S.SEED_STATIC_PIXELS
    big = S.image(2049, 2048, 4, n, n)          # one row more: rejected, nothing enqueued
    rec = torch.zeros(n * 16, dtype=torch.float32, device=DEV)
    topk = torch.empty((1, 2049, 2048, 4), dtype=torch.int32, device=DEV)
    with pytest.raises(S.SadError, match="static scratch"):
        S.seed_topk_noalloc(big, rec, topk)
    empty = S.image(20, 30, 4, 0, 0)            # no sites: every entry cleared
    t = torch.full((1, 20, 30, 4), 9, dtype=torch.int32, device=DEV)
    S.seed_topk_noalloc(empty, None, t)
    torch.cuda.synchronize()
    assert bool((t == -1).all())
