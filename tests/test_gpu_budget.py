"""GPU: adaptive budget (Sec. 4.5, App. B.5).  The statistics pass against the oracle
within a float32 bound; one prune / split / seed step against the oracle on the same
(oracle-made) statistics; the encoder's budget schedule end to end."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _helpers import planar_to_rows, rows_to_planar

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def S():
    from paper_2604_21984_amd import _lib
    return _lib


def _case(seed, H, W, N, K, cap=None, holes=0):
    cap = cap or N
    sites = synth.random_sites(seed, H, W, N, cap=cap, anisotropic=True,
                               log_tau_range=(2.5, 4.5), r_range=(1.0, 12.0))
    if holes:
        rng = np.random.default_rng(seed + 100)
        h = rng.choice(N, holes, replace=False)
        sites[0, h] = -1.0
        sites[1, h] = -1.0
    tg = synth.image_small(seed, H, W, n_shapes=10)
    s = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, s, sites, N)
    return sites, tg, s, lists


def _gpu_stats(S, H, W, K, N, cap, sites, lists, tg):
    img = S.image(H, W, K, N, cap)
    sd = torch.from_numpy(sites).to(DEV)
    rec = torch.empty(max(N, 1) * S.REC_FLOATS, dtype=torch.float32, device=DEV)
    S.prepare_sites(img, sd, rec)
    topk = torch.from_numpy(rows_to_planar(lists, H, W, K)).to(DEV)
    stats = torch.zeros((S.NSTAT, cap), dtype=torch.float32, device=DEV)
    S.site_stats(img, rec, topk, torch.from_numpy(tg).to(DEV), stats)
    torch.cuda.synchronize()
    return stats.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("H,W,N,K,holes", [(48, 64, 120, 4, 0), (70, 45, 200, 8, 17),
                                           (33, 50, 90, 16, 5), (16, 16, 3, 8, 0)])
def test_site_stats_match_oracle(S, H, W, N, K, holes):
    sites, tg, s, lists = _case(H + W, H, W, N, K, cap=N + 7, holes=holes)
    ref, sabs, sens = O.site_stats(H, W, K, s, sites, N, lists, tg, scales=True)
    got = _gpu_stats(S, H, W, K, N, N + 7, sites, lists, tg)
    # float32 bound: relative 1e-4, 2e-5 of the sum of |terms| (rounding of the sums)
    # and 1e-5 per unit of the sensitivity scale (colour error of the blend)
    floor = 1e-7 * np.abs(ref).max(axis=1, keepdims=True)
    tol = 1e-4 * np.abs(ref) + 2e-5 * sabs + 1e-5 * sens + floor
    bad = np.abs(got - ref) > tol
    assert not bad.any(), [(q, i, got[q, i], ref[q, i], tol[q, i]) for q, i in zip(*np.where(bad))][:5]
    assert (got[:, N:] == 0).all()                      # slots beyond n_slots untouched


@pytest.mark.parametrize("H,W,N,K,holes", [(48, 64, 120, 4, 0), (70, 45, 200, 8, 17),
                                           (33, 50, 90, 16, 5), (16, 16, 3, 8, 0)])
def test_site_stats_fixed_match_oracle_and_repeat(S, H, W, N, K, holes):
    """Integer-sum statistics: within the float32 bound of the oracle plus the per-term
    rounding to each statistic's unit, written (not accumulated) for every slot, and
    bit-identical from call to call."""
    sites, tg, s, lists = _case(H + W, H, W, N, K, cap=N + 7, holes=holes)
    ref, sabs, sens = O.site_stats(H, W, K, s, sites, N, lists, tg, scales=True)
    cap = N + 7
    img = S.image(H, W, K, N, cap)
    rec = torch.empty(max(N, 1) * S.REC_FLOATS, dtype=torch.float32, device=DEV)
    S.prepare_sites(img, torch.from_numpy(sites).to(DEV), rec)
    topk = torch.from_numpy(rows_to_planar(lists, H, W, K)).to(DEV)
    tgt = torch.from_numpy(tg).to(DEV)
    outs = []
    for fill in (float("nan"), 7.0):   # stale contents of stats and acc are overwritten
        stats = torch.full((S.NSTAT, cap), fill, dtype=torch.float32, device=DEV)
        acc = torch.full((2 * S.NSTAT * cap,), 12345, dtype=torch.int64, device=DEV)
        S.site_stats_fixed(img, rec, topk, tgt, acc, stats)
        torch.cuda.synchronize()
        outs.append(stats.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    got = outs[0].astype(np.float64)
    e = 0
    while (1 << (e + 1)) < H * W:
        e += 1
    unit = 2.0 ** -np.array([40, 40, 36, 36, 30, 30, 30, 40 + e], dtype=np.float64)
    floor = 1e-7 * np.abs(ref).max(axis=1, keepdims=True)
    tol = (1e-4 * np.abs(ref) + 2e-5 * sabs + 1e-5 * sens + floor +
           0.5 * H * W * unit[:, None])
    bad = np.abs(got - ref) > tol
    assert not bad.any(), [(q, i, got[q, i], ref[q, i], tol[q, i]) for q, i in zip(*np.where(bad))][:5]
    assert (got[:, N:] == 0).all()                      # slots beyond n_slots written zero


def test_deterministic_encode_with_budget_is_reproducible(S):
    """A deterministic encode with prune / split events: two runs from the same seed end
    with bit-identical sites, lists and budget counts."""
    from paper_2604_21984_amd import encode as E
    H, W = 96, 128
    tg = torch.from_numpy(synth.image_encode(4, H, W, n_polygons=25, patch=16)).to(DEV)
    sched = E.BudgetSchedule(densify_every=10, densify_start=10, densify_end=40, p_split=0.1,
                             prune_every=20, prune_start=20, prune_end=40, p_prune=0.05)
    cfg = E.EncodeConfig(K=8, n_inject=4, seed=3, budget=sched, deterministic=True)
    a, b = (E.Encoder(tg, 300, cfg, cap=900) for _ in range(2))
    for _ in range(45):
        a.step()
        b.step()
    torch.cuda.synchronize()
    assert [h["counts"] for h in a.budget_log] == [h["counts"] for h in b.budget_log]
    assert len(a.budget_log) == 4
    assert torch.equal(a.stats, b.stats)
    for x, y in ((a.sites, b.sites), (a.m, b.m), (a.v, b.v), (a.topk, b.topk)):
        assert torch.equal(x, y)


def _run_dp(S, H, W, K, sites, tg, stats, p_prune, p_split, flags, lists=None):
    cap = sites.shape[1]
    img = S.image(H, W, K, cap, cap)
    sd = torch.from_numpy(sites.copy()).to(DEV)
    am = torch.full((10, cap), 3.0, dtype=torch.float32, device=DEV)
    av = torch.full((10, cap), 5.0, dtype=torch.float32, device=DEV)
    st = torch.from_numpy(stats.astype(np.float32)).to(DEV)
    topk = None
    if lists is not None:
        topk = torch.from_numpy(rows_to_planar(lists, H, W, K)).to(DEV)
    counts = torch.zeros(6, dtype=torch.int64, device=DEV)
    ws = torch.empty(S.densify_workspace_bytes(img), dtype=torch.uint8, device=DEV)
    prm = S.budget_params(p_prune, p_split, flags)
    S.densify_prune(img, torch.from_numpy(tg).to(DEV), sd, am, av, st, prm, topk, counts, ws)
    torch.cuda.synchronize()
    out_lists = None if topk is None else planar_to_rows(topk.cpu().numpy(), H, W, K)
    return (sd.cpu().numpy(), am.cpu().numpy(), av.cpu().numpy(), counts.cpu().tolist(),
            out_lists)


def _compare_sites(got, ref):
    act_g, act_r = got[0] >= 0, ref[0] >= 0
    np.testing.assert_array_equal(act_g, act_r)
    np.testing.assert_array_equal(got[:, ~act_r][:2], ref[:, ~act_r][:2])
    # double-precision geometry on both sides, rounded to float once: equal up to the
    # last bit of a transcendental (log) or a rounding boundary
    np.testing.assert_allclose(got[:2], ref[:2], rtol=0, atol=1e-4)
    np.testing.assert_allclose(got[2:4], ref[2:4], rtol=1e-6, atol=0)
    np.testing.assert_allclose(got[7:10], ref[7:10], rtol=0, atol=2e-6)
    same_px = (np.rint(got[0]) == np.rint(ref[0])) & (np.rint(got[1]) == np.rint(ref[1]))
    np.testing.assert_array_equal(got[4:7, same_px], ref[4:7, same_px])
    assert same_px[act_r].mean() > 0.99


@pytest.mark.parametrize("flags,pp,ps", [(1, 0.2, 0.0), (2, 0.0, 0.3), (3, 0.1, 0.25),
                                         (7, 0.05, 0.5), (0, 0.5, 0.5)])
def test_densify_prune_matches_oracle(S, flags, pp, ps):
    H, W, K, N, cap = 64, 80, 8, 260, 400
    sites, tg, s, lists = _case(7, H, W, N, K, cap=cap, holes=30)
    stats = O.site_stats(H, W, K, s, sites, N, lists, tg).astype(np.float32)
    # a few sites without statistics exercise the gradient fallback
    stats[1:7, [3, 50, 77]] = 0.0
    ref = sites.copy()
    am = np.full((10, cap), 3.0, np.float32)
    av = np.full((10, cap), 5.0, np.float32)
    rl = lists.copy()
    rc = O.densify_prune(tg, ref, stats, pp, ps, flags, K=K, adam_m=am, adam_v=av,
                         lists=rl if flags & 4 else None)
    got, gm, gv, gc, gl = _run_dp(S, H, W, K, sites, tg, stats, pp, ps, flags,
                                  lists=lists if flags & 4 else None)
    assert gc == rc
    _compare_sites(got, ref)
    np.testing.assert_array_equal(gm, am)
    np.testing.assert_array_equal(gv, av)
    if flags & 4:
        np.testing.assert_array_equal(gl, rl)


def test_densify_prune_full_capacity_and_empty(S):
    H, W, K = 40, 40, 4
    sites, tg, s, lists = _case(3, H, W, 50, K)            # cap == N: nothing free
    stats = O.site_stats(H, W, K, s, sites, 50, lists, tg).astype(np.float32)
    ref = sites.copy()
    rc = O.densify_prune(tg, ref, stats, 0.0, 0.5, 2, K=K)
    got, *_, gc, _ = _run_dp(S, H, W, K, sites, tg, stats, 0.0, 0.5, 2)
    assert gc == rc and gc[2] == 0
    np.testing.assert_array_equal(got, ref)
    dead = sites.copy()
    dead[0] = -1.0
    dead[1] = -1.0
    got, *_, gc, _ = _run_dp(S, H, W, K, dead, tg, stats, 0.5, 0.5, 3)
    assert gc == [0, 0, 0, 0, 0, 0]


def test_encoder_budget_schedule(S):
    from paper_2604_21984_amd import encode as E
    H, W = 96, 128
    tg = torch.from_numpy(synth.image_encode(4, H, W, n_polygons=25, patch=16)).to(DEV)
    sched = E.BudgetSchedule(densify_every=10, densify_start=10, densify_end=60, p_split=0.1,
                             prune_every=20, prune_start=20, prune_end=60, p_prune=0.05)
    enc = E.Encoder(tg, 300, E.EncodeConfig(K=8, n_inject=4, seed=1, budget=sched), cap=900)
    p0 = enc.psnr()
    for _ in range(80):
        enc.step()
    torch.cuda.synchronize()
    hist = enc.budget_log
    assert [h["iteration"] for h in hist] == [10, 20, 30, 40, 50, 60]
    n = 300
    for h in hist:
        c = h["counts"]
        assert c[0] == n
        assert c[1] == (int(0.05 * n) if h["prune"] else 0)
        n = c[3]
    sites = enc.sites.cpu().numpy()
    active = sites[0] >= 0
    assert active.sum() == n and n > 300
    assert enc.img.n_slots >= np.nonzero(active)[0].max() + 1
    lists = enc.topk.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    ids = lists[lists != 0xFFFFFFFF]
    assert active[ids].all()                             # lists hold active sites only
    assert enc.psnr() > p0 + 3.0


def test_densify_prune_large_image_scale(S):
    """2048x2048, N = 100 000 from the initialisation in a 400 000-slot buffer, K = 16:
    statistics within the float32 bound on the oracle's lists, then one prune + split
    + seed step against the oracle on the oracle's statistics."""
    import math
    H = W = 2048
    N, cap, K = 100_000, 400_000, 16
    tg = synth.image_large(1, H, W)
    s = O.default_scale(H, W)
    lt0 = float(np.clip(math.log(2 * max(H, W) / math.sqrt(H * W / N)), 2, 20))
    sites, n = O.init_sites(tg, N, 0.3, 5, lt0, 1.0, cap)
    lists = O.seed_lists(H, W, K, s, sites, N)
    lists = O.prop_pass(H, W, K, s, sites, N, lists, O.jump(0, H, W), 4, 3, 0)
    ref, sabs, sens = O.site_stats(H, W, K, s, sites, N, lists, tg, scales=True)
    got = _gpu_stats(S, H, W, K, N, cap, sites, lists, tg)
    floor = 1e-7 * np.abs(ref).max(axis=1, keepdims=True)
    tol = 1e-4 * np.abs(ref) + 2e-5 * sabs + 1e-5 * sens + floor
    assert not (np.abs(got - ref) > tol).any()
    stats = ref.astype(np.float32)
    rs = sites.copy()
    am = np.full((10, cap), 3.0, np.float32)
    av = np.full((10, cap), 5.0, np.float32)
    rl = lists.copy()
    rc = O.densify_prune(tg, rs, stats, 0.033, 0.01, 7, K=K, adam_m=am, adam_v=av, lists=rl)
    gs, gm, gv, gc, gl = _run_dp(S, H, W, K, sites, tg, stats, 0.033, 0.01, 7, lists=lists)
    assert gc == rc and rc[1] == 3300 and rc[2] == 1000
    _compare_sites(gs, rs)
    np.testing.assert_array_equal(gm, am)
    np.testing.assert_array_equal(gv, av)
    np.testing.assert_array_equal(gl, rl)


def test_fixed_stats_small_negative_sum_keeps_sign(S):
    """A cross-moment sum of a few units below zero, formed from two large terms in two
    tiles: one site at (16, 1) owns every pixel of a 3 x 18 image (two 16 x 16 tiles);
    the residual is zero except at (x, y) = (15, 0), d_x d_y = +1, e = 2^-8, and at
    (17, 0), d_x d_y = -1, e = 2^-8 + 2^-28.  S_xy = e_A - e_B = -2^-28 = -4 units of
    2^-30 exactly; the 128-bit sum over tiles must give it with its sign (a low word
    read as unsigned would cancel it against 2^64)."""
    H, W, K, N = 3, 18, 4, 1
    sites = np.zeros((10, N), np.float32)
    sites[:, 0] = [16.0, 1.0, 3.0, 1.0, 0.5, 0.5, 0.5, 1.0, 0.0, 0.0]
    lists = np.full((H * W, K), 0xFFFFFFFF, np.uint32)
    lists[:, 0] = 0
    tg = np.full((3, H, W), 0.5, np.float32)
    tg[0, 0, 15] = 0.5 + 2.0 ** -4
    tg[0, 0, 17] = 0.5 + 2.0 ** -4
    tg[1, 0, 17] = 0.5 + 2.0 ** -14
    s = O.default_scale(H, W)
    ref = O.site_stats(H, W, K, s, sites, N, lists, tg)
    assert ref[5, 0] == -(2.0 ** -28)
    img = S.image(H, W, K, N, N)
    rec = torch.empty(16, dtype=torch.float32, device=DEV)
    S.prepare_sites(img, torch.from_numpy(sites).to(DEV), rec)
    topk = torch.from_numpy(rows_to_planar(lists, H, W, K)).to(DEV)
    acc = torch.empty(2 * S.NSTAT * N, dtype=torch.int64, device=DEV)
    stats = torch.empty((S.NSTAT, N), dtype=torch.float32, device=DEV)
    S.site_stats_fixed(img, rec, topk, torch.from_numpy(tg).to(DEV), acc, stats)
    torch.cuda.synchronize()
    got = stats.cpu().numpy()
    assert got[5, 0] == np.float32(-(2.0 ** -28)), got[5, 0]
    a = acc.cpu().numpy().reshape(2, S.NSTAT, N)
    assert a[0, 5, 0] == -4 and a[1, 5, 0] == -1     # low word -4, high word the sign
    assert got[1, 0] == np.float32(2.0 ** -7 + 2.0 ** -28)   # energy: e_A + e_B
