"""Pins of the oracle's propagation pass (Sec. 4.3), jump schedule and injection RNG."""
import math
import os

import numpy as np
import pytest

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_splitmix64_published_vectors():
    for seed, k, val in _golden("splitmix64.txt"):
        assert O.splitmix64(int(seed), int(k)) == int(val, 0)


def test_jump_schedule_matches_paper_statement():
    for row in _golden("jump_schedule.txt"):
        H, W = int(row[0]), int(row[1])
        want = [int(v) for v in row[2:]]
        assert [O.jump(t, H, W) for t in range(len(want))] == want


def test_jump_schedule_context_of_convergence_table():
    """Tab. vpt_convergence at 1024^2: 8 passes end at step 4, the step reaches 1 at
    the 10th pass, consistent with the jump in exact-match between 8 and 12 passes."""
    assert O.jump(7, 1024, 1024) == 4
    assert O.jump(9, 1024, 1024) == 1
    assert O.jump(9, 2048, 2048) == 2 and O.jump(10, 2048, 2048) == 1


def test_injection_ids_golden():
    """The counter mapping of the injection draws (which output of the stream, its high
    word, the multiply-shift to a slot) against IDs derived from the published
    SplitMix64 outputs."""
    rows = _golden("inject_ids.txt")
    assert len(rows) >= 10
    for seed, t, P, p, J, j, n, want in rows:
        got = O.inject_id(int(seed), int(t), int(P), int(p), int(J), int(j), int(n))
        assert got == int(want), (seed, t, P, p, J, j, n, got, want)


def test_injection_ids_in_range_and_uniform():
    n = 37
    ids = np.array([O.inject_id(99, t, 1000, p, 4, j, n)
                    for t in range(3) for p in range(400) for j in range(4)])
    assert ids.min() >= 0 and ids.max() < n
    counts = np.bincount(ids, minlength=n)
    exp = len(ids) / n
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 36 + 6 * math.sqrt(2 * 36)       # df = 36, ~6 sigma


def _key(sites, s, p, W, i):
    return (-O.score(sites, int(i), s, float(p % W), float(p // W)), int(i))


def _check_lists(sites, n, s, H, W, K, lists):
    for p in range(H * W):
        row = [int(i) for i in lists[p]]
        valid = [i for i in row if i != O.INVALID]
        assert row[len(valid):] == [O.INVALID] * (K - len(valid))   # sentinel tail
        assert len(set(valid)) == len(valid)                        # unique
        for i in valid:
            assert i < n and sites[0, i] >= 0                       # valid, active
        keys = [_key(sites, s, p, W, i) for i in valid]
        assert keys == sorted(keys)                                 # sorted


def _slot_scores(sites, s, H, W, K, lists):
    out = np.full((H * W, K), -np.inf)
    for p in range(H * W):
        for k, i in enumerate(lists[p]):
            if i != O.INVALID:
                out[p, k] = O.score(sites, int(i), s, float(p % W), float(p // W))
    return out


def test_pass_invariants_monotone_and_bounded_by_brute_force():
    H, W, K, N, J = 32, 32, 4, 96, 2
    sites = synth.random_sites(17, H, W, N, cap=100, anisotropic=True,
                               log_tau_range=(0, 3), r_range=(0, 2))
    sites[0, 5] = -1.0
    for dup in (3, 50, 71):                      # exact ties, broken by the lower ID
        sites[:, dup] = sites[:, 10]
    s = 0.125
    lists = O.seed_lists(H, W, K, s, sites, N)
    brute = O.brute_topk(H, W, K, s, sites, N)
    bs = _slot_scores(sites, s, H, W, K, brute)
    prev = _slot_scores(sites, s, H, W, K, lists)
    for t in range(8):
        lists = O.prop_pass(H, W, K, s, sites, N, lists, O.jump(t, H, W), J, 7, t)
        _check_lists(sites, N, s, H, W, K, lists)
        cur = _slot_scores(sites, s, H, W, K, lists)
        assert np.all(cur >= prev)            # C_{t-1} is a subset of the candidate set
        assert np.all(cur <= bs)              # never better than the exact top-K
        prev = cur


def test_converges_to_brute_force_when_k_covers_all_sites():
    H, W, K, N = 16, 16, 8, 6
    sites = synth.random_sites(3, H, W, N, anisotropic=True, r_range=(0, 2))
    s = O.default_scale(H, W)
    lists = O.seed_lists(H, W, K, s, sites, N)
    brute = O.brute_topk(H, W, K, s, sites, N)
    for t in range(40):
        new = O.prop_pass(H, W, K, s, sites, N, lists, O.jump(t, H, W), 0, 0, t)
        if np.array_equal(new, lists) and O.jump(t, H, W) == 1:
            break
        lists = new
    assert np.array_equal(lists, brute)


def test_single_site_spreads_by_cross_dilation():
    """J = 0, one site: after pass t the pixels holding it are exactly
    S_t = S_{t-1} + {0, (+-s_t, 0), (0, +-s_t)} clipped to the image."""
    H, W, K = 13, 21, 4
    sites = synth.random_sites(0, H, W, 1)
    sites[0, 0], sites[1, 0] = 6.2, 4.7
    s = O.default_scale(H, W)
    lists = O.seed_lists(H, W, K, s, sites, 1)
    S = np.zeros((H, W), bool)
    S[5, 6] = True
    for t in range(9):
        st = O.jump(t, H, W)
        lists = O.prop_pass(H, W, K, s, sites, 1, lists, st, 0, 0, t)
        nS = S.copy()
        nS[:, st:] |= S[:, :-st]
        nS[:, :-st] |= S[:, st:]
        nS[st:, :] |= S[:-st, :]
        nS[:-st, :] |= S[st:, :]
        S = nS
        assert np.array_equal((lists[:, 0] == 0).reshape(H, W), S)


def test_subset_of_pixels_equals_full_pass():
    H, W, K, N = 20, 24, 8, 60
    sites = synth.random_sites(23, H, W, N, anisotropic=True)
    s = O.default_scale(H, W)
    lists = O.seed_lists(H, W, K, s, sites, N)
    full = O.prop_pass(H, W, K, s, sites, N, lists, 8, 4, 5, 3)
    pix = np.array([0, 7, 100, H * W - 1], np.int64)
    part = O.prop_pass(H, W, K, s, sites, N, lists, 8, 4, 5, 3, pix=pix)
    assert np.array_equal(part, full[pix])
