"""Pins of the oracle's full-refresh regime (App. B.3): the evaluation grid of a list
field (downscaled candidate grid, or a new output grid), the seed pass on a grid, the
JFA flood prepass and the refresh built from them.

Each pin is an independent fact: closed forms of the grid points, coverage of a single
site by the flood passes, exact lists when at most four sites exist, brute force at the
cell points computed here from the pinned score, and reductions to already pinned
oracle functions on the image's own grid."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
INV = 0xFFFFFFFF


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return rows


def _brute_at(sites, n, s, xy, K):
    """Exact top K at arbitrary points from the pinned float32 score: (score desc, ID
    asc) over active sites, padded with the sentinel."""
    d = O.site_derived(sites, n, s)
    act = [i for i in range(n) if d[i, 0] == 1.0]
    out = np.full((len(xy), K), INV, np.uint32)
    for m, (x, y) in enumerate(xy):
        sc = [(-O.score(sites, i, s, float(x), float(y)), i) for i in act]
        sc.sort()
        for k, (_, i) in enumerate(sc[:K]):
            out[m, k] = i
    return out


# ---- grid points ----------------------------------------------------------------------

def test_grid_points_image_grid_are_pixels():
    xy, cell = O.grid_points(7, 11, 7, 11)
    jj, ii = np.meshgrid(np.arange(11), np.arange(7))
    assert np.array_equal(xy[:, 0], jj.ravel().astype(np.float32))
    assert np.array_equal(xy[:, 1], ii.ravel().astype(np.float32))
    assert np.array_equal(cell, np.arange(77))


@pytest.mark.parametrize("s", [2, 3, 4, 8])
def test_grid_points_downscaled_are_cell_centres(s):
    """W = s Wg: cell c covers pixels c s .. c s + s - 1, its point is their mean
    c s + (s - 1)/2, and pixel j maps to floor(j / s)."""
    Hg, Wg = 5, 6
    H, W = s * Hg, s * Wg
    xy, cell = O.grid_points(H, W, Hg, Wg)
    for i in range(Hg):
        for j in range(Wg):
            assert xy[i * Wg + j, 0] == j * s + (s - 1) / 2
            assert xy[i * Wg + j, 1] == i * s + (s - 1) / 2
    for p in range(H * W):
        i, j = divmod(p, W)
        assert cell[p] == (i // s) * Wg + (j // s)


def test_grid_points_finer_grid():
    """A grid twice as fine: point j' at (2 j' - 1) / 4 (UV centres of half pixels)."""
    xy, _ = O.grid_points(3, 5, 6, 10)
    for j in range(10):
        assert xy[j, 0] == (2 * j - 1) / 4


def test_grid_cells_hold_pixel_centres_ragged():
    """Ragged grid (W not a multiple of the cell size): every pixel's centre lies in the
    UV interval of its cell, checked in exact rational arithmetic."""
    H, W, Hg, Wg = 13, 29, 4, 7
    xy, cell = O.grid_points(H, W, Hg, Wg)
    for p in range(H * W):
        i, j = divmod(p, W)
        ci, cj = divmod(int(cell[p]), Wg)
        u = Fraction(2 * j + 1, 2 * W)
        v = Fraction(2 * i + 1, 2 * H)
        assert Fraction(cj, Wg) <= u < Fraction(cj + 1, Wg)
        assert Fraction(ci, Hg) <= v < Fraction(ci + 1, Hg)
    # and each cell point is the centre of its UV square, to float rounding
    for c in range(Hg * Wg):
        ci, cj = divmod(c, Wg)
        x = (cj + 0.5) / Wg * W - 0.5
        y = (ci + 0.5) / Hg * H - 0.5
        assert abs(xy[c, 0] - x) <= 1e-6 * max(1, abs(x))
        assert abs(xy[c, 1] - y) <= 1e-6 * max(1, abs(y))


# ---- seed pass on a grid --------------------------------------------------------------

def test_seed_grid_on_image_grid_equals_seed_pass():
    H, W, K, N = 23, 31, 8, 900
    s = O.default_scale(H, W)
    sites = synth.random_sites(5, H, W, N, anisotropic=True, log_tau_range=(2, 5),
                               r_range=(1, 3))
    sites[0, 7] = -1.0
    assert np.array_equal(O.seed_grid(H, W, H, W, K, K, s, sites, N),
                          O.seed_lists(H, W, K, s, sites, N))


@pytest.mark.parametrize("n_entries", [4, 8])
def test_seed_grid_by_brute_force(n_entries):
    """Each cell keeps the best n_entries of the sites whose nearest pixel falls in it,
    scored at the cell point; entries beyond n_entries stay empty."""
    H, W, Hg, Wg, K, N = 20, 26, 5, 9, 8, 400
    s = O.default_scale(H, W)
    sites = synth.random_sites(6, H, W, N, anisotropic=True, log_tau_range=(2, 5),
                               r_range=(1, 3))
    sites[0, 3] = -1.0
    got = O.seed_grid(H, W, Hg, Wg, K, n_entries, s, sites, N)
    xy, cell = O.grid_points(H, W, Hg, Wg)
    d = O.site_derived(sites, N, s)
    buckets = {}
    for i in range(N):
        if d[i, 0] != 1.0:
            continue
        pi = min(max(int(np.rint(sites[1, i])), 0), H - 1)
        pj = min(max(int(np.rint(sites[0, i])), 0), W - 1)
        buckets.setdefault(int(cell[pi * W + pj]), []).append(i)
    for c in range(Hg * Wg):
        ids = buckets.get(c, [])
        x, y = xy[c]
        order = sorted(ids, key=lambda i: (-O.score(sites, i, s, float(x), float(y)), i))
        want = order[:n_entries] + [INV] * (K - len(order[:n_entries]))
        assert list(got[c]) == want, c


# ---- JFA flood prepass ------------------------------------------------------------------

def test_jfa_steps_golden():
    for row in _golden("jfa_steps.txt"):
        assert O.jfa_steps(row[0], row[1]) == row[2:], row


@pytest.mark.parametrize("shape", [(1, 1), (5, 5), (9, 4), (16, 16), (17, 33), (40, 7)])
@pytest.mark.parametrize("corner", [0, 1])
def test_jfa_single_site_floods_every_cell(shape, corner):
    """One site seeded in a corner cell reaches every cell: the steps 2^(L-1)..1 in all
    eight directions (and staying) compose every offset up to 2^L - 1 on each axis.  A
    flood without the diagonal neighbours could not reach the far corner."""
    Hg, Wg = shape
    H, W = 2 * Hg, 3 * Wg
    sites = synth.random_sites(7, H, W, 1, anisotropic=True, log_tau_range=(2, 3))
    sites[0, 0] = 0.0 if corner == 0 else W - 1.0
    sites[1, 0] = 0.0 if corner == 0 else H - 1.0
    s = O.default_scale(H, W)
    lists = O.jfa_prepass(H, W, Hg, Wg, 8, s, sites, 1)
    assert (lists[:, 0] == 0).all()
    assert (lists[:, 1:] == INV).all()


def test_jfa_exact_with_at_most_four_sites():
    """With four active sites every ID fits every first texture, so each floods the
    whole grid and the prepass ends with the exact lists; entries 4.. stay empty."""
    H, W, Hg, Wg, K = 30, 45, 10, 15, 8
    s = O.default_scale(H, W)
    sites = synth.random_sites(8, H, W, 6, anisotropic=True, log_tau_range=(2, 5),
                               r_range=(1, 4))
    sites[0:2, 2] = -1.0       # inactive
    sites[3, 4] = np.nan       # non-finite: inactive
    lists = O.jfa_prepass(H, W, Hg, Wg, K, s, sites, 6)
    xy, _ = O.grid_points(H, W, Hg, Wg)
    want = _brute_at(sites, 6, s, xy, 4)
    assert np.array_equal(lists[:, :4], want)
    assert (lists[:, 4:] == INV).all()


def test_jfa_flood_monotone_and_below_exact():
    """Per cell, the score of each of the four entries never falls from pass to pass
    (the cell's own first texture is a candidate), and never exceeds the exact k-th
    score at the cell point."""
    H, W, K, N = 40, 52, 8, 300
    s = O.default_scale(H, W)
    sites = synth.random_sites(9, H, W, N, anisotropic=True, log_tau_range=(2, 5),
                               r_range=(1, 3))
    xy, _ = O.grid_points(H, W, H, W)

    def scores(lists):
        sc = np.full((H * W, 4), -np.inf)
        for p in range(H * W):
            for k in range(4):
                i = int(lists[p, k])
                if i != INV:
                    sc[p, k] = O.score(sites, i, s, float(xy[p, 0]), float(xy[p, 1]))
        return sc

    cur = O.seed_grid(H, W, H, W, K, 4, s, sites, N)
    prev = scores(cur)
    for step in O.jfa_steps(H, W):
        cur = O.jfa_flood(H, W, H, W, K, s, sites, N, cur, step)
        sc = scores(cur)
        assert (sc >= prev).all()
        prev = sc
    exact = O.brute_topk(H, W, 4, s, sites, N)
    ex = scores(exact)
    assert (prev <= ex).all()
    # JFA finds the owner (entry 0) almost everywhere
    assert (cur[:, 0] == exact[:, 0]).mean() > 0.95


def test_jfa_owner_quality_voronoi():
    """Isotropic equal-temperature sites: entry 0 after the prepass is the Voronoi owner
    (k-d tree nearest centre) at nearly every pixel, as jump flooding is known to be."""
    cKDTree = pytest.importorskip("scipy.spatial").cKDTree
    H = W = 128
    N = 400
    sites = synth.cell_sites(10, H, W, N, log_tau=3.0, r=1.0)
    s = O.default_scale(H, W)
    lists = O.jfa_prepass(H, W, H, W, 4, s, sites, N)
    jj, ii = np.meshgrid(np.arange(W), np.arange(H))
    pts = np.stack([jj.ravel(), ii.ravel()], 1).astype(np.float64)
    d, nn = cKDTree(np.stack([sites[0, :N], sites[1, :N]], 1).astype(np.float64)).query(pts, k=2)
    clear = (d[:, 1] - d[:, 0]) > 1e-3
    match = (lists[:, 0].astype(np.int64) == nn[:, 0])[clear].mean()
    assert match > 0.99, match


# ---- propagation and refresh on a grid -----------------------------------------------

def test_prop_grid_on_image_grid_equals_prop_pass():
    H, W, K, N, J = 25, 19, 8, 500, 4
    s = O.default_scale(H, W)
    sites = synth.random_sites(11, H, W, N, anisotropic=True, log_tau_range=(2, 5),
                               r_range=(1, 3))
    lists = O.seed_lists(H, W, K, s, sites, N)
    for t in range(4):
        a = O.prop_pass_grid(H, W, H, W, K, s, sites, N, lists, O.jump(t, H, W), J, 3, t)
        b = O.prop_pass(H, W, K, s, sites, N, lists, O.jump(t, H, W), J, 3, t)
        assert np.array_equal(a, b)
        lists = a


@pytest.mark.parametrize("jfa", [False, True])
def test_refresh_on_downscaled_grid_converges_to_exact(jfa):
    """K >= active sites on a 4x downscaled grid: after enough passes every cell holds
    the exact ranking of all active sites at its point (brute force here)."""
    H, W, Hg, Wg, K, N = 32, 48, 8, 12, 8, 7
    s = O.default_scale(H, W)
    sites = synth.random_sites(12, H, W, N, anisotropic=True, log_tau_range=(2, 5),
                               r_range=(1, 4))
    sites[0:2, 5] = -1.0
    lists = O.refresh(H, W, Hg, Wg, K, s, sites, N, jfa, 12, 2, 4)
    xy, _ = O.grid_points(H, W, Hg, Wg)
    assert np.array_equal(lists, _brute_at(sites, N, s, xy, K))


def test_refresh_zero_passes_is_its_first_step():
    H, W, Hg, Wg, K, N = 24, 30, 12, 15, 8, 200
    s = O.default_scale(H, W)
    sites = synth.random_sites(13, H, W, N, anisotropic=True, log_tau_range=(2, 5))
    assert np.array_equal(O.refresh(H, W, Hg, Wg, K, s, sites, N, False, 0, 4, 1),
                          O.seed_grid(H, W, Hg, Wg, K, K, s, sites, N))
    assert np.array_equal(O.refresh(H, W, Hg, Wg, K, s, sites, N, True, 0, 4, 1),
                          O.jfa_prepass(H, W, Hg, Wg, K, s, sites, N))
    # one pass = the propagation pass of the grid at t = 0 from that start
    pre = O.jfa_prepass(H, W, Hg, Wg, K, s, sites, N)
    one = O.prop_pass_grid(H, W, Hg, Wg, K, s, sites, N, pre, O.jump(0, Hg, Wg), 4, 1, 0)
    assert np.array_equal(O.refresh(H, W, Hg, Wg, K, s, sites, N, True, 1, 4, 1), one)


def test_blend_points_on_image_grid_equals_render():
    H, W, K, N = 17, 21, 8, 150
    s = O.default_scale(H, W)
    sites = synth.random_sites(14, H, W, N, anisotropic=True, log_tau_range=(2, 5),
                               r_range=(1, 3))
    lists = O.brute_topk(H, W, K, s, sites, N)
    xy, _ = O.grid_points(H, W, H, W)
    got = O.blend_points(K, s, sites, N, lists, xy)
    ref = O.render(H, W, K, s, sites, N, lists)
    assert np.array_equal(got.T.reshape(3, H, W), ref)


def test_expand_grid_lists_maps_each_pixel_to_its_cell():
    H, W, Hg, Wg = 10, 14, 5, 7
    lists = np.arange(Hg * Wg * 4, dtype=np.uint32).reshape(Hg * Wg, 4)
    ex = O.expand_grid_lists(H, W, Hg, Wg, lists)
    for p in range(H * W):
        i, j = divmod(p, W)
        assert np.array_equal(ex[p], lists[(i // 2) * Wg + j // 2])
