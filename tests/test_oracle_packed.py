"""Pins of the oracle's packed 16-byte inference record (App. B.2 "Packed storage for
evaluation"; Sec. 6.1 bits-per-pixel accounting): the float16 conversion against numpy,
record words derived by hand for edge values, the quantisation parameters, round-trip
error bounds, and the BPP formula."""
import math

import numpy as np

import oracle as O
import synth


def test_f16_conversion_matches_numpy():
    # every half pattern decodes as numpy decodes it, and re-encodes to itself
    h = np.arange(65536, dtype=np.uint32)
    ref = h.astype(np.uint16).view(np.float16).astype(np.float32)
    for v in h[::7].tolist() + list(range(0, 1100)) + list(range(0x7B00, 0x7C01)):
        f = O.f16_to_f32(v)
        r = float(ref[v])
        assert (math.isnan(f) and math.isnan(r)) or f == r, v
        if not math.isnan(r):
            assert O.f32_to_f16(f) == v or (v == 0x8000 and O.f32_to_f16(f) == 0x8000), v
    # random floats over the whole range, ties included, round as numpy rounds
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.normal(0, 1, 3000), rng.normal(0, 1e4, 1000),
                         rng.uniform(-7e-5, 7e-5, 2000), 2.0 ** rng.uniform(-30, 17, 2000)])
    ties = (np.arange(1, 2000, dtype=np.float32) + np.float32(0.5)) * np.float32(2.0 ** -10)
    for x in np.concatenate([xs.astype(np.float32), ties]):
        want = int(np.float32(x).astype(np.float16).view(np.uint16))
        assert O.f32_to_f16(float(x)) == want, x


def _edge_sites():
    H, W = 101, 201
    s = np.zeros((10, 4), np.float32)
    # slot 0: every value at its minimum, u = (1, 0), a = 0
    s[:, 0] = [0, 0, 2.0, 1.0, 0, 0, 0, 1, 0, 0]
    # slot 1: every value at its maximum, u = (-1, 0), a = 1
    s[:, 1] = [W - 1, H - 1, 6.0, 5.0, 1, 1, 1, -1, 0, 1.0]
    # slot 2: every value half way, u = (0, 1), a = -2
    s[:, 2] = [100, 50, 4.0, 3.0, 0.5, 0.5, 0.5, 0, 1, -2.0]
    # slot 3: inactive
    s[:, 3] = [-1, -1, 3.0, 2.0, 0.2, 0.2, 0.2, 1, 0, 0]
    return H, W, s


def test_pack_words_by_hand():
    """Words derived by hand from the layout: 15-bit x | 15-bit y << 15 | active << 31;
    11/11/10-bit colour; 16-bit log tau | 16-bit r << 16; 16-bit angle code over
    [-pi, pi] | float16(a) << 16.  Half-way values round to even codes (16383.5 ->
    16384, 32767.5 -> 32768, 1023.5 -> 1024, 511.5 -> 512); u = (1, 0) has angle 0,
    code rint(65535 / 2) = 32768; u = (-1, 0) angle pi, code 65535; u = (0, 1) angle
    pi/2, code rint(0.75 * 65535) = 49151."""
    H, W, s = _edge_sites()
    packed, q = O.pack_sites(H, W, s, 4)
    assert list(q) == [2.0, 4.0, 1.0, 4.0, 0.0, 1.0, 0.0, 1.0, 0.0, 1.0]
    want = [
        [0x80000000, 0, 0, 32768],
        [32767 | (32767 << 15) | 0x80000000, 2047 | (2047 << 11) | (1023 << 22),
         65535 | (65535 << 16), 65535 | (0x3C00 << 16)],
        [16384 | (16384 << 15) | 0x80000000, 1024 | (1024 << 11) | (512 << 22),
         32768 | (32768 << 16), 49151 | (0xC000 << 16)],
        [0, 0, 0, 0],
    ]
    assert packed.tolist() == want


def test_qparams_over_active_sites_only():
    H, W = 40, 60
    s = synth.random_sites(1, H, W, 50, log_tau_range=(2, 9), r_range=(1, 30))
    s[2, 7] = 50.0                # an inactive site's extreme values are ignored
    s[0, 7] = -1.0
    s[3, 8] = np.nan              # non-finite: inactive
    q = O.pack_qparams(s, 50)
    act = np.ones(50, bool)
    act[[7, 8]] = False
    for k, p in enumerate([2, 3, 4, 5, 6]):
        mn, mx = s[p, act].min(), s[p, act].max()
        assert q[2 * k] == mn and q[2 * k + 1] == np.float32(mx - mn)
    assert (O.pack_qparams(s[:, :0].copy(), 0) == 0).all()


def test_round_trip_error_bounds():
    H, W, N = 512, 768, 5000
    s = synth.random_sites(2, H, W, N, anisotropic=True, log_tau_range=(2, 12),
                           r_range=(1, 40))
    s[0:2, 17] = -1.0
    packed, q = O.pack_sites(H, W, s, N)
    u = O.unpack_sites(H, W, packed, q)
    act = s[0] >= 0
    assert (u[0:2, ~act] == -1).all()
    for p, span, bits in ((0, W - 1, 15), (1, H - 1, 15), (2, q[1], 16), (3, q[3], 16),
                          (4, q[5], 11), (5, q[7], 11), (6, q[9], 10)):
        err = np.abs(u[p, act].astype(np.float64) - s[p, act])
        bound = 0.5 * span / (2 ** bits - 1) + 4e-7 * max(1.0, span + abs(s[p, act]).max())
        assert err.max() <= bound, (p, err.max(), bound)
    # direction: angle error at most half a code step (pi / 65535), unit length
    th = np.arctan2(s[8, act], s[7, act])
    tu = np.arctan2(u[8, act], u[7, act])
    d = np.abs(np.angle(np.exp(1j * (tu - th))))
    assert d.max() <= math.pi / 65535 + 1e-6
    assert np.abs(np.hypot(u[7, act], u[8, act]) - 1).max() < 1e-6
    # a: exactly its float16 value
    assert np.array_equal(u[9, act], s[9, act].astype(np.float16).astype(np.float32))


def test_repack_is_stable():
    """Re-packing the decoded sites with the same parameters reproduces the codes (up to
    one step where a decoded value lands on a rounding boundary)."""
    H, W, N = 300, 400, 3000
    s = synth.random_sites(3, H, W, N, anisotropic=True, log_tau_range=(2, 8),
                           r_range=(1, 10))
    packed, q = O.pack_sites(H, W, s, N)
    again, _ = O.pack_sites(H, W, O.unpack_sites(H, W, packed, q), N, q)
    assert (again == packed).all(axis=1).mean() >= 0.999
    fields = [(0, 0, 15), (0, 15, 15), (1, 0, 11), (1, 11, 11), (1, 22, 10), (2, 0, 16),
              (2, 16, 16), (3, 0, 16)]
    for w, sh, b in fields:
        a = (packed[:, w] >> sh) & ((1 << b) - 1)
        c = (again[:, w] >> sh) & ((1 << b) - 1)
        assert np.abs(a.astype(np.int64) - c).max() <= 1


def test_bpp_formula():
    assert O.bpp(20000, 512, 768) == 20000 * 128 / (512 * 768)
    assert O.bpp(32768, 2048, 2048) == 1.0


def test_packed_render_close_to_float_render():
    """Rendering the decoded sites with the same lists changes colours by about the
    quantisation step (the paper reports no PSNR change from the packed records)."""
    H, W, K, N = 128, 160, 8, 1200
    s = synth.random_sites(4, H, W, N, anisotropic=True, log_tau_range=(3, 5),
                           r_range=(1, 3))
    sc = O.default_scale(H, W)
    lists = O.brute_topk(H, W, K, sc, s, N)
    a = O.render(H, W, K, sc, s, N, lists)
    packed, q = O.pack_sites(H, W, s, N)
    b = O.render(H, W, K, sc, O.unpack_sites(H, W, packed, q), N, lists)
    mse = np.mean((a - b) ** 2)
    assert 10 * np.log10(1.0 / max(mse, 1e-30)) > 50
