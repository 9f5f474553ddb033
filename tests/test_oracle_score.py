"""Pins of the oracle's per-site metric and score (Sec. 4.1-4.2) against closed forms
computed independently here in float64 numpy."""
import math

import numpy as np
import pytest

import oracle as O
import synth


def _rot_score(site, s, X, Y):
    """Independent float64 form: q = d^T R^T diag(e^a, e^-a) R d with R the rotation
    taking the unit direction u to (1, 0)."""
    x, y, lt, r, _, _, _, ux, uy, a = [float(v) for v in site]
    nu = math.hypot(ux, uy)
    th = math.atan2(uy, ux)
    c, sn = math.cos(th), math.sin(th)
    dx, dy = X - x, Y - y
    p = c * dx + sn * dy          # along u
    q = -sn * dx + c * dy         # along the perpendicular
    quad = (math.exp(a) * p * p + math.exp(-a) * q * q) * nu * nu
    n = math.sqrt(quad)
    return math.exp(lt) * s * (r - n), n


def test_metric_eigen_structure():
    sites = synth.random_sites(3, 40, 50, 64, anisotropic=True)
    d = O.site_derived(sites, 64, 1.0 / 50)
    for i in range(64):
        valid, tau, ep, em, kap, g11, g12, g22 = d[i]
        assert valid == 1.0
        G = np.array([[g11, g12], [g12, g22]], np.float64)
        a = float(sites[9, i])
        u = sites[7:9, i].astype(np.float64)
        w, V = np.linalg.eigh(G)
        np.testing.assert_allclose(sorted(w), sorted([math.exp(a), math.exp(-a)]), rtol=2e-6)
        assert abs(np.linalg.det(G) - 1.0) < 5e-6               # det G = 1 (Sec. 4.1)
        top = V[:, np.argmax(w)] if a > 1e-3 else V[:, np.argmin(w)]
        if abs(a) > 1e-3:
            assert abs(abs(top @ u) - 1.0) < 1e-5               # e^a along u
        assert tau == np.float32(math.exp(float(sites[2, i])))
        assert ep == np.float32(math.exp(a)) and em == np.float32(math.exp(-a))
        assert kap == np.float32(tau * np.float32(1.0 / 50))


def test_score_matches_rotated_closed_form():
    rng = np.random.default_rng(0)
    sites = synth.random_sites(5, 30, 40, 32, anisotropic=True, log_tau_range=(0, 6),
                               r_range=(0, 5))
    s = O.default_scale(30, 40)
    for _ in range(400):
        i = int(rng.integers(0, 32))
        X, Y = float(rng.integers(0, 40)), float(rng.integers(0, 30))
        ref, n = _rot_score(sites[:, i], s, X, Y)
        got32 = O.score(sites, i, s, X, Y)
        got64 = O.score_f64(sites, i, s, X, Y)
        scale = abs(math.exp(float(sites[2, i])) * s) * (abs(float(sites[3, i])) + n + 1)
        assert abs(got64 - ref) <= 1e-12 * scale
        assert abs(got32 - ref) <= 2e-6 * scale


def test_isotropic_is_euclidean_apollonius():
    sites = synth.random_sites(6, 20, 20, 16, log_tau=1.5, r=2.0)
    s = 0.125
    for i in range(16):
        for (X, Y) in [(0.0, 0.0), (7.0, 3.0), (19.0, 19.0)]:
            d = math.hypot(X - sites[0, i], Y - sites[1, i])
            ref = math.exp(1.5) * s * (2.0 - d)                 # Eq. apollonius_dist
            assert abs(O.score(sites, i, s, X, Y) - ref) <= 2e-6 * (abs(ref) + 1)


def test_score_signed_zero_and_inactive():
    sites = synth.random_sites(1, 8, 8, 4)
    sites[0, 0], sites[1, 0], sites[3, 0] = 3.0, 4.0, -0.0
    v = O.score(sites, 0, 0.125, 3.0, 4.0)      # kappa * (-0 - 0) would be -0
    assert v == 0.0 and math.copysign(1.0, v) == 1.0            # +0, never -0
    sites[0, 1] = -1.0                                          # inactive (App. B.2)
    sites[4, 2] = np.nan                                        # non-finite parameter
    assert O.score(sites, 1, 0.125, 0.0, 0.0) == -math.inf
    assert O.score(sites, 2, 0.125, 0.0, 0.0) == -math.inf
    d = O.site_derived(sites, 4, 0.125)
    assert list(d[:, 0]) == [1.0, 0.0, 0.0, 1.0]


@pytest.mark.parametrize("c", [2.0, 8.0, 0.25])
def test_scale_absorbed_into_temperature(c):
    """Sec. 4.1: a constant scale of the score can be absorbed into tau:
    (s * c, log_tau - log c) gives the same logit."""
    sites = synth.random_sites(9, 16, 16, 8, anisotropic=True, log_tau_range=(1, 4),
                               r_range=(0, 3))
    s2 = sites.copy()
    s2[2] -= math.log(c)
    for i in range(8):
        for X, Y in [(1.0, 2.0), (15.0, 0.0), (8.0, 8.0)]:
            a = O.score_f64(sites, i, 1 / 16, X, Y)
            b = O.score_f64(s2, i, c / 16, X, Y)
            assert abs(a - b) <= 1e-6 * (abs(a) + 1)   # log_tau is stored in float32


def test_small_config_reading_equivalence():
    """Isotropic metric scale 1/8 px^-1 with tau = 1 equals s = 1/64 with
    log_tau = ln 8 (the reading of the 64x64 workload)."""
    sites = synth.random_sites(2, 64, 64, 32)
    s2 = sites.copy()
    s2[2] = np.float32(math.log(8.0))
    for i in range(32):
        for X, Y in [(0.0, 0.0), (31.0, 17.0), (63.0, 63.0)]:
            a = O.score(sites, i, 0.125, X, Y)
            b = O.score(s2, i, 1.0 / 64, X, Y)
            assert abs(a - b) <= 1e-6 * max(1.0, abs(a))
