"""Seeded synthetic inputs shared by the CPU oracle's tests and the GPU path's tests.

This module holds no arithmetic of the method (no scores, blends or gradients): only
pictures and random site parameters, drawn with numpy's PCG64 from an explicit seed.
The shapes and value distributions stand in for the paper's workloads (photographs of
the Kodak / Image-GS / DIV2K sets, which are not available here):

* ``image_small``   64x64: linear colour ramp + 12 hard-edged ellipses / triangles.
* ``image_encode``  any size: multi-octave gradient noise + random polygons + a patch of
                    1-pixel line texture (the 768x512 encode workload).
* ``image_large``   any size: multi-octave noise + many anisotropic ellipses (2048^2).
* ``random_sites``  uniform centres, random colours, optional random anisotropy.

All images are float32 [3, H, W] in [0, 1].  Site arrays are float32 [10, cap] in the
order (x, y, log_tau, r, c_r, c_g, c_b, u_x, u_y, a); unused slots are inactive
(x = y = -1).
"""
import numpy as np

NPARAM = 10


def _rng(seed):
    return np.random.default_rng(np.random.PCG64(seed))


# ----------------------------------------------------------------------------------
# gradient noise (Perlin-style: random unit gradients on a lattice, quintic fade)
# ----------------------------------------------------------------------------------
def _gradient_noise(rng, H, W, period):
    gh = int(np.ceil(H / period)) + 2
    gw = int(np.ceil(W / period)) + 2
    ang = rng.uniform(0, 2 * np.pi, size=(gh, gw))
    gx, gy = np.cos(ang), np.sin(ang)
    y = (np.arange(H) + 0.5) / period
    x = (np.arange(W) + 0.5) / period
    y0 = np.floor(y).astype(np.int64)
    x0 = np.floor(x).astype(np.int64)
    fy = (y - y0)[:, None]
    fx = (x - x0)[None, :]

    def corner(dy, dx):
        g_x = gx[(y0 + dy)[:, None], (x0 + dx)[None, :]]
        g_y = gy[(y0 + dy)[:, None], (x0 + dx)[None, :]]
        return g_x * (fx - dx) + g_y * (fy - dy)

    def fade(t):
        return t * t * t * (t * (t * 6 - 15) + 10)

    u, v = fade(fx), fade(fy)
    n00, n01, n10, n11 = corner(0, 0), corner(0, 1), corner(1, 0), corner(1, 1)
    a = n00 + u * (n01 - n00)
    b = n10 + u * (n11 - n10)
    return a + v * (b - a)


def _octave_noise(rng, H, W, base_period, octaves):
    out = np.zeros((H, W))
    amp, per, tot = 1.0, float(base_period), 0.0
    for _ in range(octaves):
        out += amp * _gradient_noise(rng, H, W, max(per, 2.0))
        tot += amp
        amp *= 0.5
        per *= 0.5
    out /= tot
    lo, hi = out.min(), out.max()
    return (out - lo) / max(hi - lo, 1e-12)


def _noise_background(rng, H, W, base_period, octaves):
    return np.stack([_octave_noise(rng, H, W, base_period, octaves) for _ in range(3)])


# ----------------------------------------------------------------------------------
# shapes with hard edges (inside tests at pixel centres, no antialiasing)
# ----------------------------------------------------------------------------------
def _paint_ellipse(img, rng, cx, cy, a, b, theta, colour):
    _, H, W = img.shape
    R = max(a, b)
    i0, i1 = max(int(np.floor(cy - R)), 0), min(int(np.ceil(cy + R)) + 1, H)
    j0, j1 = max(int(np.floor(cx - R)), 0), min(int(np.ceil(cx + R)) + 1, W)
    if i0 >= i1 or j0 >= j1:
        return
    yy, xx = np.mgrid[i0:i1, j0:j1].astype(np.float64)
    dx, dy = xx - cx, yy - cy
    c, s = np.cos(theta), np.sin(theta)
    p = (c * dx + s * dy) / a
    q = (-s * dx + c * dy) / b
    m = p * p + q * q <= 1.0
    for ch in range(3):
        img[ch, i0:i1, j0:j1][m] = colour[ch]


def _paint_polygon(img, verts, colour):
    """Even-odd fill of a closed polygon, verts (n, 2) as (x, y)."""
    _, H, W = img.shape
    xs, ys = verts[:, 0], verts[:, 1]
    i0, i1 = max(int(np.floor(ys.min())), 0), min(int(np.ceil(ys.max())) + 1, H)
    j0, j1 = max(int(np.floor(xs.min())), 0), min(int(np.ceil(xs.max())) + 1, W)
    if i0 >= i1 or j0 >= j1:
        return
    yy, xx = np.mgrid[i0:i1, j0:j1].astype(np.float64)
    inside = np.zeros(yy.shape, bool)
    n = len(verts)
    for k in range(n):
        xa, ya = verts[k]
        xb, yb = verts[(k + 1) % n]
        cond = (ya > yy) != (yb > yy)
        with np.errstate(divide="ignore", invalid="ignore"):
            xint = xa + (yy - ya) * (xb - xa) / (yb - ya)
        inside ^= cond & (xx < xint)
    for ch in range(3):
        img[ch, i0:i1, j0:j1][inside] = colour[ch]


def image_small(seed, H=64, W=64, n_shapes=12):
    """64x64 test picture: linear ramp between two random colours along a random
    direction, then n_shapes ellipses (semi-axes U[2,16] px, random rotation) or
    triangles (vertices uniform in the image), each with p = 1/2."""
    rng = _rng(seed)
    c0, c1 = rng.uniform(0, 1, 3), rng.uniform(0, 1, 3)
    th = rng.uniform(0, 2 * np.pi)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    t = np.cos(th) * xx + np.sin(th) * yy
    t = (t - t.min()) / max(t.max() - t.min(), 1e-12)
    img = c0[:, None, None] * (1 - t)[None] + c1[:, None, None] * t[None]
    for _ in range(n_shapes):
        col = rng.uniform(0, 1, 3)
        if rng.uniform() < 0.5:
            cx, cy = rng.uniform(0, W - 1), rng.uniform(0, H - 1)
            a, b = rng.uniform(2, 16), rng.uniform(2, 16)
            _paint_ellipse(img, rng, cx, cy, a, b, rng.uniform(0, np.pi), col)
        else:
            v = np.stack([rng.uniform(0, W - 1, 3), rng.uniform(0, H - 1, 3)], axis=1)
            _paint_polygon(img, v, col)
    return np.clip(img, 0, 1).astype(np.float32)


def image_encode(seed, H=512, W=768, n_polygons=200, octaves=4, base_period=128,
                 patch=128):
    """Encode workload picture: multi-octave gradient noise per channel, n_polygons
    star-shaped polygons (3-8 vertices, radius 5-150 px scaled with the image), and one
    patch x patch square of 1-px lines (period 2-3 px, orientation 0/45/90 degrees,
    two colours)."""
    rng = _rng(seed)
    img = _noise_background(rng, H, W, base_period, octaves)
    scale = np.sqrt(H * W / (512 * 768))
    for _ in range(n_polygons):
        nv = int(rng.integers(3, 9))
        R = rng.uniform(5, 150) * scale
        cx, cy = rng.uniform(0, W - 1), rng.uniform(0, H - 1)
        ang = np.sort(rng.uniform(0, 2 * np.pi, nv))
        rad = R * rng.uniform(0.5, 1.0, nv)
        verts = np.stack([cx + rad * np.cos(ang), cy + rad * np.sin(ang)], axis=1)
        _paint_polygon(img, verts, rng.uniform(0, 1, 3))
    ps = min(patch, H, W)
    if ps >= 4:
        py0 = int(rng.integers(0, H - ps + 1))
        px0 = int(rng.integers(0, W - ps + 1))
        period = int(rng.integers(2, 4))
        orient = int(rng.integers(0, 3))
        ca, cb = rng.uniform(0, 1, 3), rng.uniform(0, 1, 3)
        yy, xx = np.mgrid[0:ps, 0:ps]
        coord = [xx, xx + yy, yy][orient]
        line = (coord % period) == 0
        for ch in range(3):
            blk = img[ch, py0:py0 + ps, px0:px0 + ps]
            blk[line] = ca[ch]
            blk[~line] = cb[ch]
    return np.clip(img, 0, 1).astype(np.float32)


def image_large(seed, H=2048, W=2048, n_ellipses=2000, octaves=6, base_period=256):
    """Large picture: 6-octave noise + n_ellipses ellipses with axis ratio log-uniform
    in [1, 20] and major semi-axis 2-200 px (scaled with the image)."""
    rng = _rng(seed)
    img = _noise_background(rng, H, W, base_period, octaves)
    scale = np.sqrt(H * W / (2048 * 2048))
    for _ in range(n_ellipses):
        a = rng.uniform(2, 200) * scale
        ratio = np.exp(rng.uniform(0, np.log(20)))
        b = max(a / ratio, 0.5)
        _paint_ellipse(img, rng, rng.uniform(0, W - 1), rng.uniform(0, H - 1), a, b,
                       rng.uniform(0, np.pi), rng.uniform(0, 1, 3))
    return np.clip(img, 0, 1).astype(np.float32)


def random_sites(seed, H, W, n, cap=None, log_tau=0.0, r=0.0, anisotropic=False,
                 log_tau_range=None, r_range=None, a_range=(-2.0, 2.0)):
    """n sites with centres uniform in [0, W-1] x [0, H-1] and colours uniform in
    [0,1]^3.  Isotropic by default (a = 0, u = (1, 0)); with anisotropic=True the
    direction is uniform on the circle and a uniform in a_range.  log_tau and r are
    constants unless a (lo, hi) range is given."""
    rng = _rng(seed)
    cap = n if cap is None else cap
    s = np.zeros((NPARAM, cap), np.float32)
    s[0, :] = -1.0
    s[1, :] = -1.0
    s[0, :n] = rng.uniform(0, W - 1, n)
    s[1, :n] = rng.uniform(0, H - 1, n)
    s[2, :n] = rng.uniform(*log_tau_range, n) if log_tau_range else log_tau
    s[3, :n] = rng.uniform(*r_range, n) if r_range else r
    s[4:7, :n] = rng.uniform(0, 1, (3, n))
    if anisotropic:
        th = rng.uniform(0, 2 * np.pi, n)
        s[7, :n] = np.cos(th)
        s[8, :n] = np.sin(th)
        s[9, :n] = rng.uniform(*a_range, n)
    else:
        s[7, :n] = 1.0
        s[8, :n] = 0.0
        s[9, :n] = 0.0
    return s


def cell_sites(seed, H, W, n, log_tau=3.0, r=1.0):
    """n isotropic sites at distinct pixel cells (drawn without replacement) plus a
    uniform subpixel offset in [-0.5, 0.5)^2 each, equal log_tau and r (so a pixel's
    exact top-K is its K nearest centres), colours uniform in [0, 1]^3: the site layout
    of the propagation-convergence measurement (Sec. 6.5)."""
    rng = _rng(seed)
    cells = rng.choice(H * W, n, replace=False)
    s = np.zeros((NPARAM, n), np.float32)
    s[0] = np.clip(cells % W + rng.uniform(-0.5, 0.5, n), 0, W - 1)
    s[1] = np.clip(cells // W + rng.uniform(-0.5, 0.5, n), 0, H - 1)
    s[2] = log_tau
    s[3] = r
    s[4:7] = rng.uniform(0, 1, (3, n))
    s[7] = 1.0
    return s


def batch_shapes(seed, n_images=64, lo=256, hi=1024, density=0.05):
    """Uneven image sizes: area log-uniform in [lo^2, hi^2], aspect U[1, 2] with random
    orientation; returns a list of (H, W, n_sites)."""
    rng = _rng(seed)
    out = []
    for _ in range(n_images):
        area = np.exp(rng.uniform(np.log(lo * lo), np.log(hi * hi)))
        asp = rng.uniform(1, 2)
        a = int(round(np.sqrt(area * asp)))
        b = int(round(np.sqrt(area / asp)))
        H, W = (a, b) if rng.uniform() < 0.5 else (b, a)
        out.append((H, W, int(round(density * H * W))))
    return out


def serve_shapes(seed, n_sets=32, lo=512, hi=4096, density=0.05):
    """Resident-set sizes: side log-uniform in [lo, hi] (square), the extremes forced."""
    rng = _rng(seed)
    sides = [lo, hi] + [int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
                        for _ in range(n_sets - 2)]
    return [(sd, sd, int(round(density * sd * sd))) for sd in sides]


def perturb_sites(seed, sites, n, H, W, jitter=0.5, on_centre=0.1, a_range=(-1.5, 1.5),
                  log_tau_jitter=0.5, r_range=(1.0, 3.0)):
    """A copy of sites [10, cap] whose first n slots look like a state part-way through
    an encode: centres moved by U[-jitter, jitter]^2 (a share `on_centre` left exactly
    on their pixel), random directions, anisotropy uniform in a_range, log_tau moved by
    U[-log_tau_jitter, log_tau_jitter], r uniform in r_range.  Positions stay inside
    [0, W-1] x [0, H-1]."""
    rng = _rng(seed)
    s = np.array(sites, dtype=np.float32, copy=True)
    move = rng.uniform(size=n) >= on_centre
    s[0, :n] = np.where(move, np.clip(s[0, :n] + rng.uniform(-jitter, jitter, n), 0, W - 1),
                        s[0, :n])
    s[1, :n] = np.where(move, np.clip(s[1, :n] + rng.uniform(-jitter, jitter, n), 0, H - 1),
                        s[1, :n])
    s[2, :n] += rng.uniform(-log_tau_jitter, log_tau_jitter, n)
    s[3, :n] = rng.uniform(*r_range, n)
    th = rng.uniform(0, 2 * np.pi, n)
    s[7, :n] = np.cos(th)
    s[8, :n] = np.sin(th)
    s[9, :n] = rng.uniform(*a_range, n)
    return s


def sites1d(seed, M, n, cap=None, log_tau_range=(2.0, 5.0), r_range=(1.0, 4.0)):
    """Sites of a one-dimensional signal, float32 [4, cap] in the order (p, c, log_tau, r):
    positions uniform in [0, M-1], values uniform in [-1, 1], log_tau and r uniform in
    their ranges; slots n..cap-1 inactive (p = -1)."""
    rng = _rng(seed)
    cap = n if cap is None else cap
    s = np.zeros((4, cap), np.float32)
    s[0, :] = -1.0
    s[0, :n] = rng.uniform(0, M - 1, n)
    s[1, :n] = rng.uniform(-1, 1, n)
    s[2, :n] = rng.uniform(*log_tau_range, n)
    s[3, :n] = rng.uniform(*r_range, n)
    return s


def signal1d(seed, M, n_steps=12):
    """A one-dimensional target of M samples: n_steps random jumps (piecewise constant,
    values in [-1, 1]) plus a slow sine and a linear ramp, float32 [M]."""
    rng = _rng(seed)
    x = np.arange(M, dtype=np.float64)
    edges = np.sort(rng.uniform(0, M, n_steps))
    levels = rng.uniform(-1, 1, n_steps + 1)
    y = levels[np.searchsorted(edges, x)]
    y = 0.6 * y + 0.25 * np.sin(2 * np.pi * x / rng.uniform(M / 8, M / 2)) + 0.15 * (x / M - 0.5)
    return y.astype(np.float32)
