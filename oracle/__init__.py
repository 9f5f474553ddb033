"""CPU oracle for the Soft Anisotropic Diagrams hot path (numpy front end).

TEST INFRASTRUCTURE ONLY.  This package wraps ``liboracle_sad.so`` (plain C, see
``sad_oracle.c``).  Only ``tests/``, the smoke check in ``__graft_entry__`` and the
CPU-baseline leg of ``bench.py`` may import it; the GPU library and its Python binding
never do.

Layouts follow the C file: ``sites`` float32[10, cap] (x, y, log_tau, r, c_r, c_g, c_b,
u_x, u_y, a), ``lists`` uint32[H*W, K] (pixel-major), images [3, H, W].
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_sad.so")
_lib = None

INVALID = 0xFFFFFFFF
SCORE_F32, SCORE_F64 = 0, 1

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")


def _opt(ptype):
    """ndpointer that also accepts None (a NULL pointer)."""
    class _T(ptype):
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return ptype.from_param(obj)
    return _T


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"oracle library not built: {_LIB_PATH} (run oracle/build.py)")
        L = C.CDLL(_LIB_PATH)
        i64, i32, f32, f64, u64, u32 = C.c_int64, C.c_int, C.c_float, C.c_double, C.c_uint64, C.c_uint32
        L.ora_site_derived.argtypes = [_f32p, i64, i64, f32, _f32p]
        L.ora_score.argtypes = [_f32p, i64, i64, f32, f32, f32]
        L.ora_score.restype = f32
        L.ora_score_f64.argtypes = [_f32p, i64, i64, f64, f64, f64]
        L.ora_score_f64.restype = f64
        L.ora_brute_topk.argtypes = [i32, i32, i32, f32, _f32p, i64, i64, _opt(_i64p), i64, _u32p]
        L.ora_seed.argtypes = [i32, i32, i32, f32, _f32p, i64, i64, _u32p]
        L.ora_jump.argtypes = [i64, i32, i32]
        L.ora_jump.restype = i32
        L.ora_splitmix64.argtypes = [u64, u64]
        L.ora_splitmix64.restype = u64
        L.ora_inject_id.argtypes = [u64, u64, i64, i64, i32, i32, u32]
        L.ora_inject_id.restype = u32
        L.ora_prop_pass.argtypes = [i32, i32, i32, f32, _f32p, i64, i64, _u32p, _u32p, i32, i32,
                                    u64, u64, _opt(_i64p), i64]
        L.ora_render.argtypes = [i32, i32, i32, f32, _f32p, i64, i64, _u32p, i32, _f64p]
        L.ora_query.argtypes = [i32, i32, i32, f32, _f32p, i64, i64, _u32p, _f32p, i64, _f64p]
        L.ora_loss_grad.argtypes = [i32, i32, _f64p, _f32p, _opt(_f64p)]
        L.ora_loss_grad.restype = f64
        L.ora_render_bwd.argtypes = [i32, i32, i32, f32, _f32p, i64, i64, _u32p, _f64p,
                                     _opt(_f32p), i32, _f64p, _opt(_f64p), _opt(_f64p)]
        L.ora_adam.argtypes = [i32, i32, _f64p, _f64p, _f64p, _f64p, i64, i64, _f64p, f64, f64,
                               f64, i64]
        L.ora_init_sites.argtypes = [i32, i32, _f32p, i64, f64, u64, f32, f32, _f32p, i64,
                                     _opt(_f64p)]
        L.ora_init_sites.restype = i64
        L.ora_site_stats.argtypes = [i32, i32, i32, f32, _f32p, i64, i64, _u32p, _f32p, _f64p,
                                     _opt(_f64p), _opt(_f64p)]
        L.ora_densify_prune.argtypes = [i32, i32, i32, _f32p, _f32p, i64, _opt(_f32p),
                                        _opt(_f32p), _f32p, f64, f64, f64, f64, f64, i32,
                                        _opt(_u32p), _i64p]
        L.ora_grid_points.argtypes = [i32, i32, i32, i32, _opt(_f32p), _opt(_i64p)]
        L.ora_prop_pass_grid.argtypes = [i32, i32, i32, i32, i32, f32, _f32p, i64, i64, _u32p,
                                         _u32p, i32, i32, u64, u64]
        L.ora_seed_grid.argtypes = [i32, i32, i32, i32, i32, i32, f32, _f32p, i64, i64, _u32p]
        L.ora_jfa_steps.argtypes = [i32, i32, C.POINTER(C.c_int)]
        L.ora_jfa_steps.restype = i32
        L.ora_jfa_flood.argtypes = [i32, i32, i32, i32, i32, f32, _f32p, i64, i64, _u32p, _u32p,
                                    i32]
        L.ora_jfa_prepass.argtypes = [i32, i32, i32, i32, i32, f32, _f32p, i64, i64, _u32p]
        L.ora_refresh.argtypes = [i32, i32, i32, i32, i32, f32, _f32p, i64, i64, i32, i32, i32,
                                  u64, _u32p]
        L.ora_blend_points.argtypes = [i32, f32, _f32p, i64, i64, _u32p, _f32p, i64, _f64p]
        L.ora_f32_to_f16.argtypes = [f32]
        L.ora_f32_to_f16.restype = C.c_uint16
        L.ora_f16_to_f32.argtypes = [C.c_uint16]
        L.ora_f16_to_f32.restype = f32
        L.ora_pack_qparams.argtypes = [_f32p, i64, i64, _f32p]
        L.ora_pack_sites.argtypes = [i32, i32, _f32p, i64, i64, _f32p, _u32p]
        L.ora_unpack_sites.argtypes = [i32, i32, _u32p, i64, _f32p, _f32p, i64]
        L.ora_tau_diffusion.argtypes = [i32, i32, i32, f32, _f32p, i64, i64, _u32p, _f64p, f64,
                                         _f64p]
        L.ora1d_brute_topk.argtypes = [i32, i32, f32, _f32p, i64, i64, _u32p]
        L.ora1d_seed.argtypes = [i32, i32, f32, _f32p, i64, i64, _u32p]
        L.ora1d_prop_pass.argtypes = [i32, i32, f32, _f32p, i64, i64, _u32p, _u32p, i32, i32, u64,
                                      u64]
        L.ora1d_render_loss_bwd.argtypes = [i32, i32, f32, _f32p, i64, i64, _u32p, _opt(_f32p),
                                            i32, _opt(_f64p), _opt(_f64p), _opt(_f64p)]
        L.ora1d_render_loss_bwd.restype = f64
        L.ora1d_adam.argtypes = [i32, _f64p, _f64p, _f64p, _f64p, i64, i64, _f64p, f64, f64, f64,
                                 i64]
        L.ora_set_threads.argtypes = [i32]
        L.ora_set_threads.restype = i32
        _lib = L
    return _lib


def set_threads(n):
    """Threads of the oracle's per-pixel loops (1 = one core); returns the previous
    number.  n <= 0 only queries it."""
    return int(lib().ora_set_threads(int(n)))


def _sites(sites):
    s = np.ascontiguousarray(sites, dtype=np.float32)
    assert s.ndim == 2 and s.shape[0] == 10, s.shape
    return s


def _lists(lists, HW, K):
    a = np.ascontiguousarray(lists, dtype=np.uint32).reshape(HW, K)
    return a


def default_scale(H, W):
    """s = 1 / max(H, W) (Sec. 4.1), as a float32."""
    return float(np.float32(1.0) / np.float32(max(H, W)))


def site_derived(sites, n, s):
    sites = _sites(sites)
    out = np.zeros((n, 8), np.float32)
    lib().ora_site_derived(sites, sites.shape[1], n, s, out)
    return out


def score(sites, i, s, X, Y):
    sites = _sites(sites)
    return float(lib().ora_score(sites, sites.shape[1], i, s, X, Y))


def score_f64(sites, i, s, X, Y):
    sites = _sites(sites)
    return float(lib().ora_score_f64(sites, sites.shape[1], i, s, X, Y))


def brute_topk(H, W, K, s, sites, n, pix=None):
    sites = _sites(sites)
    if pix is not None:
        pix = np.ascontiguousarray(pix, dtype=np.int64)
        npix = len(pix)
    else:
        npix = H * W
    out = np.empty((npix, K), np.uint32)
    lib().ora_brute_topk(H, W, K, s, sites, sites.shape[1], n, pix, npix, out)
    return out


def seed_lists(H, W, K, s, sites, n):
    sites = _sites(sites)
    out = np.empty((H * W, K), np.uint32)
    lib().ora_seed(H, W, K, s, sites, sites.shape[1], n, out)
    return out


def jump(t, H, W):
    return int(lib().ora_jump(t, H, W))


def splitmix64(seed, k):
    return int(lib().ora_splitmix64(seed, k))


def inject_id(seed, t, P, p, J, j, n_slots):
    return int(lib().ora_inject_id(seed, t, P, p, J, j, n_slots))


def prop_pass(H, W, K, s, sites, n, lists, jump_, J, seed, t, pix=None):
    sites = _sites(sites)
    lin = _lists(lists, H * W, K)
    if pix is not None:
        pix = np.ascontiguousarray(pix, dtype=np.int64)
        npix = len(pix)
    else:
        npix = H * W
    out = np.empty((npix, K), np.uint32)
    lib().ora_prop_pass(H, W, K, s, sites, sites.shape[1], n, lin, out, jump_, J, seed, t, pix, npix)
    return out


def render(H, W, K, s, sites, n, lists, mode=SCORE_F32):
    sites = _sites(sites)
    out = np.empty((3, H, W), np.float64)
    lib().ora_render(H, W, K, s, sites, sites.shape[1], n, _lists(lists, H * W, K), mode, out)
    return out


def query(H, W, K, s, sites, n, lists, xy):
    sites = _sites(sites)
    xy = np.ascontiguousarray(xy, dtype=np.float32).reshape(-1, 2)
    out = np.empty((len(xy), 3), np.float64)
    lib().ora_query(H, W, K, s, sites, sites.shape[1], n, _lists(lists, H * W, K), xy, len(xy), out)
    return out


def loss_grad(img, target):
    img = np.ascontiguousarray(img, dtype=np.float64)
    target = np.ascontiguousarray(target, dtype=np.float32)
    _, H, W = img.shape
    g = np.empty_like(img)
    L = lib().ora_loss_grad(H, W, img, target, g)
    return float(L), g


def render_bwd(H, W, K, s, sites, n, lists, grad_img, target=None, mode=SCORE_F32,
               removal_delta=False, abs_sum=False):
    """Gradient [10, cap]; with removal_delta=True also the removal delta [cap]; with
    abs_sum=True also the sum of absolute per-pixel terms [10, cap] (returned last)."""
    sites = _sites(sites)
    cap = sites.shape[1]
    grad_img = np.ascontiguousarray(grad_img, dtype=np.float64)
    grad = np.zeros((10, cap), np.float64)
    rd = np.zeros(cap, np.float64) if removal_delta else None
    ga = np.zeros((10, cap), np.float64) if abs_sum else None
    tgt = np.ascontiguousarray(target, dtype=np.float32) if target is not None else None
    lib().ora_render_bwd(H, W, K, s, sites, cap, n, _lists(lists, H * W, K), grad_img, tgt, mode,
                         grad, rd, ga)
    out = [grad]
    if removal_delta:
        out.append(rd)
    if abs_sum:
        out.append(ga)
    return out[0] if len(out) == 1 else tuple(out)


def adam(H, W, sites, grad, m, v, n, lr, b1, b2, eps, t):
    """In place on float64 arrays sites/m/v [10, cap]."""
    cap = sites.shape[1]
    lr = np.ascontiguousarray(lr, dtype=np.float64)
    lib().ora_adam(H, W, sites, np.ascontiguousarray(grad, np.float64), m, v, cap, n, lr,
                   b1, b2, eps, t)


def init_sites(target, N, lam, seed, log_tau0, r0, cap, return_keys=False):
    target = np.ascontiguousarray(target, dtype=np.float32)
    _, H, W = target.shape
    sites = np.empty((10, cap), np.float32)
    keys = np.empty(H * W, np.float64) if return_keys else None
    k = lib().ora_init_sites(H, W, target, N, lam, seed, log_tau0, r0, sites, cap, keys)
    return (sites, int(k), keys) if return_keys else (sites, int(k))


NSTAT = 8
DP_PRUNE, DP_SPLIT, DP_SEED = 1, 2, 4


def site_stats(H, W, K, s, sites, n, lists, target, scales=False):
    """Statistics [8, cap] (m, E, S_x, S_y, S_xx, S_xy, S_yy, removal delta); with
    scales=True also the sums of |term| and the sensitivity scales, each [8, cap]."""
    L = lib()
    sites = _sites(sites)
    cap = sites.shape[1]
    out = np.zeros((NSTAT, cap), np.float64)
    sa = np.zeros((NSTAT, cap), np.float64) if scales else None
    ss = np.zeros((NSTAT, cap), np.float64) if scales else None
    L.ora_site_stats(H, W, K, s, sites, cap, n, _lists(lists, H * W, K),
                     np.ascontiguousarray(target, dtype=np.float32), out, sa, ss)
    return (out, sa, ss) if scales else out


def densify_prune(target, sites, stats, p_prune, p_split, flags, K=8, adam_m=None, adam_v=None,
                  lists=None, alpha=0.7, eps=1e-8, min_mass=1.0):
    """One budget step, in place on float32 sites [10, cap] (and adam_m / adam_v, lists
    [H*W, K] if given).  Returns counts (n_active, n_pruned, n_split, n_after, high
    water, candidates)."""
    L = lib()
    target = np.ascontiguousarray(target, dtype=np.float32)
    _, H, W = target.shape
    assert sites.dtype == np.float32 and sites.flags.c_contiguous
    cap = sites.shape[1]
    st = np.ascontiguousarray(stats, dtype=np.float32)
    assert st.shape == (NSTAT, cap)
    counts = np.zeros(6, np.int64)
    if lists is not None:
        assert lists.dtype == np.uint32 and lists.flags.c_contiguous
    L.ora_densify_prune(H, W, K, target, sites, cap, adam_m, adam_v, st, p_prune, p_split, alpha,
                        eps, min_mass, flags, lists, counts)
    return [int(c) for c in counts]


# ---- evaluation grids and the full refresh (App. B.3) ---------------------------------

def grid_points(H, W, Hg, Wg):
    """Points of the cells of an Hg x Wg grid over an H x W image: float32 [Hg*Wg, 2]
    (x, y), and the cell of every image pixel: int64 [H*W]."""
    xy = np.empty((Hg * Wg, 2), np.float32)
    cell = np.empty(H * W, np.int64)
    lib().ora_grid_points(H, W, Hg, Wg, xy, cell)
    return xy, cell


def prop_pass_grid(H, W, Hg, Wg, K, s, sites, n, lists, jump_, J, seed, t):
    sites = _sites(sites)
    out = np.empty((Hg * Wg, K), np.uint32)
    lib().ora_prop_pass_grid(H, W, Hg, Wg, K, s, sites, sites.shape[1], n,
                             _lists(lists, Hg * Wg, K), out, jump_, J, seed, t)
    return out


def seed_grid(H, W, Hg, Wg, K, n_entries, s, sites, n):
    sites = _sites(sites)
    out = np.empty((Hg * Wg, K), np.uint32)
    lib().ora_seed_grid(H, W, Hg, Wg, K, n_entries, s, sites, sites.shape[1], n, out)
    return out


def jfa_steps(Hg, Wg):
    buf = (C.c_int * 32)()
    L = int(lib().ora_jfa_steps(Hg, Wg, buf))
    return [int(buf[k]) for k in range(L)]


def jfa_flood(H, W, Hg, Wg, K, s, sites, n, lists, step, out=None):
    """One flood pass; entries 4..K-1 of the result are those of `out` (default: a copy
    of the input lists), since the pass writes the first four entries only."""
    sites = _sites(sites)
    lin = _lists(lists, Hg * Wg, K)
    res = lin.copy() if out is None else np.ascontiguousarray(out, dtype=np.uint32).copy()
    lib().ora_jfa_flood(H, W, Hg, Wg, K, s, sites, sites.shape[1], n, lin, res, step)
    return res


def jfa_prepass(H, W, Hg, Wg, K, s, sites, n):
    sites = _sites(sites)
    out = np.empty((Hg * Wg, K), np.uint32)
    lib().ora_jfa_prepass(H, W, Hg, Wg, K, s, sites, sites.shape[1], n, out)
    return out


def refresh(H, W, Hg, Wg, K, s, sites, n, jfa, n_pass, J, seed):
    sites = _sites(sites)
    out = np.empty((Hg * Wg, K), np.uint32)
    lib().ora_refresh(H, W, Hg, Wg, K, s, sites, sites.shape[1], n, int(bool(jfa)), n_pass, J,
                      seed, out)
    return out


def blend_points(K, s, sites, n, lists, xy):
    sites = _sites(sites)
    xy = np.ascontiguousarray(xy, dtype=np.float32).reshape(-1, 2)
    out = np.empty((len(xy), 3), np.float64)
    lib().ora_blend_points(K, s, sites, sites.shape[1], n, _lists(lists, len(xy), K), xy,
                           len(xy), out)
    return out


def expand_grid_lists(H, W, Hg, Wg, lists):
    """Per-pixel lists of an image whose list field lives on a candidate grid: pixel p
    takes the list of its cell (the integer map of App. B.3)."""
    _, cell = grid_points(H, W, Hg, Wg)
    return np.ascontiguousarray(np.asarray(lists, np.uint32).reshape(Hg * Wg, -1)[cell])


# ---- packed 16-byte inference record (App. B.2; Sec. 6.1) -------------------------------

def f32_to_f16(x):
    return int(lib().ora_f32_to_f16(float(x)))


def f16_to_f32(h):
    return float(lib().ora_f16_to_f32(int(h)))


def pack_qparams(sites, n):
    sites = _sites(sites)
    q = np.zeros(10, np.float32)
    lib().ora_pack_qparams(sites, sites.shape[1], n, q)
    return q


def pack_sites(H, W, sites, n, q=None):
    """(packed uint32 [n, 4], qparams float32 [10])."""
    sites = _sites(sites)
    q = pack_qparams(sites, n) if q is None else np.ascontiguousarray(q, np.float32)
    out = np.zeros((n, 4), np.uint32)
    lib().ora_pack_sites(H, W, sites, sites.shape[1], n, q, out)
    return out, q


def unpack_sites(H, W, packed, q, cap=None):
    packed = np.ascontiguousarray(packed, np.uint32).reshape(-1, 4)
    n = len(packed)
    cap = n if cap is None else cap
    out = np.zeros((10, cap), np.float32)
    out[0:2, :] = -1.0
    lib().ora_unpack_sites(H, W, packed, n, np.ascontiguousarray(q, np.float32), out, cap)
    return out


def bpp(n, H, W):
    """Parameter-space bits per pixel of n packed records (Sec. 6.1): n 16 8 / (H W)."""
    return n * 16 * 8 / (H * W)


# ---- tau diffusion (App. B.6) ----------------------------------------------------------

def tau_diffusion(H, W, K, s, sites, n, lists, g, lam):
    """One Jacobi step of the log tau gradient smoothing; g: [n] -> [n] (float64)."""
    sites = _sites(sites)
    g = np.ascontiguousarray(g, np.float64)
    out = np.empty(n, np.float64)
    lib().ora_tau_diffusion(H, W, K, s, sites, sites.shape[1], n, _lists(lists, H * W, K), g,
                            float(lam), out)
    return out


# ---- one-dimensional SAD (Sec. 7) ----------------------------------------------------------

def _sites1(sites):
    s = np.ascontiguousarray(sites, dtype=np.float32)
    assert s.ndim == 2 and s.shape[0] == 4, s.shape
    return s


def scale1d(M):
    return float(np.float32(1.0) / np.float32(M))


def brute_topk1d(M, K, s, sites, n):
    sites = _sites1(sites)
    out = np.empty((M, K), np.uint32)
    lib().ora1d_brute_topk(M, K, s, sites, sites.shape[1], n, out)
    return out


def seed1d(M, K, s, sites, n):
    sites = _sites1(sites)
    out = np.empty((M, K), np.uint32)
    lib().ora1d_seed(M, K, s, sites, sites.shape[1], n, out)
    return out


def prop_pass1d(M, K, s, sites, n, lists, jump_, J, seed, t):
    sites = _sites1(sites)
    out = np.empty((M, K), np.uint32)
    lib().ora1d_prop_pass(M, K, s, sites, sites.shape[1], n, _lists(lists, M, K), out, jump_, J,
                          seed, t)
    return out


def render1d(M, K, s, sites, n, lists, target=None, mode=SCORE_F32, grad=False, abs_sum=False):
    """(colours [M], loss or None, gradient [4, cap] or None, abs sums or None)."""
    sites = _sites1(sites)
    cap = sites.shape[1]
    out = np.empty(M, np.float64)
    g = np.zeros((4, cap), np.float64) if grad else None
    ga = np.zeros((4, cap), np.float64) if abs_sum else None
    tgt = None if target is None else np.ascontiguousarray(target, np.float32)
    L = lib().ora1d_render_loss_bwd(M, K, s, sites, cap, n, _lists(lists, M, K), tgt, mode, out,
                                    g, ga)
    return out, (L if target is not None else None), g, ga


def adam1d(M, sites, grad, m, v, n, lr, b1, b2, eps, t):
    cap = sites.shape[1]
    lib().ora1d_adam(M, sites, np.ascontiguousarray(grad, np.float64), m, v, cap, n,
                     np.ascontiguousarray(lr, np.float64), b1, b2, eps, t)
