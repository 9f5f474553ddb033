"""ctypes binding of ``libsad.so`` -- the C ABI declared in ``include/sad.h``.

Argument marshalling only: every function takes torch tensors (device memory owned by
the caller), checks dtype / device / size, and passes raw pointers, sizes and the
current HIP stream to the entry point of the same name.  All computation happens in
the library's kernels.  If the library is missing this module raises at import time:
there is no fallback path.
"""
import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# SAD_LIBRARY may name another build of the same library (same ABI), e.g. for A/B timing
LIB_PATH = os.environ.get("SAD_LIBRARY") or os.path.join(_HERE, "libsad.so")

NPARAM = 10
REC_FLOATS = 16
LOSS_PARTS = 64
LOSS_ACC_FLOATS = 1 + LOSS_PARTS          # sad_loss_acc
STEP_STATE_INT64 = (16 + 4 * LOSS_ACC_FLOATS + 7) // 8 + 1   # sad_step_state (+ block counter)
INVALID_ID = 0xFFFFFFFF
MAX_K = 32


class SadError(RuntimeError):
    pass


class SadImage(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("K", C.c_int32), ("n_slots", C.c_int32),
                ("cap", C.c_int64), ("score_scale", C.c_float)]


class SadAdamParams(C.Structure):
    _fields_ = [("lr", C.c_float * NPARAM), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


class SadTrainConfig(C.Structure):
    _fields_ = [("n_inject", C.c_int32), ("fixed_jump", C.c_int32), ("seed", C.c_uint64),
                ("adam", SadAdamParams), ("prop_every", C.c_int32), ("flags", C.c_uint32)]


class SadBatchImage(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("n_slots", C.c_int32), ("tile0", C.c_int32),
                ("cap", C.c_int64), ("px0", C.c_int64), ("site0", C.c_int64),
                ("score_scale", C.c_float), ("pad", C.c_int32)]


class SadBatch(C.Structure):
    _fields_ = [("n_images", C.c_int32), ("K", C.c_int32), ("n_items", C.c_int32),
                ("grid", C.c_int32), ("chunked", C.c_int32), ("tile_w", C.c_int32),
                ("n_site_slots", C.c_int64), ("images", C.c_void_p)]


class SadBudgetParams(C.Structure):
    _fields_ = [("p_prune", C.c_double), ("p_split", C.c_double), ("alpha", C.c_double),
                ("eps", C.c_double), ("min_mass", C.c_double), ("flags", C.c_uint32),
                ("pad", C.c_uint32)]


class SadQueryJob(C.Structure):
    _fields_ = [("rec", C.c_void_p), ("topk", C.c_void_p), ("xy", C.c_void_p), ("out", C.c_void_p),
                ("M", C.c_int64), ("q0", C.c_int64), ("H", C.c_int32), ("W", C.c_int32),
                ("n_slots", C.c_int32), ("pad", C.c_int32)]


class SadSignal(C.Structure):
    _fields_ = [("M", C.c_int32), ("K", C.c_int32), ("n_slots", C.c_int32), ("pad", C.c_int32),
                ("cap", C.c_int64), ("score_scale", C.c_float)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, U64, F32, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_float, C.c_size_t
    IMG = C.POINTER(SadImage)
    sig = {
        "sad_prepare_sites": [IMG, P, P, P],
        "sad_seed_topk": [IMG, P, P, P, P],
        "sad_seed_topk_noalloc": [IMG, P, P, P],
        "sad_propagate_topk": [IMG, P, P, P, I32, I32, U64, U64, P],
        "sad_render_fwd": [IMG, P, P, P, P],
        "sad_loss_grad": [IMG, P, P, P, P, P],
        "sad_render_bwd": [IMG, P, P, P, P, P, P, P],
        "sad_adam_step": [IMG, P, P, P, P, C.POINTER(SadAdamParams), I64, P, C.c_uint32, P],
        "sad_propagate_topk_state": [IMG, P, P, P, I32, U64, P, P],
        "sad_adam_step_state": [IMG, P, P, P, P, C.POINTER(SadAdamParams), P, C.c_uint32, P, P],
        "sad_render_fwd_loss": [IMG, P, P, P, P, P, P, P],
        "sad_query_points": [IMG, P, P, P, I64, P, P],
        "sad_init_sites": [IMG, P, I32, F32, U64, F32, F32, P, P, C.POINTER(SZ), P],
        "sad_train_step": [IMG, C.POINTER(SadTrainConfig), P, P, P, P, P, P, P, P, P, P, P, P],
        "sad_train_image_pass": [IMG, C.POINTER(SadTrainConfig), P, P, P, P, P, P, P, P, P],
        "sad_query_batch": [P, I32, I64, I32, P],
        "sad_site_stats": [IMG, P, P, P, P, P],
        "sad_site_stats_fixed": [IMG, P, P, P, P, P, P],
        "sad_exact_topk": [IMG, P, P, I64, P, P],
        "sad_densify_prune": [IMG, P, P, P, P, P, C.POINTER(SadBudgetParams), P, P, P,
                              C.POINTER(SZ), P],
        "sad_batch_train_step": [C.POINTER(SadBatch), C.POINTER(SadTrainConfig), P, P, P, P, P, P,
                                 P, P, P, P, P, P],
        "sad_seed_grid": [IMG, I32, I32, I32, P, P, P, P],
        "sad_propagate_grid": [IMG, I32, I32, P, P, P, I32, I32, U64, U64, P],
        "sad_jfa_flood": [IMG, I32, I32, P, P, P, I32, P],
        "sad_refresh": [IMG, I32, I32, C.c_uint32, I32, I32, U64, P, P, P, P, P],
        "sad_render_grid": [IMG, I32, I32, P, P, I32, I32, P, P],
        "sad_pack_qparams": [IMG, P, P, P],
        "sad_pack_sites": [IMG, P, P, P, P],
        "sad_unpack_sites": [IMG, P, P, P, P],
        "sad_prepare_packed": [IMG, P, P, P, P],
        "sad_render_packed": [IMG, P, P, P, P, P],
        "sad_query_packed": [IMG, P, P, P, P, I64, P, P],
        "sad_tau_diffusion": [IMG, P, P, P, I64, F32, P, I64, P],
        "sad_grad_to_params": [IMG, P, P, P, C.c_uint32, P],
        "sad1d_prepare": [C.POINTER(SadSignal), P, P, P],
        "sad1d_seed": [C.POINTER(SadSignal), P, P, P, P],
        "sad1d_propagate": [C.POINTER(SadSignal), P, P, P, I32, I32, U64, U64, P],
        "sad1d_render": [C.POINTER(SadSignal), P, P, P, P, P, P, P],
        "sad1d_adam": [C.POINTER(SadSignal), P, P, P, P, C.POINTER(F32), F32, F32, F32, I64, P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.sad_jump_step.argtypes = [I64, I32, I32]
    L.sad_jump_step.restype = I32
    L.sad_jfa_steps.argtypes = [I32, I32, C.POINTER(I32)]
    L.sad_jfa_steps.restype = I32
    for name in ("sad_status_string",):
        getattr(L, name).argtypes = [C.c_int]
        getattr(L, name).restype = C.c_char_p
    L.sad_last_error.argtypes = []
    L.sad_last_error.restype = C.c_char_p
    L.sad_version.argtypes = []
    L.sad_version.restype = C.c_char_p
    return L


lib = _load()


def _check(status, name):
    if status != 0:
        msg = lib.sad_last_error().decode(errors="replace")
        raise SadError(f"{name}: {lib.sad_status_string(status).decode()} ({status}): {msg}")


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream():
    """The current HIP stream of the current device (the one torch launches on)."""
    if _raw_stream is not None:   # no Stream object: this runs once per call
        return C.c_void_p(_raw_stream(torch._C._cuda_getDevice()))
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise TypeError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: needs at least {numel} elements, has {t.numel()}")
    return C.c_void_p(t.data_ptr())


def image(H, W, K, n_slots, cap=None, score_scale=0.0):
    """Image descriptor (sad_image)."""
    return SadImage(int(H), int(W), int(K), int(n_slots), int(cap if cap is not None else n_slots),
                    float(score_scale))


def prepare_sites(img, sites, rec):
    _check(lib.sad_prepare_sites(C.byref(img), _ptr(sites, torch.float32, NPARAM * img.cap, "sites"),
                                 _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"), _stream()),
           "sad_prepare_sites")


def seed_topk(img, rec, topk, scratch):
    P = img.H * img.W
    if scratch.numel() * scratch.element_size() < 8 * P:
        raise ValueError("seed_topk: scratch needs 8 bytes per pixel")
    _check(lib.sad_seed_topk(C.byref(img), _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                             _ptr(topk, torch.int32, img.K * P, "topk"),
                             _ptr(scratch, scratch.dtype, None, "scratch"), _stream()),
           "sad_seed_topk")


SEED_STATIC_PIXELS = 1 << 22


def seed_topk_noalloc(img, rec, topk):
    """sad_seed_topk with the library's static per-device scratch (no allocation); images
    of up to SEED_STATIC_PIXELS pixels."""
    P = img.H * img.W
    _check(lib.sad_seed_topk_noalloc(C.byref(img),
                                     _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                                     _ptr(topk, torch.int32, img.K * P, "topk"), _stream()),
           "sad_seed_topk_noalloc")


def propagate_topk(img, rec, topk_in, topk_out, jump, n_inject, seed, pass_index):
    P = img.H * img.W
    _check(lib.sad_propagate_topk(C.byref(img), _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                                  _ptr(topk_in, torch.int32, img.K * P, "topk_in"),
                                  _ptr(topk_out, torch.int32, img.K * P, "topk_out"),
                                  int(jump), int(n_inject), int(seed) & (2 ** 64 - 1),
                                  int(pass_index), _stream()),
           "sad_propagate_topk")


def propagate_topk_state(img, rec, topk_in, topk_out, n_inject, seed, state):
    """sad_propagate_topk_state: pass index and jump from state (a step_state())."""
    P = img.H * img.W
    _check(lib.sad_propagate_topk_state(C.byref(img),
                                        _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                                        _ptr(topk_in, torch.int32, img.K * P, "topk_in"),
                                        _ptr(topk_out, torch.int32, img.K * P, "topk_out"),
                                        int(n_inject), int(seed) & (2 ** 64 - 1),
                                        _ptr(state, torch.int64, STEP_STATE_INT64, "state"),
                                        _stream()),
           "sad_propagate_topk_state")


def jump_step(t, H, W):
    return int(lib.sad_jump_step(int(t), int(H), int(W)))


def render_fwd(img, rec, topk, out):
    P = img.H * img.W
    _check(lib.sad_render_fwd(C.byref(img), _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                              _ptr(topk, torch.int32, img.K * P, "topk"),
                              _ptr(out, torch.float32, 3 * P, "out"), _stream()),
           "sad_render_fwd")


def loss_acc(device="cuda"):
    """A zeroed sad_loss_acc on the device (value = element 0)."""
    return torch.zeros(LOSS_ACC_FLOATS, dtype=torch.float32, device=device)


def step_state(device="cuda"):
    """A zeroed sad_step_state on the device."""
    return torch.zeros(STEP_STATE_INT64, dtype=torch.int64, device=device)


def state_counters(state):
    """(pass, adam_step) of a sad_step_state tensor (device tensor of 2 int64)."""
    return state[:2]


def state_loss(state):
    """loss.value of a sad_step_state tensor (0-d device float tensor)."""
    return state.view(torch.float32)[4]


def loss_grad(img, rendered, target, grad, loss=None):
    P = img.H * img.W
    _check(lib.sad_loss_grad(C.byref(img), _ptr(rendered, torch.float32, 3 * P, "rendered"),
                             _ptr(target, torch.float32, 3 * P, "target"),
                             _ptr(grad, torch.float32, 3 * P, "grad"),
                             _ptr(loss, torch.float32, LOSS_ACC_FLOATS, "loss"), _stream()),
           "sad_loss_grad")


def render_bwd(img, rec, topk, grad_img, grad_sites, target=None, removal_delta=None):
    P = img.H * img.W
    _check(lib.sad_render_bwd(C.byref(img), _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                              _ptr(topk, torch.int32, img.K * P, "topk"),
                              _ptr(grad_img, torch.float32, 3 * P, "grad_img"),
                              _ptr(target, torch.float32, 3 * P, "target"),
                              _ptr(grad_sites, torch.float32, NPARAM * img.cap, "grad_sites"),
                              _ptr(removal_delta, torch.float32, img.cap, "removal_delta"), _stream()),
           "sad_render_bwd")


def adam_params(lr, beta1=0.9, beta2=0.999, eps=1e-8):
    p = SadAdamParams()
    for i in range(NPARAM):
        p.lr[i] = float(lr[i])
    p.beta1, p.beta2, p.eps = float(beta1), float(beta2), float(eps)
    return p


ADAM_ZERO_GRAD = 1
ADAM_GRAD_SITE_MAJOR = 2
ADAM_GRAD_FIXED = 4
TRAIN_DETERMINISTIC = 1
TRAIN_LOSS_SET = 2


def _grad_dtype(cfg):
    """Element type of a training step's gradient accumulator under cfg."""
    return torch.int64 if cfg.flags & TRAIN_DETERMINISTIC else torch.float32


def adam_step(img, sites, grad, m, v, params, step, rec=None, zero_grad=False,
              grad_site_major=False, grad_fixed=False):
    """sad_adam_step; grad is [10][cap], or the training step's [cap][10] accumulator
    with grad_site_major=True; int64 fixed point (a deterministic step's accumulator)
    with grad_fixed=True."""
    n = NPARAM * img.cap
    _check(lib.sad_adam_step(C.byref(img), _ptr(sites, torch.float32, n, "sites"),
                             _ptr(grad, torch.int64 if grad_fixed else torch.float32, n, "grad"),
                             _ptr(m, torch.float32, n, "m"),
                             _ptr(v, torch.float32, n, "v"), C.byref(params), int(step),
                             _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                             (ADAM_ZERO_GRAD if zero_grad else 0) |
                             (ADAM_GRAD_SITE_MAJOR if grad_site_major else 0) |
                             (ADAM_GRAD_FIXED if grad_fixed else 0), _stream()),
           "sad_adam_step")


def render_fwd_loss(img, rec, topk, target, grad_img, rendered=None, loss=None):
    P = img.H * img.W
    _check(lib.sad_render_fwd_loss(C.byref(img), _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                                   _ptr(topk, torch.int32, img.K * P, "topk"),
                                   _ptr(target, torch.float32, 3 * P, "target"),
                                   _ptr(rendered, torch.float32, 3 * P, "rendered"),
                                   _ptr(grad_img, torch.float32, 3 * P, "grad_img"),
                                   _ptr(loss, torch.float32, LOSS_ACC_FLOATS, "loss"), _stream()),
           "sad_render_fwd_loss")


def query_points(img, rec, topk, xy, out):
    M = xy.shape[0] if xy.dim() == 2 else xy.numel() // 2
    P = img.H * img.W
    _check(lib.sad_query_points(C.byref(img), _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                                _ptr(topk, torch.int32, img.K * P, "topk"),
                                _ptr(xy, torch.float32, 2 * M, "xy"), int(M),
                                _ptr(out, torch.float32, 3 * M, "out"), _stream()),
           "sad_query_points")


def init_workspace_bytes(img):
    n = C.c_size_t(0)
    _check(lib.sad_init_sites(C.byref(img), None, 0, 0.0, 0, 0.0, 0.0, None, None, C.byref(n), None),
           "sad_init_sites")
    return int(n.value)


def init_sites(img, target, n_sites, lam, seed, log_tau0, r0, sites, workspace):
    P = img.H * img.W
    nbytes = C.c_size_t(workspace.numel() * workspace.element_size())
    _check(lib.sad_init_sites(C.byref(img), _ptr(target, torch.float32, 3 * P, "target"), int(n_sites),
                              float(lam), int(seed) & (2 ** 64 - 1), float(log_tau0), float(r0),
                              _ptr(sites, torch.float32, NPARAM * img.cap, "sites"),
                              _ptr(workspace, workspace.dtype, None, "workspace"), C.byref(nbytes),
                              _stream()),
           "sad_init_sites")


def exact_topk(img, rec, pix, out):
    """Brute-force top-K of the pixels pix (device int64) into out [n, K] (sad_exact_topk)."""
    n = pix.numel()
    _check(lib.sad_exact_topk(C.byref(img), _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                              _ptr(pix, torch.int64, n, "pix"), int(n),
                              _ptr(out, torch.int32, n * img.K, "out"), _stream()),
           "sad_exact_topk")


NSTAT = 8
DP_PRUNE, DP_SPLIT, DP_SEED = 1, 2, 4


def site_stats(img, rec, topk, target, stats):
    """Accumulate the per-site statistics into stats [8, cap] (sad_site_stats)."""
    P = img.H * img.W
    _check(lib.sad_site_stats(C.byref(img), _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                              _ptr(topk, torch.int32, img.K * P, "topk"),
                              _ptr(target, torch.float32, 3 * P, "target"),
                              _ptr(stats, torch.float32, NSTAT * img.cap, "stats"), _stream()),
           "sad_site_stats")


def site_stats_fixed(img, rec, topk, target, acc, stats):
    """Write the per-site statistics into stats [8, cap] with integer sums that do not
    depend on scheduling (sad_site_stats_fixed); acc: int64 workspace of 16 * cap."""
    P = img.H * img.W
    _check(lib.sad_site_stats_fixed(C.byref(img),
                                    _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                                    _ptr(topk, torch.int32, img.K * P, "topk"),
                                    _ptr(target, torch.float32, 3 * P, "target"),
                                    _ptr(acc, torch.int64, 2 * NSTAT * img.cap, "acc"),
                                    _ptr(stats, torch.float32, NSTAT * img.cap, "stats"),
                                    _stream()),
           "sad_site_stats_fixed")


def budget_params(p_prune, p_split, flags, alpha=0.7, eps=1e-8, min_mass=1.0):
    return SadBudgetParams(float(p_prune), float(p_split), float(alpha), float(eps),
                           float(min_mass), int(flags), 0)


def densify_workspace_bytes(img):
    n = C.c_size_t(0)
    _check(lib.sad_densify_prune(C.byref(img), None, None, None, None, None, None, None, None, None,
                                 C.byref(n), None), "sad_densify_prune")
    return int(n.value)


def densify_prune(img, target, sites, adam_m, adam_v, stats, params, topk, counts, workspace):
    """One budget step (sad_densify_prune); counts: device int64[6]."""
    P = img.H * img.W
    nbytes = C.c_size_t(workspace.numel() * workspace.element_size())
    _check(lib.sad_densify_prune(C.byref(img), _ptr(target, torch.float32, 3 * P, "target"),
                                 _ptr(sites, torch.float32, NPARAM * img.cap, "sites"),
                                 _ptr(adam_m, torch.float32, NPARAM * img.cap, "adam_m"),
                                 _ptr(adam_v, torch.float32, NPARAM * img.cap, "adam_v"),
                                 _ptr(stats, torch.float32, NSTAT * img.cap, "stats"),
                                 C.byref(params), _ptr(topk, torch.int32, img.K * P, "topk"),
                                 _ptr(counts, torch.int64, 6, "counts"),
                                 _ptr(workspace, workspace.dtype, None, "workspace"), C.byref(nbytes),
                                 _stream()),
           "sad_densify_prune")


def version():
    return lib.sad_version().decode()


def train_config(n_inject, seed, adam, fixed_jump=0, prop_every=1, deterministic=False,
                 loss_set=False):
    """sad_train_config; deterministic=True makes the gradient accumulator int64 fixed
    point (allocate it as torch.int64, same shape) and the sums bit-reproducible;
    loss_set=True makes sad_train_image_pass store L instead of adding it."""
    c = SadTrainConfig()
    c.n_inject, c.fixed_jump, c.seed, c.adam = int(n_inject), int(fixed_jump), int(seed) & (2 ** 64 - 1), adam
    c.prop_every = int(prop_every)
    c.flags = (TRAIN_DETERMINISTIC if deterministic else 0) | (TRAIN_LOSS_SET if loss_set else 0)
    return c


def adam_step_state(img, sites, grad, m, v, params, rec, state, zero_grad=False,
                    grad_site_major=False):
    """sad_adam_step_state: step from state, whose counters advance at the end."""
    n = NPARAM * img.cap
    _check(lib.sad_adam_step_state(C.byref(img), _ptr(sites, torch.float32, n, "sites"),
                                   _ptr(grad, torch.float32, n, "grad"),
                                   _ptr(m, torch.float32, n, "m"), _ptr(v, torch.float32, n, "v"),
                                   C.byref(params),
                                   _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                                   (ADAM_ZERO_GRAD if zero_grad else 0) |
                                   (ADAM_GRAD_SITE_MAJOR if grad_site_major else 0),
                                   _ptr(state, torch.int64, STEP_STATE_INT64, "state"), _stream()),
           "sad_adam_step_state")


def train_step(img, cfg, target, sites, rec, topk_in, topk_out, grad, m, v, rendered, grad_img,
               state):
    """One iteration (sad_train_step); state: a sad_step_state tensor (step_state())."""
    P = img.H * img.W
    n = NPARAM * img.cap
    _check(lib.sad_train_step(C.byref(img), C.byref(cfg), _ptr(target, torch.float32, 3 * P, "target"),
                              _ptr(sites, torch.float32, n, "sites"),
                              _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                              _ptr(topk_in, torch.int32, img.K * P, "topk_in"),
                              _ptr(topk_out, torch.int32, img.K * P, "topk_out"),
                              _ptr(grad, _grad_dtype(cfg), n, "grad"), _ptr(m, torch.float32, n, "m"),
                              _ptr(v, torch.float32, n, "v"),
                              _ptr(rendered, torch.float32, 3 * P, "rendered"),
                              _ptr(grad_img, torch.float32, 3 * P, "grad_img"),
                              _ptr(state, torch.int64, STEP_STATE_INT64, "state"), _stream()),
           "sad_train_step")


def train_image_pass(img, cfg, target, rec, topk_in, topk_out, grad, rendered, grad_img, state):
    """Rows a3-a6 of one iteration as one kernel (sad_train_image_pass)."""
    P = img.H * img.W
    _check(lib.sad_train_image_pass(C.byref(img), C.byref(cfg), _ptr(target, torch.float32, 3 * P, "target"),
                                    _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                                    _ptr(topk_in, torch.int32, img.K * P, "topk_in"),
                                    _ptr(topk_out, torch.int32, img.K * P, "topk_out"),
                                    _ptr(grad, _grad_dtype(cfg), NPARAM * img.cap, "grad"),
                                    _ptr(rendered, torch.float32, 3 * P, "rendered"),
                                    _ptr(grad_img, torch.float32, 3 * P, "grad_img"),
                                    _ptr(state, torch.int64, STEP_STATE_INT64, "state"), _stream()),
           "sad_train_image_pass")


GRAD_CLEAR_SOURCE = 1


def grad_to_params(img, grad_site_major, grad, scale=None, clear=False):
    """grad [10][cap] = scale * transpose(grad_site_major [cap][10]) (sad_grad_to_params);
    scale: a device float tensor or None; clear zeroes the source."""
    n = NPARAM * img.cap
    _check(lib.sad_grad_to_params(C.byref(img), _ptr(grad_site_major, torch.float32, n, "grad_site_major"),
                                  _ptr(scale, torch.float32, 1, "scale"),
                                  _ptr(grad, torch.float32, n, "grad"),
                                  GRAD_CLEAR_SOURCE if clear else 0, _stream()),
           "sad_grad_to_params")


def batch_train_step(batch, cfg, target, sites, rec, topk_in, topk_out, grad, m, v, rendered,
                     grad_img, states):
    """One iteration of every image of a batch (sad_batch_train_step).  Buffers are the
    pooled tensors; states: int64 tensor of n_images sad_step_state records."""
    n = NPARAM * batch.n_site_slots
    _check(lib.sad_batch_train_step(C.byref(batch), C.byref(cfg), _ptr(target, torch.float32, None, "target"),
                                    _ptr(sites, torch.float32, n, "sites"),
                                    _ptr(rec, torch.float32, REC_FLOATS * batch.n_site_slots, "rec"),
                                    _ptr(topk_in, torch.int32, None, "topk_in"),
                                    _ptr(topk_out, torch.int32, None, "topk_out"),
                                    _ptr(grad, _grad_dtype(cfg), n, "grad"), _ptr(m, torch.float32, n, "m"),
                                    _ptr(v, torch.float32, n, "v"),
                                    _ptr(rendered, torch.float32, None, "rendered"),
                                    _ptr(grad_img, torch.float32, None, "grad_img"),
                                    _ptr(states, torch.int64, STEP_STATE_INT64 * batch.n_images, "states"),
                                    _stream()),
           "sad_batch_train_step")


def query_batch(jobs_dev, n_jobs, total, K):
    """Point queries of many jobs (sad_query_batch); jobs_dev: device uint8 tensor holding
    n_jobs SadQueryJob records."""
    _check(lib.sad_query_batch(C.c_void_p(jobs_dev.data_ptr()), int(n_jobs), int(total), int(K),
                               _stream()),
           "sad_query_batch")


# ---- full-refresh regime: list fields on a grid of cells (sad_seed_grid ... sad_render_grid)

REFRESH_JFA = 1


def _scratch_ptr(scratch, n_bytes, name):
    if scratch.numel() * scratch.element_size() < n_bytes:
        raise ValueError(f"{name}: scratch needs {n_bytes} bytes")
    return _ptr(scratch, scratch.dtype, None, "scratch")


def seed_grid(img, Hg, Wg, n_entries, rec, topk, scratch):
    """Seed pass on an Hg x Wg grid keeping n_entries per cell (sad_seed_grid)."""
    Pg = int(Hg) * int(Wg)
    _check(lib.sad_seed_grid(C.byref(img), int(Hg), int(Wg), int(n_entries),
                             _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                             _ptr(topk, torch.int32, img.K * Pg, "topk"),
                             _scratch_ptr(scratch, 8 * Pg, "seed_grid"), _stream()),
           "sad_seed_grid")


def propagate_grid(img, Hg, Wg, rec, topk_in, topk_out, jump, n_inject, seed, pass_index):
    """One propagation pass on an Hg x Wg grid (sad_propagate_grid)."""
    Pg = int(Hg) * int(Wg)
    _check(lib.sad_propagate_grid(C.byref(img), int(Hg), int(Wg),
                                  _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                                  _ptr(topk_in, torch.int32, img.K * Pg, "topk_in"),
                                  _ptr(topk_out, torch.int32, img.K * Pg, "topk_out"),
                                  int(jump), int(n_inject), int(seed) & (2 ** 64 - 1),
                                  int(pass_index), _stream()),
           "sad_propagate_grid")


def jfa_flood(img, Hg, Wg, rec, topk_in, topk_out, step):
    """One JFA flood pass on plane 0 of an Hg x Wg list field (sad_jfa_flood)."""
    Pg = int(Hg) * int(Wg)
    _check(lib.sad_jfa_flood(C.byref(img), int(Hg), int(Wg),
                             _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                             _ptr(topk_in, torch.int32, 4 * Pg, "topk_in"),
                             _ptr(topk_out, torch.int32, 4 * Pg, "topk_out"), int(step), _stream()),
           "sad_jfa_flood")


def jfa_steps(Hg, Wg):
    buf = (C.c_int32 * 32)()
    n = int(lib.sad_jfa_steps(int(Hg), int(Wg), buf))
    if n < 0:
        raise SadError("sad_jfa_steps: bad grid")
    return [int(buf[k]) for k in range(n)]


def refresh(img, Hg, Wg, rec, topk, topk_tmp, scratch, n_pass, n_inject, seed, jfa=True):
    """Full refresh of an Hg x Wg list field (sad_refresh): JFA prepass (or seed pass),
    then n_pass propagation passes; the result is in topk."""
    Pg = int(Hg) * int(Wg)
    _check(lib.sad_refresh(C.byref(img), int(Hg), int(Wg), REFRESH_JFA if jfa else 0, int(n_pass),
                           int(n_inject), int(seed) & (2 ** 64 - 1),
                           _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                           _ptr(topk, torch.int32, img.K * Pg, "topk"),
                           _ptr(topk_tmp, torch.int32, img.K * Pg, "topk_tmp"),
                           _scratch_ptr(scratch, 8 * Pg, "refresh"), _stream()),
           "sad_refresh")


def render_grid(img, Hg, Wg, rec, topk, Ho, Wo, out):
    """Render an Ho x Wo output grid from an Hg x Wg list field (sad_render_grid)."""
    _check(lib.sad_render_grid(C.byref(img), int(Hg), int(Wg),
                               _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                               _ptr(topk, torch.int32, img.K * int(Hg) * int(Wg), "topk"),
                               int(Ho), int(Wo), _ptr(out, torch.float32, 3 * int(Ho) * int(Wo), "out"),
                               _stream()),
           "sad_render_grid")


# ---- packed 16-byte inference record (sad_pack_qparams ... sad_query_packed)

NQPARAM = 10


def pack_qparams(img, sites, q):
    """Per-image quantisation parameters q [10] (device float32) from sites."""
    _check(lib.sad_pack_qparams(C.byref(img), _ptr(sites, torch.float32, NPARAM * img.cap, "sites"),
                                _ptr(q, torch.float32, NQPARAM, "q"), _stream()),
           "sad_pack_qparams")


def pack_sites(img, sites, q, packed):
    """packed [n_slots, 4] int32 (the uint32 words) from sites with parameters q."""
    _check(lib.sad_pack_sites(C.byref(img), _ptr(sites, torch.float32, NPARAM * img.cap, "sites"),
                              _ptr(q, torch.float32, NQPARAM, "q"),
                              _ptr(packed, torch.int32, 4 * img.n_slots, "packed"), _stream()),
           "sad_pack_sites")


def unpack_sites(img, packed, q, sites):
    _check(lib.sad_unpack_sites(C.byref(img), _ptr(packed, torch.int32, 4 * img.n_slots, "packed"),
                                _ptr(q, torch.float32, NQPARAM, "q"),
                                _ptr(sites, torch.float32, NPARAM * img.cap, "sites"), _stream()),
           "sad_unpack_sites")


def prepare_packed(img, packed, q, rec):
    _check(lib.sad_prepare_packed(C.byref(img), _ptr(packed, torch.int32, 4 * img.n_slots, "packed"),
                                  _ptr(q, torch.float32, NQPARAM, "q"),
                                  _ptr(rec, torch.float32, REC_FLOATS * img.n_slots, "rec"),
                                  _stream()),
           "sad_prepare_packed")


def render_packed(img, packed, q, topk, out):
    P = img.H * img.W
    _check(lib.sad_render_packed(C.byref(img), _ptr(packed, torch.int32, 4 * img.n_slots, "packed"),
                                 _ptr(q, torch.float32, NQPARAM, "q"),
                                 _ptr(topk, torch.int32, img.K * P, "topk"),
                                 _ptr(out, torch.float32, 3 * P, "out"), _stream()),
           "sad_render_packed")


def query_packed(img, packed, q, topk, xy, out):
    M = xy.shape[0] if xy.dim() == 2 else xy.numel() // 2
    P = img.H * img.W
    _check(lib.sad_query_packed(C.byref(img), _ptr(packed, torch.int32, 4 * img.n_slots, "packed"),
                                _ptr(q, torch.float32, NQPARAM, "q"),
                                _ptr(topk, torch.int32, img.K * P, "topk"),
                                _ptr(xy, torch.float32, 2 * M, "xy"), int(M),
                                _ptr(out, torch.float32, 3 * M, "out"), _stream()),
           "sad_query_packed")


def bpp(n_sites, H, W):
    """Bits per pixel of n_sites packed 16-byte records over an H x W image (Sec. 6.1)."""
    return n_sites * 16 * 8 / (H * W)


# ---- tau diffusion and the one-dimensional SAD (sad_tau_diffusion, sad1d_*)


def tau_diffusion(img, rec, topk, g_in, in_stride, lam, g_out, out_stride):
    """One Jacobi step of the log tau gradient smoothing (sad_tau_diffusion); g_in, g_out
    are float32 views whose element i sits at i * stride."""
    n = img.n_slots
    need_in = (n - 1) * int(in_stride) + 1 if n else 0
    need_out = (n - 1) * int(out_stride) + 1 if n else 0
    _check(lib.sad_tau_diffusion(C.byref(img), _ptr(rec, torch.float32, REC_FLOATS * n, "rec"),
                                 _ptr(topk, torch.int32, img.K * img.H * img.W, "topk"),
                                 _ptr(g_in, torch.float32, need_in, "g_in"), int(in_stride),
                                 float(lam), _ptr(g_out, torch.float32, need_out, "g_out"),
                                 int(out_stride), _stream()),
           "sad_tau_diffusion")


def signal(M, K, n_slots, cap=None, score_scale=0.0):
    """Descriptor of a one-dimensional signal (sad_signal)."""
    return SadSignal(int(M), int(K), int(n_slots), 0, int(cap if cap is not None else n_slots),
                     float(score_scale))


def prepare1d(sg, sites, rec1):
    _check(lib.sad1d_prepare(C.byref(sg), _ptr(sites, torch.float32, 4 * sg.cap, "sites"),
                             _ptr(rec1, torch.float32, 4 * sg.n_slots, "rec1"), _stream()),
           "sad1d_prepare")


def seed1d(sg, rec1, topk, scratch):
    if scratch.numel() * scratch.element_size() < 8 * sg.M:
        raise ValueError("seed1d: scratch needs 8 bytes per sample")
    _check(lib.sad1d_seed(C.byref(sg), _ptr(rec1, torch.float32, 4 * sg.n_slots, "rec1"),
                          _ptr(topk, torch.int32, sg.K * sg.M, "topk"),
                          _ptr(scratch, scratch.dtype, None, "scratch"), _stream()),
           "sad1d_seed")


def propagate1d(sg, rec1, topk_in, topk_out, jump, n_inject, seed, pass_index):
    _check(lib.sad1d_propagate(C.byref(sg), _ptr(rec1, torch.float32, 4 * sg.n_slots, "rec1"),
                               _ptr(topk_in, torch.int32, sg.K * sg.M, "topk_in"),
                               _ptr(topk_out, torch.int32, sg.K * sg.M, "topk_out"), int(jump),
                               int(n_inject), int(seed) & (2 ** 64 - 1), int(pass_index),
                               _stream()),
           "sad1d_propagate")


def render1d(sg, rec1, topk, target=None, out=None, grad=None, loss=None):
    _check(lib.sad1d_render(C.byref(sg), _ptr(rec1, torch.float32, 4 * sg.n_slots, "rec1"),
                            _ptr(topk, torch.int32, sg.K * sg.M, "topk"),
                            _ptr(target, torch.float32, sg.M, "target"),
                            _ptr(out, torch.float32, sg.M, "out"),
                            _ptr(grad, torch.float32, 4 * sg.cap, "grad"),
                            _ptr(loss, torch.float32, LOSS_ACC_FLOATS, "loss"), _stream()),
           "sad1d_render")


def adam1d(sg, sites, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    n = 4 * sg.cap
    lr4 = (C.c_float * 4)(*[float(x) for x in lr])
    _check(lib.sad1d_adam(C.byref(sg), _ptr(sites, torch.float32, n, "sites"),
                          _ptr(grad, torch.float32, n, "grad"), _ptr(m, torch.float32, n, "m"),
                          _ptr(v, torch.float32, n, "v"), lr4, float(beta1), float(beta2),
                          float(eps), int(step), _stream()),
           "sad1d_adam")
