"""The C ABI library loads on a machine without a GPU, exports every entry point that
include/sad.h declares, and rejects bad arguments on the host before enqueueing."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sad.h")
LIB = os.path.join(ROOT, "paper_2604_21984_amd", "libsad.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sad_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


class Img(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("K", C.c_int32), ("n_slots", C.c_int32),
                ("cap", C.c_int64), ("score_scale", C.c_float)]


def test_host_validation_without_device(lib):
    lib.sad_last_error.restype = C.c_char_p
    lib.sad_status_string.restype = C.c_char_p
    bad_k = Img(8, 8, 6, 4, 4, 0.0)
    assert lib.sad_render_fwd(C.byref(bad_k), None, None, None, None) == 2
    assert b"K = 6" in lib.sad_last_error()
    bad_hw = Img(0, 8, 8, 4, 4, 0.0)
    assert lib.sad_prepare_sites(C.byref(bad_hw), None, None, None) == 1
    bad_cap = Img(8, 8, 8, 5, 4, 0.0)
    assert lib.sad_render_bwd(C.byref(bad_cap), None, None, None, None, None, None, None) == 1
    ok = Img(8, 8, 8, 4, 4, 0.0)
    # aliasing in/out lists is refused (Jacobi pass)
    buf = (C.c_uint32 * 1024)()
    p = C.cast(buf, C.c_void_p)
    assert lib.sad_propagate_topk(C.byref(ok), p, p, p, C.c_int32(1), C.c_int32(4),
                                  C.c_uint64(0), C.c_uint64(0), None) == 1
    lib.sad_jump_step.restype = C.c_int32
    lib.sad_jump_step.argtypes = [C.c_int64, C.c_int32, C.c_int32]
    assert [lib.sad_jump_step(t, 512, 768) for t in range(11)] == [512, 256, 128, 64, 32, 16, 8, 4, 2, 1, 1]
    n = C.c_size_t(0)
    assert lib.sad_init_sites(C.byref(ok), None, 0, C.c_float(0), C.c_uint64(0), C.c_float(0),
                              C.c_float(0), None, None, C.byref(n), None) == 0
    assert n.value >= 8 * 64
    assert lib.sad_status_string(3) == b"workspace too small"


def test_host_validation_of_state_forms_and_flags(lib):
    """The device-counter entry points and the training / Adam flags are checked on the
    host before anything is enqueued (no device is touched)."""
    from paper_2604_21984_amd import _lib as S
    ok = Img(8, 8, 8, 4, 4, 0.0)
    buf = (C.c_uint32 * 4096)()
    base = (C.addressof(buf) + 15) & ~15
    p, q = C.c_void_p(base), C.c_void_p(base + 4096)
    # propagation from a state: NULL state, aliasing lists
    assert lib.sad_propagate_topk_state(C.byref(ok), p, p, q, C.c_int32(4), C.c_uint64(0),
                                        None, None) == 1
    assert lib.sad_propagate_topk_state(C.byref(ok), p, p, p, C.c_int32(4), C.c_uint64(0),
                                        p, None) == 1
    # Adam: unknown flag bits, NULL state
    params = S.adam_params([1e-3] * 10, 0.9, 0.999, 1e-8)
    assert lib.sad_adam_step(C.byref(ok), p, p, p, p, C.byref(params), C.c_int64(1), None,
                             C.c_uint32(8), None) == 1
    assert b"unknown flags" in lib.sad_last_error()
    assert lib.sad_adam_step_state(C.byref(ok), p, p, p, p, C.byref(params), None,
                                   C.c_uint32(0), None, None) == 1
    # training pass: unknown training flags
    cfg = S.train_config(4, 0, params)
    cfg.flags = 4
    assert lib.sad_train_image_pass(C.byref(ok), C.byref(cfg), p, p, p, q, p, None, None, p,
                                    None) == 1
    assert b"unknown flags" in lib.sad_last_error()
    # fixed-point statistics: NULL or misaligned workspace
    assert lib.sad_site_stats_fixed(C.byref(ok), p, p, p, None, p, None) == 1
    assert lib.sad_site_stats_fixed(C.byref(ok), p, p, p, C.c_void_p(base + 4), p, None) == 1
    assert b"8-byte aligned" in lib.sad_last_error()
    assert S.train_config(4, 0, params, deterministic=True).flags == S.TRAIN_DETERMINISTIC
    assert S.train_config(4, 0, params).flags == 0
    assert S.train_config(4, 0, params, loss_set=True).flags == S.TRAIN_LOSS_SET == 2
