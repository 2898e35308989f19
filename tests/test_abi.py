"""CPU checks of the C ABI: the library loads, exports every function that
include/bmpl.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bmpl.h")
LIB = os.path.join(ROOT, "paper_1302_5010_amd", "libbmpl.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bmpl_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libbmpl.so is not built; run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert {"bmpl_create", "bmpl_solve", "bmpl_destroy", "bmpl_options_default", "bmpl_last_error"} <= set(names)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in bmpl.h but not exported"


def test_options_default(lib):
    from paper_1302_5010_amd._binding import _Options
    o = _Options()
    assert lib.bmpl_options_default(ctypes.byref(o)) == 0
    assert o.rho == 10 and o.max_outer == 0 and o.max_active == 0 and o.kkt_tol == 1e-4 and o.screen == 0
    assert o.omega == 1 and o.flags == 0
    assert o.eps_early == 0.0 and o.r_inf_rel == 0.0 and o.r2_rel == 0.0
    assert lib.bmpl_options_default(None) == -1


def test_argument_errors_without_gpu(lib):
    lib.bmpl_last_error.restype = ctypes.c_char_p
    lib.bmpl_last_error.argtypes = [ctypes.c_void_p]
    vp = ctypes.c_void_p
    lib.bmpl_create.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.c_double,
                                vp, vp, ctypes.POINTER(vp)]
    h = vp()
    fake = ctypes.c_void_p(0x1000)
    assert lib.bmpl_create(None, 4, 4, 4, 0, 0.1, None, None, ctypes.byref(h)) == -1
    assert b"NULL A" in lib.bmpl_last_error(None)
    assert lib.bmpl_create(fake, 2, 4, 4, 0, 0.1, None, None, ctypes.byref(h)) == -1     # lda < n
    assert lib.bmpl_create(fake, 4, 4, 0, 0, 0.1, None, None, ctypes.byref(h)) == -1     # m = 0
    assert lib.bmpl_create(fake, 4, 4, 4, 0, -1.0, None, None, ctypes.byref(h)) == -1    # lambda < 0
    assert lib.bmpl_create(fake, 4, 4, 4, 0, float("nan"), None, None, ctypes.byref(h)) == -1
    assert lib.bmpl_create(fake, 4, 4, 4, 7, 0.1, None, None, ctypes.byref(h)) == -1     # bad mode
    from paper_1302_5010_amd._binding import _Options
    o = _Options()
    lib.bmpl_options_default(ctypes.byref(o))
    o.rho = 0
    assert lib.bmpl_create(fake, 4, 4, 4, 0, 0.1, ctypes.byref(o), None, ctypes.byref(h)) == -1
    o.rho, o.omega = 10, 0
    assert lib.bmpl_create(fake, 4, 4, 4, 0, 0.1, ctypes.byref(o), None, ctypes.byref(h)) == -1
    o.omega = 7                                  # omega * rho > 64
    assert lib.bmpl_create(fake, 4, 4, 4, 0, 0.1, ctypes.byref(o), None, ctypes.byref(h)) == -1
    o.omega = 1
    for field in ("eps_early", "r_inf_rel", "r2_rel"):   # early-stop tolerances: finite, >= 0
        for bad in (-1e-3, float("nan"), float("inf")):
            setattr(o, field, bad)
            assert lib.bmpl_create(fake, 4, 4, 4, 0, 0.1, ctypes.byref(o), None, ctypes.byref(h)) == -1
            assert b"eps_early" in lib.bmpl_last_error(None)
        setattr(o, field, 0.0)
    o.screen = 9
    assert lib.bmpl_create(fake, 4, 4, 4, 0, 0.1, ctypes.byref(o), None, ctypes.byref(h)) == -4
    assert h.value is None
    assert lib.bmpl_solve(None, None, 4, 1, None, None, 0, None, None) == -1
    assert lib.bmpl_destroy(None) == 0
    assert lib.bmpl_get_timing(None, None) == -1
    assert lib.bmpl_correlate(None, None, 4, 1, None, 4, None) == -1


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_1302_5010_amd._binding as b
    monkeypatch.setattr(b, "_LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        b._load()


def test_proposal_argument_errors_without_gpu(lib):
    lib.bmpl_last_error.restype = ctypes.c_char_p
    lib.bmpl_last_error.argtypes = [ctypes.c_void_p]
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.bmpl_mlp_param_count.restype = i64
    lib.bmpl_mlp_param_count.argtypes = [i32, i32, i32]
    assert lib.bmpl_mlp_param_count(2048, 2048, 20000) == 2048 * 2048 * 2 + 2048 * 2 + 20000 * 2048 + 20000
    assert lib.bmpl_mlp_param_count(0, 64, 10) == 0
    lib.bmpl_mlp_create.argtypes = [vp, i64, i32, i32, vp, i32, i32, i32, vp, ctypes.POINTER(vp)]
    h = vp()
    fake = ctypes.c_void_p(0x1000)
    assert lib.bmpl_mlp_create(None, 4, 4, 4, fake, 64, 64, 8, None, ctypes.byref(h)) == -1
    assert b"NULL A or P" in lib.bmpl_last_error(None)
    assert lib.bmpl_mlp_create(fake, 4, 4, 4, fake, 100, 64, 8, None, ctypes.byref(h)) == -1   # d_in % 64
    assert lib.bmpl_mlp_create(fake, 4, 4, 4, fake, 64, 0, 8, None, ctypes.byref(h)) == -1    # d_hidden
    assert lib.bmpl_mlp_create(fake, 4, 4, 40000, fake, 64, 64, 8, None, ctypes.byref(h)) == -1   # m too wide
    assert b"exceeds" in lib.bmpl_last_error(None)
    assert lib.bmpl_mlp_create(fake, 2, 4, 4, fake, 64, 64, 8, None, ctypes.byref(h)) == -1   # lda < n
    assert h.value is None
    assert lib.bmpl_mlp_destroy(None) == 0
    lib.bmpl_mlp_forward.argtypes = [vp, vp, i64, i32, vp, i64, vp]
    assert lib.bmpl_mlp_forward(None, fake, 4, 1, fake, 4, None) == -1
    lib.bmpl_topk.argtypes = [vp, i64, i32, i32, i32, vp, i32, vp]
    assert lib.bmpl_topk(fake, 10, 1, 10, 0, fake, 4, None) == -1       # k = 0
    assert lib.bmpl_topk(fake, 10, 1, 10, 257, fake, 300, None) == -1   # k > 256
    assert lib.bmpl_topk(fake, 10, 1, 10, 8, fake, 4, None) == -1       # ld_idx < k
    assert lib.bmpl_topk(fake, 50000, 1, 50000, 8, fake, 8, None) == -1  # row too long
    lib.bmpl_mlp_adam_step.argtypes = [vp, vp, vp, vp]
    assert lib.bmpl_mlp_adam_step(None, None, None, None) == -1


def test_classify_argument_errors_without_gpu(lib):
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.bmpl_classify.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp, vp]
    assert lib.bmpl_classify(None, None, 4, 1, None, None, None, None, None) == -1
