"""C ABI checks that need no GPU: the library loads, exports every symbol
that include/ta.h declares, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

LIB = os.path.join(ROOT, "paper_2502_10831_amd", "libta.so")
HEADER = os.path.join(ROOT, "include", "ta.h")

OK, EINVAL, EDTYPE, EOVERLAP, EHIP = range(5)
F32, F16, BF16, F64 = range(4)
A, B = 0x100000, 0x200000   # fake device addresses: never dereferenced


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libta.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:ta_status|const char \*|int)\s*(ta_\w+)\(",
                                 text, re.M)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 21
    for name in names:
        assert hasattr(lib, name), name


def _fn(lib, name, *argtypes):
    f = getattr(lib, name)
    f.argtypes = list(argtypes)
    f.restype = ctypes.c_int
    return f


vp, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32


def test_unary_validation(lib):
    for name in ("ta_sin", "ta_cos", "ta_tan"):
        f = _fn(lib, name, vp, vp, i64, i32, vp)
        assert f(A, B, 16, 7, None) == EDTYPE
        assert f(A, B, -1, F32, None) == EINVAL
        assert f(None, B, 16, F32, None) == EINVAL
        assert f(A, None, 16, F32, None) == EINVAL
        assert f(A, A + 4, 16, F32, None) == EOVERLAP     # partial overlap
        assert f(None, None, 0, F32, None) == OK          # n == 0: no launch
        assert f(A, A - 2, 8, BF16, None) == EOVERLAP


def test_sincos_validation(lib):
    f = _fn(lib, "ta_sincos_ex", vp, vp, vp, vp, i64, i32, vp, u32)
    assert f(A, B, None, None, 16, F32, None, 0) == EINVAL    # yc required
    # FP32 reduction: not for FP64 storage, not with the FP64 flag
    assert f(A, B, B + 128, None, 16, F64, None, 4) == EINVAL
    assert f(A, B, B + 32, None, 16, F32, None, 6) == EINVAL
    assert f(A, B, B + 32, None, 16, F32, None, 8) == EINVAL  # paper-only flag
    assert f(A, B, B + 32, None, 16, F32, None, 16) == EINVAL  # unknown
    assert f(A, B, B + 32, B + 16, 16, F32, None, 0) == EOVERLAP
    assert f(A, B, B, None, 16, F32, None, 0) == EOVERLAP     # ys == yc
    assert f(A, B, B + 64, B + 128, 16, 4, None, 0) == EDTYPE
    # FP64 elements are 8 bytes: 16 of them end at +128
    assert f(A, B, B + 64, None, 16, F64, None, 0) == EOVERLAP
    assert f(A, B, B + 64, None, 0, F32, None, 0) == OK
    for name in ("ta_sin_ex", "ta_cos_ex", "ta_tan_ex"):
        g = _fn(lib, name, vp, vp, i64, i32, vp, u32)
        assert g(A, B, 16, F64, None, 4) == EINVAL, name
        assert g(A, B, 16, F32, None, 6) == EINVAL, name
        assert g(A, B, 16, F32, None, 8) == EINVAL, name
        assert g(A, B, 16, F32, None, 16) == EINVAL, name
        assert g(A, B, 16, 7, None, 0) == EDTYPE, name
        assert g(A, A + 4, 16, F32, None, 4) == EOVERLAP, name
        assert g(None, None, 0, F32, None, 4) == OK, name


def test_taylor_validation(lib):
    for name in ("ta_taylor_sin", "ta_taylor_cos", "ta_taylor_tan"):
        f = _fn(lib, name, vp, vp, i64, i32, i32, vp)
        for bad in (0, 3, 4, 6, 8, 11):
            assert f(A, B, 16, bad, F32, None) == EINVAL
        assert f(A, B, 16, 5, 9, None) == EDTYPE
        assert f(A, B, 0, 7, F32, None) == OK


def test_backward_validation(lib):
    for name in ("ta_sin_bwd", "ta_cos_bwd", "ta_tan_bwd"):
        f = _fn(lib, name, vp, vp, vp, i64, i32, vp)
        assert f(A, None, B, 16, F32, None) == EINVAL
        assert f(A, B, A + 8, 16, F32, None) == EOVERLAP
        assert f(A, B, B + 4, 16, F32, None) == EOVERLAP
        assert f(A, B, B + 64, 16, F64, None) == EOVERLAP
        assert f(A, B, None, 0, F32, None) == OK
    f = _fn(lib, "ta_sincos_bwd", vp, vp, vp, vp, i64, i32, vp)
    assert f(A, None, None, B, 16, F32, None) == EINVAL      # no gradient
    assert f(A, None, None, B, 0, F32, None) == OK
    assert f(A, B, None, None, 16, F32, None) == EINVAL
    for name in ("ta_sin_fwdbwd", "ta_cos_fwdbwd", "ta_tan_fwdbwd"):
        f = _fn(lib, name, vp, vp, vp, vp, i64, i32, vp)
        assert f(A, B, None, B + 512, 16, F32, None) == EINVAL
        assert f(A, B, B + 512, B + 520, 16, F32, None) == EOVERLAP
        assert f(A, B, B + 512, B + 1024, 16, 5, None) == EDTYPE


def test_paper_validation(lib):
    f = _fn(lib, "ta_paper_sincos", vp, vp, vp, vp, i64, i32, vp, u32)
    assert f(A, None, None, None, 16, F32, None, 0) == EINVAL   # no output
    assert f(A, None, None, None, 0, F32, None, 0) == OK
    assert f(A, B, None, None, 16, F32, None, 4) == EINVAL      # bad flag
    assert f(A, B, None, None, 16, F32, None, 16) == EINVAL
    assert f(A, B, None, None, 16, 5, None, 0) == EDTYPE
    assert f(A, B, B + 8, None, 16, F32, None, 3) == EOVERLAP
    assert f(None, B, None, None, 16, F32, None, 0) == EINVAL


def test_encode_validation(lib):
    f = _fn(lib, "ta_sincos_encode", vp, vp, i64, i32, i32, vp)
    for bad in (0, 17, -1):
        assert f(A, B, 16, bad, F32, None) == EINVAL
    assert f(A, B, -1, 4, F32, None) == EINVAL
    assert f(A, B, 16, 4, 7, None) == EDTYPE
    assert f(None, B, 16, 4, F32, None) == EINVAL
    assert f(A, None, 16, 4, F32, None) == EINVAL
    assert f(A, A + 32, 16, 4, F32, None) == EOVERLAP   # y starts inside x
    assert f(B + 8, B, 16, 4, F32, None) == EOVERLAP    # x inside y's planes
    assert f(A, B, 0, 4, F32, None) == OK


def test_comparator_validation(lib):
    f = _fn(lib, "ta_builtin_sincos", vp, vp, vp, vp, i64, i32, i32, vp)
    assert f(A, B, B + 256, None, 16, 0, 7, None) == EDTYPE
    assert f(A, B, B + 256, None, 16, 3, F32, None) == EINVAL
    assert f(A, B, B + 256, None, 16, -1, F16, None) == EINVAL
    # no FP64 hardware approximations: kind 1 is not available for FP64
    assert f(A, B, B + 256, None, 16, 1, F64, None) == EDTYPE
    # outputs: ys, ys + yc or ys + yc + yt
    assert f(A, None, B, None, 16, 0, F32, None) == EINVAL
    assert f(A, B, None, B + 512, 16, 0, BF16, None) == EINVAL
    assert f(A, None, None, None, 0, 0, F32, None) == OK
    assert f(A, B, None, None, -1, 0, F32, None) == EINVAL
    assert f(A, A + 4, None, None, 16, 0, F32, None) == EOVERLAP
    fb = _fn(lib, "ta_builtin_sin_fwdbwd", vp, vp, vp, vp, i64, i32, i32, vp)
    assert fb(A, B, B + 256, B + 512, 16, 2, F32, None) == EINVAL
    assert fb(A, B, B + 256, B + 512, 16, 1, F64, None) == EDTYPE
    assert fb(A, B, B + 256, B + 512, 16, 0, 9, None) == EDTYPE
    assert fb(A, None, B + 256, B + 512, 16, 0, F32, None) == EINVAL
    assert fb(A, B, B + 256, B + 256, 16, 0, F32, None) == EOVERLAP
    assert fb(A, B, B + 256, B + 512, 0, 0, F32, None) == OK


def test_stream_probe_validation(lib):
    f = _fn(lib, "ta_stream_probe", i32, vp, ctypes.POINTER(vp), i32, i64,
            u32, vp)
    outs = (vp * 3)(B, B + 0x10000, B + 0x20000)
    assert f(3, A, outs, 1, 16, 0, None) == EINVAL          # unknown kind
    assert f(0, A, outs, 2, 16, 0, None) == EINVAL          # read: one sink
    assert f(1, A, outs, 0, 16, 0, None) == EINVAL
    assert f(2, A, outs, 4, 16, 0, None) == EINVAL
    assert f(2, A, outs, 1, 18, 0, None) == EINVAL          # n % 4
    assert f(2, A + 4, outs, 1, 16, 0, None) == EINVAL      # alignment
    assert f(1, None, outs, 3, 16, 16, None) == EINVAL      # unknown flag
    assert f(1, None, outs, 3, 16, 8, None) == EINVAL       # scope w/o nt
    assert f(2, A, outs, 1, -4, 0, None) == EINVAL
    assert f(2, None, outs, 1, 16, 0, None) == EINVAL       # copy needs x
    assert f(2, B + 16, outs, 1, 16, 0, None) == EOVERLAP
    same = (vp * 2)(B, B + 32)
    assert f(1, None, same, 2, 16, 0, None) == EOVERLAP
    sink = (vp * 1)(A + 1024)
    assert f(0, A, sink, 1, 1024, 0, None) == EOVERLAP      # sink in x
    assert f(2, A, outs, 3, 0, 7, None) == OK
    c = _fn(lib, "ta_copy", ctypes.POINTER(vp), i32, ctypes.POINTER(vp), i32,
            i64, i32, vp)
    ins = (vp * 1)(A)
    outs = (vp * 4)(B, B + 256, B + 512, B + 768)
    assert c(ins, 0, outs, 1, 16, F32, None) == EINVAL
    assert c(ins, 1, outs, 4, 16, F32, None) == EINVAL
    assert c(ins, 1, outs, 1, 16, 9, None) == EDTYPE


def test_status_strings(lib):
    lib.ta_status_str.restype = ctypes.c_char_p
    lib.ta_status_str.argtypes = [ctypes.c_int]
    for s in range(5):
        assert lib.ta_status_str(s).startswith(b"TA_")
    lib.ta_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.ta_version()
    lib.ta_last_hip_error.restype = ctypes.c_int
    assert lib.ta_last_hip_error() == 0


def test_binding_refuses_cpu_tensors():
    """The Python layer has no CPU path: host tensors raise before any
    library call."""
    torch = pytest.importorskip("torch")
    import paper_2502_10831_amd as ta
    x = torch.zeros(8)
    for fn in (ta.sin, ta.cos, ta.tan, ta.sincos):
        with pytest.raises(ta.TaError):
            fn(x)
    with pytest.raises(ta.TaError):
        ta.SinFn.apply(x)


def test_c_example_links_against_the_header_and_library():
    """tests/c_abi/ta_example is plain C (C99, -Werror) compiled against
    include/ta.h and linked to libta.so; without arguments it prints its
    usage and exits 2 before any HIP call."""
    import subprocess
    exe = os.path.join(ROOT, "tests", "c_abi", "ta_example")
    if not os.path.exists(exe):
        pytest.fail("tests/c_abi/ta_example is not built "
                    "(run __graft_entry__.build())")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr
