"""MI355X (gfx950) piecewise trigonometric approximations of Goyal & Arora,
arXiv 2502.10831: a thin Python binding over the C ABI of ``libta.so``.

Layers:
  * ``ta_*`` functions: the C entry points under the same names.  Argument
    marshalling only (device pointers, element count, dtype code, the current
    HIP stream); every step of the computation runs in the HIP kernels.
  * ``sin``, ``cos``, ``tan``, ``sincos`` ...: allocate outputs and call the
    entry points.
  * ``SinFn``/``CosFn``/``TanFn``/``SinCosFn``: ``torch.autograd.Function``
    front ends whose backward is the hand-written derivative kernel.

PyTorch is used for device memory and streams only.  There is no CPU path:
tensors must live on a HIP device and ``libta.so`` must be built (see
``__graft_entry__.build``); otherwise these functions raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "TaError", "lib_path", "load",
    "ta_sin", "ta_cos", "ta_tan", "ta_tan_ex", "ta_sincos", "ta_sincos_ex",
    "ta_taylor_sin", "ta_taylor_cos", "ta_taylor_tan",
    "ta_sin_bwd", "ta_cos_bwd", "ta_tan_bwd", "ta_sincos_bwd",
    "ta_sin_fwdbwd", "ta_cos_fwdbwd", "ta_tan_fwdbwd",
    "ta_paper_sincos", "ta_sincos_encode", "ta_builtin_sincos",
    "ta_builtin_sin_fwdbwd", "ta_copy", "ta_stream_probe",
    "TA_PROBE_NT_LOAD", "TA_PROBE_NT_STORE", "TA_PROBE_BLOCK256",
    "TA_PROBE_DEVICE_SCOPE",
    "sin", "cos", "tan", "sincos", "taylor",
    "SinFn", "CosFn", "TanFn", "SinCosFn",
    "TA_FLAG_TAN_GUARD", "TA_FLAG_LITERAL_DIVISOR",
    "TA_FLAG_FORCE_FP64_REDUCTION", "TA_FLAG_FORCE_FP32_REDUCTION",
    "ta_sin_ex", "ta_cos_ex", "paper_sincos", "encode",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libta.so")

TA_F32, TA_F16, TA_BF16, TA_F64 = 0, 1, 2, 3
TA_FLAG_TAN_GUARD = 1
TA_FLAG_FORCE_FP64_REDUCTION = 2
TA_FLAG_FORCE_FP32_REDUCTION = 4
TA_FLAG_LITERAL_DIVISOR = 8
TA_PROBE_NT_LOAD, TA_PROBE_NT_STORE, TA_PROBE_BLOCK256 = 1, 2, 4
TA_PROBE_DEVICE_SCOPE = 8
_DTYPE_CODE = {torch.float32: TA_F32, torch.float16: TA_F16,
               torch.bfloat16: TA_BF16, torch.float64: TA_F64}

_lib = None


class TaError(RuntimeError):
    """A libta entry point returned a non-OK status."""


def lib_path() -> str:
    return _LIB


def load(path: str | None = None):
    """Load libta.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or _LIB
    if not os.path.exists(path):
        raise TaError(f"{path} is missing: build it first "
                      "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    vp, i64, i32, u32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                         ctypes.c_uint32)
    sigs = {
        "ta_sin": [vp, vp, i64, i32, vp],
        "ta_cos": [vp, vp, i64, i32, vp],
        "ta_tan": [vp, vp, i64, i32, vp],
        "ta_tan_ex": [vp, vp, i64, i32, vp, u32],
        "ta_sin_ex": [vp, vp, i64, i32, vp, u32],
        "ta_cos_ex": [vp, vp, i64, i32, vp, u32],
        "ta_sincos": [vp, vp, vp, vp, i64, i32, vp],
        "ta_sincos_ex": [vp, vp, vp, vp, i64, i32, vp, u32],
        "ta_taylor_sin": [vp, vp, i64, i32, i32, vp],
        "ta_taylor_cos": [vp, vp, i64, i32, i32, vp],
        "ta_taylor_tan": [vp, vp, i64, i32, i32, vp],
        "ta_sin_bwd": [vp, vp, vp, i64, i32, vp],
        "ta_cos_bwd": [vp, vp, vp, i64, i32, vp],
        "ta_tan_bwd": [vp, vp, vp, i64, i32, vp],
        "ta_sincos_bwd": [vp, vp, vp, vp, i64, i32, vp],
        "ta_sin_fwdbwd": [vp, vp, vp, vp, i64, i32, vp],
        "ta_cos_fwdbwd": [vp, vp, vp, vp, i64, i32, vp],
        "ta_tan_fwdbwd": [vp, vp, vp, vp, i64, i32, vp],
        "ta_paper_sincos": [vp, vp, vp, vp, i64, i32, vp, u32],
        "ta_sincos_encode": [vp, vp, i64, i32, i32, vp],
        "ta_builtin_sincos": [vp, vp, vp, vp, i64, i32, i32, vp],
        "ta_builtin_sin_fwdbwd": [vp, vp, vp, vp, i64, i32, i32, vp],
        "ta_stream_probe": [i32, vp, ctypes.POINTER(vp), i32, i64, u32, vp],
        "ta_copy": [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), i32, i64,
                    i32, vp],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.ta_status_str.argtypes = [ctypes.c_int]
    lib.ta_status_str.restype = ctypes.c_char_p
    lib.ta_last_hip_error.argtypes = []
    lib.ta_last_hip_error.restype = ctypes.c_int
    lib.ta_version.argtypes = []
    lib.ta_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _dev(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise TaError(f"{name} is on {t.device}: libta runs on HIP devices "
                      "only (no CPU fallback)")
    if t.dtype not in _DTYPE_CODE:
        raise TaError(f"{name} has unsupported dtype {t.dtype}")
    if not t.is_contiguous():
        raise TaError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _same(ref: torch.Tensor, *others):
    for name, o in others:
        if o is None:
            continue
        _dev(o, name)
        if o.dtype != ref.dtype or o.numel() != ref.numel() or \
                o.device != ref.device:
            raise TaError(f"{name} must match x in dtype, size and device")


def _check(status: int):
    if status != 0:
        lib = load()
        msg = lib.ta_status_str(status).decode()
        if status == 4:
            msg += f" (hipError {lib.ta_last_hip_error()})"
        raise TaError(msg)


def _args(x):
    return x.numel(), _DTYPE_CODE[x.dtype], _stream(x)


# ---------------------------------------------------------------------------
# C entry points under their own names (outputs passed in)
# ---------------------------------------------------------------------------

def ta_sin(x, y):
    _dev(x, "x"); _same(x, ("y", y))
    n, dt, s = _args(x)
    _check(load().ta_sin(_ptr(x), _ptr(y), n, dt, s))


def ta_cos(x, y):
    _dev(x, "x"); _same(x, ("y", y))
    n, dt, s = _args(x)
    _check(load().ta_cos(_ptr(x), _ptr(y), n, dt, s))


def ta_tan(x, y):
    _dev(x, "x"); _same(x, ("y", y))
    n, dt, s = _args(x)
    _check(load().ta_tan(_ptr(x), _ptr(y), n, dt, s))


def ta_sin_ex(x, y, flags: int):
    _dev(x, "x"); _same(x, ("y", y))
    n, dt, s = _args(x)
    _check(load().ta_sin_ex(_ptr(x), _ptr(y), n, dt, s, int(flags)))


def ta_cos_ex(x, y, flags: int):
    _dev(x, "x"); _same(x, ("y", y))
    n, dt, s = _args(x)
    _check(load().ta_cos_ex(_ptr(x), _ptr(y), n, dt, s, int(flags)))


def ta_tan_ex(x, y, flags: int):
    _dev(x, "x"); _same(x, ("y", y))
    n, dt, s = _args(x)
    _check(load().ta_tan_ex(_ptr(x), _ptr(y), n, dt, s, int(flags)))


def ta_sincos(x, ys, yc, yt=None):
    _dev(x, "x"); _same(x, ("ys", ys), ("yc", yc), ("yt", yt))
    n, dt, s = _args(x)
    _check(load().ta_sincos(_ptr(x), _ptr(ys), _ptr(yc), _ptr(yt), n, dt, s))


def ta_sincos_ex(x, ys, yc, yt, flags: int):
    _dev(x, "x"); _same(x, ("ys", ys), ("yc", yc), ("yt", yt))
    n, dt, s = _args(x)
    _check(load().ta_sincos_ex(_ptr(x), _ptr(ys), _ptr(yc), _ptr(yt), n, dt,
                               s, int(flags)))


def _taylor_entry(name):
    def fn(x, y, terms: int):
        _dev(x, "x"); _same(x, ("y", y))
        n, dt, s = _args(x)
        _check(getattr(load(), name)(_ptr(x), _ptr(y), n, int(terms), dt, s))
    fn.__name__ = name
    return fn


ta_taylor_sin = _taylor_entry("ta_taylor_sin")
ta_taylor_cos = _taylor_entry("ta_taylor_cos")
ta_taylor_tan = _taylor_entry("ta_taylor_tan")


def _bwd_entry(name):
    def fn(x, gy, gx):
        _dev(x, "x"); _same(x, ("gy", gy), ("gx", gx))
        n, dt, s = _args(x)
        _check(getattr(load(), name)(_ptr(x), _ptr(gy), _ptr(gx), n, dt, s))
    fn.__name__ = name
    return fn


ta_sin_bwd = _bwd_entry("ta_sin_bwd")
ta_cos_bwd = _bwd_entry("ta_cos_bwd")
ta_tan_bwd = _bwd_entry("ta_tan_bwd")


def ta_sincos_bwd(x, gs, gc, gx):
    _dev(x, "x"); _same(x, ("gs", gs), ("gc", gc), ("gx", gx))
    n, dt, s = _args(x)
    _check(load().ta_sincos_bwd(_ptr(x), _ptr(gs), _ptr(gc), _ptr(gx), n, dt,
                                s))


def _fwdbwd_entry(name):
    def fn(x, gy, y, gx):
        _dev(x, "x"); _same(x, ("gy", gy), ("y", y), ("gx", gx))
        n, dt, s = _args(x)
        _check(getattr(load(), name)(_ptr(x), _ptr(gy), _ptr(y), _ptr(gx), n,
                                     dt, s))
    fn.__name__ = name
    return fn


ta_sin_fwdbwd = _fwdbwd_entry("ta_sin_fwdbwd")
ta_cos_fwdbwd = _fwdbwd_entry("ta_cos_fwdbwd")
ta_tan_fwdbwd = _fwdbwd_entry("ta_tan_fwdbwd")


def ta_paper_sincos(x, ys=None, yc=None, yt=None, flags: int = 0):
    """The paper's literal arithmetic (Algorithms 1-4: FISR in FP64) on the
    same fold; any non-empty subset of outputs."""
    _dev(x, "x"); _same(x, ("ys", ys), ("yc", yc), ("yt", yt))
    n, dt, s = _args(x)
    _check(load().ta_paper_sincos(_ptr(x), _ptr(ys), _ptr(yc), _ptr(yt), n,
                                  dt, s, int(flags)))


def ta_sincos_encode(x, y, nfreq: int):
    """y (2*nfreq*x.numel() elements, plane-major): plane 2j = sin_a(2^j x),
    plane 2j+1 = cos_a(2^j x)."""
    _dev(x, "x"); _dev(y, "y")
    if y.dtype != x.dtype or y.device != x.device or \
            y.numel() != 2 * int(nfreq) * x.numel():
        raise TaError("y must hold 2*nfreq*x.numel() elements of x's dtype")
    n, dt, s = _args(x)
    _check(load().ta_sincos_encode(_ptr(x), _ptr(y), n, int(nfreq), dt, s))


def ta_builtin_sincos(x, ys, yc=None, yt=None, kind: int = 0):
    """Comparator: the GPU's built-in sinf/cosf/tanf (kind 0), __sinf/...
    (kind 1) or sincosf (kind 2) in the same streaming skeleton; outputs ys,
    ys + yc, or ys + yc + yt."""
    _dev(x, "x"); _same(x, ("ys", ys), ("yc", yc), ("yt", yt))
    n, dt, s = _args(x)
    _check(load().ta_builtin_sincos(_ptr(x), _ptr(ys), _ptr(yc), _ptr(yt), n,
                                    int(kind), dt, s))


def ta_builtin_sin_fwdbwd(x, gy, y, gx, kind: int = 0):
    """Comparator: y = sin x, gx = gy cos x with the built-in functions
    (kind 0 sincosf, kind 1 __sinf/__cosf) in the fused skeleton."""
    _dev(x, "x"); _same(x, ("gy", gy), ("y", y), ("gx", gx))
    n, dt, s = _args(x)
    _check(load().ta_builtin_sin_fwdbwd(_ptr(x), _ptr(gy), _ptr(y), _ptr(gx),
                                        n, int(kind), dt, s))


def ta_stream_probe(kind: int, x, outs, flags: int = 0):
    """Bandwidth probe (kind 0 read x into a 1024-word sink outs[0], 1 write
    outs, 2 copy x into outs) over FP32 arrays of x's size."""
    _dev(x, "x")
    if x.dtype != torch.float32:
        raise TaError("ta_stream_probe streams FP32 arrays")
    for i, t in enumerate(outs):
        _dev(t, f"out{i}")
    n = x.numel()
    s = torch.cuda.current_stream(x.device).cuda_stream
    pout = (ctypes.c_void_p * len(outs))(*[t.data_ptr() for t in outs])
    _check(load().ta_stream_probe(int(kind), _ptr(x), pout, len(outs), n,
                                  int(flags), s))


def ta_copy(ins, outs):
    """Streaming copy with the kernels' access pattern (HBM ceiling)."""
    x = ins[0]
    _dev(x, "in0")
    _same(x, *[(f"in{i}", t) for i, t in enumerate(ins)],
          *[(f"out{i}", t) for i, t in enumerate(outs)])
    n, dt, s = _args(x)
    pin = (ctypes.c_void_p * len(ins))(*[t.data_ptr() for t in ins])
    pout = (ctypes.c_void_p * len(outs))(*[t.data_ptr() for t in outs])
    _check(load().ta_copy(pin, len(ins), pout, len(outs), n, dt, s))


# ---------------------------------------------------------------------------
# allocating helpers
# ---------------------------------------------------------------------------

def _c(x):
    return _dev(x.contiguous(), "x")


def sin(x):
    x = _c(x); y = torch.empty_like(x); ta_sin(x, y); return y


def cos(x):
    x = _c(x); y = torch.empty_like(x); ta_cos(x, y); return y


def tan(x, guard: bool = False):
    x = _c(x); y = torch.empty_like(x)
    ta_tan_ex(x, y, TA_FLAG_TAN_GUARD if guard else 0)
    return y


def sincos(x, with_tan: bool = False, guard: bool = False):
    x = _c(x)
    ys, yc = torch.empty_like(x), torch.empty_like(x)
    yt = torch.empty_like(x) if with_tan else None
    ta_sincos_ex(x, ys, yc, yt, TA_FLAG_TAN_GUARD if guard else 0)
    return (ys, yc, yt) if with_tan else (ys, yc)


def paper_sincos(x, guard: bool = False, literal_divisor: bool = False):
    """(sin, cos, tan) with the paper's literal arithmetic."""
    x = _c(x)
    ys, yc, yt = (torch.empty_like(x) for _ in range(3))
    flags = (TA_FLAG_TAN_GUARD if guard else 0) | \
        (TA_FLAG_LITERAL_DIVISOR if literal_divisor else 0)
    ta_paper_sincos(x, ys, yc, yt, flags)
    return ys, yc, yt


def encode(x, nfreq: int):
    """Tensor [2*nfreq, *x.shape]: sin_a(2^j x), cos_a(2^j x) for j < nfreq."""
    x = _c(x)
    y = torch.empty((2 * int(nfreq),) + tuple(x.shape), dtype=x.dtype,
                    device=x.device)
    ta_sincos_encode(x, y, nfreq)
    return y


def taylor(x, fn: str, terms: int = 5):
    x = _c(x); y = torch.empty_like(x)
    {"sin": ta_taylor_sin, "cos": ta_taylor_cos,
     "tan": ta_taylor_tan}[fn](x, y, terms)
    return y


# ---------------------------------------------------------------------------
# autograd front ends (backward = analytic derivative kernel, recomputed
# from x: only x is saved)
# ---------------------------------------------------------------------------

class SinFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        x = _c(x)
        ctx.save_for_backward(x)
        y = torch.empty_like(x); ta_sin(x, y); return y

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        gx = torch.empty_like(x); ta_sin_bwd(x, g.contiguous(), gx); return gx


class CosFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        x = _c(x)
        ctx.save_for_backward(x)
        y = torch.empty_like(x); ta_cos(x, y); return y

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        gx = torch.empty_like(x); ta_cos_bwd(x, g.contiguous(), gx); return gx


class TanFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        x = _c(x)
        ctx.save_for_backward(x)
        y = torch.empty_like(x); ta_tan(x, y); return y

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        gx = torch.empty_like(x); ta_tan_bwd(x, g.contiguous(), gx); return gx


class SinCosFn(torch.autograd.Function):
    """(sin_a(x), cos_a(x)) with one fused backward kernel."""

    @staticmethod
    def forward(ctx, x):
        x = _c(x)
        ctx.save_for_backward(x)
        ys, yc = torch.empty_like(x), torch.empty_like(x)
        ta_sincos(x, ys, yc, None)
        return ys, yc

    @staticmethod
    def backward(ctx, gs, gc):
        (x,) = ctx.saved_tensors
        gx = torch.empty_like(x)
        if gs is None and gc is None:
            return torch.zeros_like(x)
        ta_sincos_bwd(x, None if gs is None else gs.contiguous(),
                      None if gc is None else gc.contiguous(), gx)
        return gx
