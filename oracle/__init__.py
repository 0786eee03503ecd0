"""Plain FP64 CPU oracle for the piecewise sin/cos/tan approximations of
arXiv 2502.10831 (Goyal & Arora).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the benchmark's ``cpu_baseline`` leg, never by the GPU package.  The C
source (``ta_oracle.c``) shares nothing with the HIP kernels.

Functions take float64 numpy arrays (FP32 or 16-bit inputs convert to float64
exactly) and return float64 arrays; the ``*_ld`` forms evaluate the same
definitions in x87 long double (64-bit significand) and return np.longdouble
arrays, for checking FP64 outputs.  See ``ta_oracle.c`` for the readings of
the paper that the oracle takes where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ta_oracle.c")
_LIB = os.path.join(_HERE, "libta_oracle.so")

TAN_GUARD = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", _SRC,
               "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    D = ctypes.POINTER(ctypes.c_double)
    I32 = ctypes.POINTER(ctypes.c_int32)
    i64 = ctypes.c_int64
    lib.ta_or_map.argtypes = [D, i64, D, D, D, ctypes.c_uint, ctypes.c_int]
    lib.ta_or_map.restype = ctypes.c_int
    lib.ta_or_fold_map.argtypes = [D, i64, D, D, I32, I32, I32]
    lib.ta_or_taylor_map.argtypes = [D, i64, ctypes.c_int, D, D, D, D, D, D]
    lib.ta_or_grad_map.argtypes = [D, i64, ctypes.c_int, D, D, D]
    lib.ta_or_fisr_map.argtypes = [D, i64, ctypes.c_double, D, D, D]
    lib.ta_or_paper_map.argtypes = [D, i64, ctypes.c_double, ctypes.c_uint,
                                    D, D, D]
    lib.ta_or_piece.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                D, D]
    lib.ta_or_piece_scs.argtypes = [ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, D, D, D]
    L = ctypes.POINTER(ctypes.c_longdouble)
    lib.ta_or_map_ld.argtypes = [D, i64, L, L, L, ctypes.c_uint, ctypes.c_int]
    lib.ta_or_map_ld.restype = ctypes.c_int
    lib.ta_or_fold_map_ld.argtypes = [D, i64, L, L, I32]
    lib.ta_or_grad_map_ld.argtypes = [D, i64, ctypes.c_int, L, L, L]
    lib.ta_or_segment.argtypes = [ctypes.c_double]
    lib.ta_or_segment.restype = ctypes.c_int
    _lib = lib
    return lib


def _dp(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _x(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def forward(x, flags: int = 0, nthreads: int = 0, want=("sin", "cos", "tan")):
    """The method: returns dict name -> float64 array (Section 2 formulas on
    the Section 3 fold).  Also returns 'threads' = OpenMP threads used."""
    lib = _load()
    x = _x(x)
    n = x.size
    out = {k: np.empty(n, np.float64) for k in want}
    used = lib.ta_or_map(_dp(x), n, _dp(out.get("sin")), _dp(out.get("cos")),
                         _dp(out.get("tan")), flags, nthreads)
    out["threads"] = used
    return out


def sin(x):
    return forward(x, want=("sin",))["sin"]


def cos(x):
    return forward(x, want=("cos",))["cos"]


def tan(x, flags: int = 0):
    return forward(x, flags=flags, want=("tan",))["tan"]


def fold(x):
    """Fold angle rho, complement v, piece index k, sign bits of sin and cos."""
    lib = _load()
    x = _x(x)
    n = x.size
    rho = np.empty(n); v = np.empty(n)
    k = np.empty(n, np.int32); ns = np.empty(n, np.int32)
    nc = np.empty(n, np.int32)
    I32 = ctypes.POINTER(ctypes.c_int32)
    lib.ta_or_fold_map(_dp(x), n, _dp(rho), _dp(v), k.ctypes.data_as(I32),
                       ns.ctypes.data_as(I32), nc.ctypes.data_as(I32))
    return rho, v, k, ns, nc


def piece(k: int, rho: float, v: float):
    """Numerator and denominator (degree units) of piece k at (rho, v)."""
    lib = _load()
    n = ctypes.c_double(); d = ctypes.c_double()
    lib.ta_or_piece(int(k), float(rho), float(v), ctypes.byref(n),
                    ctypes.byref(d))
    return n.value, d.value


def piece_scs(k: int, rho: float, v: float):
    """Unsigned (sin, cos, tan) of piece k at (rho, v)."""
    lib = _load()
    s = ctypes.c_double(); c = ctypes.c_double(); t = ctypes.c_double()
    lib.ta_or_piece_scs(int(k), float(rho), float(v), ctypes.byref(s),
                        ctypes.byref(c), ctypes.byref(t))
    return s.value, c.value, t.value


def segment(rho: float) -> int:
    return _load().ta_or_segment(float(rho))


def taylor(x, terms: int):
    """Taylor-N baseline on the folded angle; also the sums of |terms|."""
    lib = _load()
    x = _x(x)
    n = x.size
    out = {k: np.empty(n) for k in ("sin", "cos", "tan", "abs_sin", "abs_cos",
                                    "abs_tan")}
    lib.ta_or_taylor_map(_dp(x), n, int(terms), _dp(out["sin"]),
                         _dp(out["cos"]), _dp(out["tan"]), _dp(out["abs_sin"]),
                         _dp(out["abs_cos"]), _dp(out["abs_tan"]))
    return out


def grad(x, shift: int = 0):
    """d/dx of the method's sin, cos and tan (derivative of the piece);
    shift evaluates piece k + shift (clamped) instead of the piece rho falls
    in."""
    lib = _load()
    x = _x(x)
    n = x.size
    out = {k: np.empty(n) for k in ("sin", "cos", "tan")}
    lib.ta_or_grad_map(_dp(x), n, int(shift), _dp(out["sin"]),
                       _dp(out["cos"]), _dp(out["tan"]))
    return out


def fisr(rho, divisor: float = np.pi / 12):
    """The paper's literal arithmetic (fast inverse square root) on folded
    angles rho in [0, pi/2]; unsigned values."""
    lib = _load()
    rho = _x(rho)
    n = rho.size
    out = {k: np.empty(n) for k in ("sin", "cos", "tan")}
    lib.ta_or_fisr_map(_dp(rho), n, float(divisor), _dp(out["sin"]),
                       _dp(out["cos"]), _dp(out["tan"]))
    return out


def paper(x, divisor: float = np.pi / 12, flags: int = 0):
    """The paper's literal arithmetic (fold, Algorithms 1-4, guard) on
    angles x; signed outputs."""
    lib = _load()
    x = _x(x)
    n = x.size
    out = {k: np.empty(n) for k in ("sin", "cos", "tan")}
    lib.ta_or_paper_map(_dp(x), n, float(divisor), int(flags),
                        _dp(out["sin"]), _dp(out["cos"]), _dp(out["tan"]))
    return out


# ---- extended precision (long double) forms, for checking FP64 outputs ----
def _lp(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_longdouble)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_longdouble))


def _check_longdouble():
    if np.finfo(np.longdouble).nmant < 63:
        raise RuntimeError("the extended-precision oracle needs an 80-bit "
                           "long double")


def forward_ld(x, flags: int = 0, shift: int = 0,
               want=("sin", "cos", "tan")):
    """The method in long double (64-bit significand) on double inputs:
    dict name -> np.longdouble array.  shift evaluates piece k + shift
    (clamped) instead of the piece rho falls in."""
    _check_longdouble()
    lib = _load()
    x = _x(x)
    n = x.size
    out = {k: np.empty(n, np.longdouble) for k in want}
    lib.ta_or_map_ld(_dp(x), n, _lp(out.get("sin")), _lp(out.get("cos")),
                     _lp(out.get("tan")), flags, int(shift))
    return out


def fold_ld(x):
    """Fold angle rho, complement v (np.longdouble) and piece index k."""
    _check_longdouble()
    lib = _load()
    x = _x(x)
    n = x.size
    rho = np.empty(n, np.longdouble)
    v = np.empty(n, np.longdouble)
    k = np.empty(n, np.int32)
    lib.ta_or_fold_map_ld(_dp(x), n, _lp(rho), _lp(v),
                          k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return rho, v, k


def grad_ld(x, shift: int = 0):
    """d/dx of the method's sin, cos and tan in long double."""
    _check_longdouble()
    lib = _load()
    x = _x(x)
    n = x.size
    out = {k: np.empty(n, np.longdouble) for k in ("sin", "cos", "tan")}
    lib.ta_or_grad_map_ld(_dp(x), n, int(shift), _lp(out["sin"]),
                          _lp(out["cos"]), _lp(out["tan"]))
    return out
