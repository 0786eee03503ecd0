"""Parity rules used by the GPU tests (test infrastructure).

FP32 outputs: |gpu - oracle| <= 4 ulp_f32(oracle), with
    ulp_f32(y) = 2^(max(floor(log2|y|), -126) - 23),
NaN where the oracle is NaN, an exact zero returned with the oracle's sign.

Several-correct-results band: the approximation jumps at 15, 30, 60 and 75
degrees, so an input whose fold angle lies within BAND rad of one of those
nodes may legitimately be evaluated on either neighbouring piece; there the
GPU value must be within the rule of one of the two pieces.

16-bit outputs: the GPU value must be what rounding (RNE) some value within
4 ulp_f32 of the oracle gives: RNE16(ref - tol) <= gpu <= RNE16(ref + tol).
"""
from __future__ import annotations

import math

import numpy as np

import oracle
from paper_2502_10831_amd.workloads import decode_16, round_to_16

BAND = 2.5e-7          # rad, ~2 FP32 ulp of pi/2
U24 = 2.0 ** -24       # unit roundoff of FP32
JUMP_NODES = np.array([1, 2, 4, 5]) * (math.pi / 12)


def ulp32(y):
    y = np.abs(np.asarray(y, np.float64))
    _, e = np.frexp(y)                       # y = m 2^e, 0.5 <= m < 1
    e = np.where(y > 0, np.maximum(e - 1, -126), -126)  # floor(log2 y)
    return np.ldexp(1.0, e - 23)


def neighbour_values(x):
    """For inputs near a jump node: the oracle's values on the piece across
    the nearest node (signed like the outputs); NaN elsewhere."""
    rho, v, k, ns, nc = oracle.fold(x)
    step = math.pi / 12
    knode = np.rint(rho / step)
    near = (np.abs(rho - knode * step) < BAND) & np.isin(knode, (1, 2, 4, 5))
    alt = {name: np.full(len(x), np.nan) for name in ("sin", "cos", "tan")}
    for i in np.nonzero(near)[0]:
        node = knode[i] * step
        k_alt = int(knode[i]) - (1 if rho[i] >= node else 0)
        s, c, t = oracle.piece_scs(k_alt, rho[i], v[i])
        alt["sin"][i] = -s if ns[i] else s
        alt["cos"][i] = -c if nc[i] else c
        alt["tan"][i] = -t if ns[i] != nc[i] else t
    return near, alt


def neighbour_grads(x):
    """For inputs near a jump node: the oracle's derivatives (sin, cos, tan)
    of the piece across the nearest node; NaN elsewhere.  Returns (near,
    alt) like neighbour_values."""
    rho, _, _, _, _ = oracle.fold(x)
    step = math.pi / 12
    knode = np.rint(rho / step)
    near = (np.abs(rho - knode * step) < BAND) & np.isin(knode, (1, 2, 4, 5))
    alt = {name: np.full(len(x), np.nan) for name in ("sin", "cos", "tan")}
    idx = np.nonzero(near)[0]
    if idx.size:
        below = rho[idx] < knode[idx] * step   # neighbour: the next piece
        for shift, sel in ((1, below), (-1, ~below)):
            j = idx[sel]
            if j.size:
                g = oracle.grad(np.asarray(x, np.float64)[j], shift=shift)
                for name in alt:
                    alt[name][j] = g[name]
    return near, alt


def grad_bad(gpu, ref, tol, near=None, alt=None, tol_alt=None):
    """Mask of gradient elements outside `tol` of `ref` that are not, in the
    jump-node band (`near`), within `tol_alt` of the neighbouring piece's
    value `alt`."""
    gpu = np.asarray(gpu, np.float64)
    bad = ~(np.abs(gpu - ref) <= tol)
    if near is not None and bad.any():
        ok_alt = np.abs(gpu - alt) <= tol_alt
        bad &= ~(near & ok_alt)
    return bad


def ulp_error(gpu, ref):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    with np.errstate(invalid="ignore"):
        return np.abs(gpu - ref) / ulp32(ref)


def check_f32(name, x, gpu, ref, alt=None, near=None, max_ulp=4.0):
    """Assert the FP32 rule; returns the max ulp error (see check_f32_counted)."""
    return check_f32_counted(name, x, gpu, ref, alt, near, max_ulp)[0]


def check_f32_counted(name, x, gpu, ref, alt=None, near=None, max_ulp=4.0):
    """Assert the FP32 rule; returns (max ulp error, number of band inputs
    that matched only the neighbouring piece).  Elements that miss the rule
    and lie in the jump-node band are re-checked against the neighbouring
    piece (computed here unless `alt`/`near` are given).  `name` ends with
    the function (sin/cos/tan)."""
    fn = name.rsplit(":", 1)[-1].split("_")[-1].rsplit("-", 1)[-1]
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    nan_ref = np.isnan(ref)
    assert np.array_equal(np.isnan(gpu), nan_ref), \
        f"{name}: NaN mismatch at {np.nonzero(np.isnan(gpu) != nan_ref)[0][:5]}"
    err = ulp_error(gpu, ref)
    err[nan_ref] = 0.0
    rescued = 0
    bad = np.nonzero(err > max_ulp)[0]
    if bad.size:
        if alt is None or near is None:
            near_b, alt_b = neighbour_values(np.asarray(x, np.float64)[bad])
            alt_b = alt_b[fn]
        else:
            near_b, alt_b = near[bad], alt[fn][bad]
        err_alt = ulp_error(gpu[bad], alt_b)
        ok = near_b & (err_alt <= max_ulp)
        rescued = int(ok.sum())
        err[bad[ok]] = err_alt[ok]
    zero = (ref == 0) & ~nan_ref
    if zero.any():
        assert np.array_equal(np.signbit(gpu[zero]), np.signbit(ref[zero])), \
            f"{name}: sign of zero differs"
    worst = float(err.max()) if err.size else 0.0
    if worst > max_ulp:
        i = int(np.argmax(err))
        raise AssertionError(
            f"{name}: {worst:.3f} ulp > {max_ulp} at x={x[i]!r} "
            f"gpu={gpu[i]!r} oracle={ref[i]!r}")
    return worst, rescued


def check_16(name, kind, gpu_raw, ref, tol_abs, alt=None, near=None):
    """16-bit rule: gpu must equal RNE16(y) for some y in ref +- tol_abs
    (or, in the band, around the neighbouring piece's value).  `name` ends
    with the function name (sin/cos/tan)."""
    g = decode_16(gpu_raw, kind)
    ref = np.asarray(ref, np.float64)
    nan_ref = np.isnan(ref)
    assert np.array_equal(np.isnan(g), nan_ref), f"{name}: NaN mismatch"

    def ok_for(r):
        lo = decode_16(round_to_16(r - tol_abs, kind), kind)
        hi = decode_16(round_to_16(r + tol_abs, kind), kind)
        with np.errstate(invalid="ignore"):
            return (g >= lo) & (g <= hi)

    ok = ok_for(ref) | nan_ref
    zero = ref == 0
    ok[zero] &= np.signbit(g[zero]) == np.signbit(ref[zero])
    if alt is not None and near is not None and near.any():
        fn = name.rsplit("-", 1)[-1].rsplit(":", 1)[-1]
        ok_alt = ok_for(np.where(near, alt[fn], ref))
        ok = ok | (near & ok_alt)
    if not ok.all():
        i = int(np.nonzero(~ok)[0][0])
        raise AssertionError(f"{name}/{kind}: gpu={g[i]!r} oracle={ref[i]!r} "
                             f"({(~ok).sum()} bad)")
