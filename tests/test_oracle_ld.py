"""Pins for the extended-precision (long double) oracle used to check FP64
outputs (CPU only).

Each test ties it to something other than itself: an independent 60-digit
reduction (mpmath) over double inputs including the hardest ones for the
fold, the FP64 oracle (itself pinned to the paper's printed numbers), exact
rational values of the Appendix A forms at the piece nodes, closed-form
limits at 0 and at the pole, the identities sin^2 + cos^2 = 1 and
tan = sin / cos, symmetry, and finite differences for the derivative.
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle

RNG_SEED = 2024873
LD_EPS = float(np.finfo(np.longdouble).eps)  # 2^-63

# Doubles closest to a multiple of pi/2 (the hardest inputs for any
# reduction); the first is the closest over all finite doubles.
HARD_DOUBLES = [6381956970095103.0 * 2.0 ** 797, 5.319372648326541e+255,
                float.fromhex("0x1.921fb54442d18p+0"),
                float.fromhex("0x1.921fb54442d18p+1"),
                float.fromhex("0x1.2d97c7f3321d2p+2"), 1e22, 355.0,
                float.fromhex("0x1.921fb54442d18p+10")]


def _mp(v):
    """A long double as an exact mpmath number (sum of two doubles)."""
    hi = float(v)
    return mpmath.mpf(hi) + mpmath.mpf(float(v - np.longdouble(hi)))


def _doubles(n, seed):
    rng = np.random.default_rng(seed)
    mag = 10.0 ** rng.uniform(-30, 300, n)
    return np.where(rng.random(n) < 0.5, -mag, mag)


def test_ld_fold_against_mpmath():
    mpmath.mp.dps = 80
    xs = HARD_DOUBLES + [float(v) for v in _doubles(150, RNG_SEED)] + \
        [float(v) for v in np.random.default_rng(7).uniform(-1e6, 1e6, 100)]
    rho, v, k = oracle.fold_ld(xs)
    for i, x in enumerate(xs):
        s = mpmath.sin(mpmath.mpf(x))
        c = mpmath.cos(mpmath.mpf(x))
        r_mp = mpmath.asin(abs(s)) if abs(s) < abs(c) else mpmath.acos(abs(c))
        v_mp = mpmath.pi / 2 - r_mp
        for got, ref in ((rho[i], r_mp), (v[i], v_mp)):
            err = abs(_mp(got) - ref)
            assert err <= 8 * LD_EPS * ref, (x, float(got), ref)
        assert k[i] == min(int(mpmath.floor(r_mp / (mpmath.pi / 12))), 5), x


def _node_band(rho, width):
    q = rho / (np.longdouble(math.pi) / 12)
    return np.abs(q - np.round(q)) < width


def test_ld_agrees_with_fp64_oracle():
    x = np.concatenate([_doubles(20000, RNG_SEED + 1),
                        np.random.default_rng(3).uniform(-100, 100, 20000)])
    ld = oracle.forward_ld(x)
    f64 = oracle.forward(x)
    rho, v, _ = oracle.fold_ld(x)
    keep = ~_node_band(rho, 1e-9)
    for name in ("sin", "cos", "tan"):
        ref = ld[name][keep]
        err = np.abs(f64[name][keep].astype(np.longdouble) - ref)
        ulp = np.spacing(np.abs(ref.astype(np.float64)))
        assert float((err / ulp).max()) <= 6.0, name


def test_ld_identities_and_symmetry():
    x = np.concatenate([_doubles(5000, RNG_SEED + 2), HARD_DOUBLES])
    r = oracle.forward_ld(x)
    one = r["sin"] ** 2 + r["cos"] ** 2
    assert float(np.abs(one - 1).max()) <= 8 * LD_EPS
    rel = np.abs(r["tan"] * r["cos"] - r["sin"]) / np.abs(r["sin"])
    assert float(rel.max()) <= 8 * LD_EPS
    m = oracle.forward_ld(-x)
    assert np.array_equal(m["sin"], -r["sin"])
    assert np.array_equal(m["cos"], r["cos"])
    assert np.array_equal(m["tan"], -r["tan"])
    z = oracle.forward_ld([0.0, -0.0])
    assert z["cos"][0] == 1 and z["cos"][1] == 1
    assert z["sin"][0] == 0 and np.signbit(z["sin"][1])
    s = oracle.forward_ld([math.nan, math.inf, -math.inf])
    assert all(np.isnan(s[n]).all() for n in ("sin", "cos", "tan"))


def test_ld_node_values_are_appendix_a_rationals():
    """At the five interior nodes the pieces take the exact rational tan
    values of their integer forms (Appendix A, eqs. 5-10); the nearest double
    misses the node by dx, which moves tan by (a d - b c)/D^2 per degree."""
    a = [11, 10, 6, 10, 4, 1]
    b = [0, 10, 46, 217, 297, 542]
    c = [-1, -4, -5, -13, -10, -11]
    d = [632, 657, 541, 1252, 910, 990]
    mpmath.mp.dps = 40
    for node in range(1, 6):
        t = 15 * node
        x = float(mpmath.pi * t / 180)      # nearest double to the node
        dx_deg = (mpmath.mpf(x) * 180 / mpmath.pi) - t
        for shift in (-1, 0, 1):
            r = oracle.forward_ld([x], shift=shift)
            rho, _, k = oracle.fold_ld([x])
            kk = min(max(int(k[0]) + shift, 0), 5)
            exact = Fraction(a[kk] * t + b[kk], c[kk] * t + d[kk])
            # d tan/dt of the piece = (a d - b c) / D^2 (per degree)
            slope = Fraction(a[kk] * d[kk] - b[kk] * c[kk],
                             (c[kk] * t + d[kk]) ** 2)
            ref = mpmath.mpf(exact.numerator) / exact.denominator + \
                mpmath.mpf(slope.numerator) / slope.denominator * dx_deg
            got = _mp(r["tan"][0])
            assert abs(got - ref) <= 16 * LD_EPS * ref, (t, shift, kk)


def test_ld_limits_at_zero_and_pole():
    """sin_a(x)/x -> 11 K / 632 as x -> 0 (piece 0: N = 11 t, D = 632 - t,
    K = 180/pi) and tan_a(pi/2 + e) ~ -632 / (11 K e) (piece 5 about 90
    degrees: N -> 632, D = 11 K e)."""
    mpmath.mp.dps = 40
    K = 180 / mpmath.pi
    x = 2.0 ** -64
    s = oracle.forward_ld([x])["sin"][0]
    assert abs(_mp(s) / mpmath.mpf(x) / (11 * K / 632) - 1) < 4 * LD_EPS
    e = 2.0 ** -60
    xp = float(mpmath.pi / 2)   # below pi/2 by ~6.1e-17
    r = oracle.forward_ld([xp, -xp])
    gap = mpmath.pi / 2 - mpmath.mpf(xp)
    ref = 632 / (11 * K * gap)
    assert abs(_mp(r["tan"][0]) / ref - 1) < 1e-15
    assert abs(_mp(r["tan"][1]) / -ref - 1) < 1e-15
    assert gap > 0 and e < gap


def test_ld_gradient_matches_finite_differences():
    rng = np.random.default_rng(RNG_SEED + 3)
    x = rng.uniform(-60, 60, 3000)
    h = 2.0 ** -20
    rho, v, _ = oracle.fold_ld(x)
    keep = ~_node_band(rho, 1e-4) & (v > 1e-2)
    x = x[keep]
    g = oracle.grad_ld(x)
    fp = oracle.forward_ld(x + h)
    fm = oracle.forward_ld(x - h)
    f = oracle.forward_ld(x)
    fp2 = oracle.forward_ld(x + h / 2)
    fm2 = oracle.forward_ld(x - h / 2)
    for name in ("sin", "cos", "tan"):
        # Richardson: (4 D(h/2) - D(h)) / 3 cancels the h^2 term
        d1 = (fp[name] - fm[name]) / np.longdouble(2 * h)
        d2 = (fp2[name] - fm2[name]) / np.longdouble(h)
        fd = (4 * d2 - d1) / 3
        scale = np.maximum(np.abs(g[name]), 1)
        assert float((np.abs(g[name] - fd) / scale).max()) < 1e-10, name
    om_s = g["sin"] / f["cos"]
    om_c = -g["cos"] / f["sin"]
    om_t = g["tan"] / (1 + f["tan"] ** 2)
    assert float(np.abs(om_c / om_s - 1).max()) < 64 * LD_EPS
    assert float(np.abs(om_t / om_s - 1).max()) < 64 * LD_EPS
    g64 = oracle.grad(x)
    assert float(np.abs(g64["sin"] - g["sin"]).max()) < 1e-14


def test_ld_tan_guard_threshold():
    """The guarded long-double tan switches to +infinity, unsigned, exactly
    where proposed_tan's guard (Section 3) does: folded angle within 1e-3 of
    pi/2 (v = 1e-3 - 1e-9 guarded, v = 1e-3 + 1e-9 not), for both signs of
    x and both sides of a pole; sin and cos do not depend on the flag."""
    for m in (0, 3, 300):
        pole = (2 * m + 1) * math.pi / 2
        for sgn in (1.0, -1.0):
            for side in (1.0, -1.0):
                x = [sgn * (pole + side * (1e-3 - 1e-9)),
                     sgn * (pole + side * (1e-3 + 1e-9))]
                g = oracle.forward_ld(x, flags=oracle.TAN_GUARD)
                p = oracle.forward_ld(x)
                assert np.isposinf(g["tan"][0]), (m, sgn, side)
                assert np.isfinite(g["tan"][1]) and g["tan"][1] == p["tan"][1]
                assert np.isfinite(p["tan"][0])
                for name in ("sin", "cos"):
                    np.testing.assert_array_equal(g[name], p[name])
