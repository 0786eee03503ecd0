"""Pins for the FP64 oracle (CPU only).

Each test ties the oracle to something other than itself: numbers printed in
the paper (golden fixtures under tests/golden/, each with its citation), exact
values fixed by mathematics, identities of the Appendix A construction, closed
form limits, an independent 60-digit reduction (mpmath), libm, and finite
differences.  A dropped term, a wrong sign or index, or a swapped coefficient
anywhere in the oracle fails at least one of them.
"""
import math
import os

import mpmath
import numpy as np
import pytest

import oracle
from conftest import read_table

K = 180.0 / math.pi
RNG_SEED = 2024873  # the seed quoted in Section 4 of the paper


def _piece_at_deg(k, t_deg):
    rho = math.radians(t_deg)
    v = math.radians(90.0 - t_deg)
    return oracle.piece(k, rho, v)


def _piece_tan_deg(k, t_deg):
    rho = math.radians(t_deg)
    v = math.radians(90.0 - t_deg)
    return oracle.piece_scs(k, rho, v)[2]


# --------------------------------------------------------------------------
# Coefficients: Section 2 printed values and Appendix A forms
# --------------------------------------------------------------------------

def _extract_radian_coefficients(k):
    """Slope/intercept of the oracle's N and D for piece k, in radian units
    (the scale Section 2 prints)."""
    r1, r2 = 0.1, 1.1
    n1, d1 = oracle.piece(k, r1, math.pi / 2 - r1)
    n2, d2 = oracle.piece(k, r2, math.pi / 2 - r2)
    A = (n2 - n1) / (r2 - r1)
    C = (d2 - d1) / (r2 - r1)
    b = n1 - A * r1
    d = d1 - C * r1
    return A, b, C, d


def test_section2_printed_coefficients_are_truncations(golden_dir):
    rows = read_table(os.path.join(golden_dir,
                                   "section2_printed_coefficients.txt"))
    assert len(rows) == 6
    checked = 0
    for row in rows:
        k = int(row[0])
        printed = [float(v) for v in row[1:]]
        A, b, C, d = _extract_radian_coefficients(k)
        qx = A * A + C * C          # Appendix A.4 quadratic, expanded
        qy = 2.0 * (A * b + C * d)
        qz = b * b + d * d
        for p, val in zip(printed, (A, b, C, d, qx, qy, qz)):
            # truncation toward zero to two decimals
            if p == 0.0:
                assert abs(val) < 1e-9
            else:
                assert math.copysign(1.0, p) == math.copysign(1.0, val)
                assert abs(p) <= abs(val) + 1e-7, (k, p, val)
                assert abs(val) < abs(p) + 0.01, (k, p, val)
            checked += 1
    assert checked == 42


def test_appendix_integer_forms(golden_dir):
    rows = read_table(os.path.join(golden_dir, "appendix_a_integer_forms.txt"))
    assert [int(r[0]) for r in rows] == list(range(6))
    for row in rows:
        k = int(row[0])
        t_lo, t_hi = float(row[2]), float(row[3])
        a, b, c, d = (float(v) for v in row[4:8])
        for t in np.linspace(t_lo, t_hi, 7):
            n, den = _piece_at_deg(k, t)
            assert n == pytest.approx(a * t + b, abs=1e-9)
            assert den == pytest.approx(c * t + d, abs=1e-9)


def test_appendix_decimal_forms_from_sin_interpolation(golden_dir):
    """Appendix A.1/A.2: each tan piece on 15-75 degrees is the ratio of two
    two-point interpolants of sin on 15-degree nodes.  Recompute the decimal
    forms from libm sin at the nodes, compare with the printed (truncated)
    decimals, and check the oracle's integer pieces follow them."""
    rows = read_table(os.path.join(golden_dir, "appendix_a_decimal_forms.txt"))
    sd = lambda deg: math.sin(math.radians(deg))
    for row in rows:
        k = int(row[0])
        p_ns, p_ni, p_ds, p_di = (float(v) for v in row[2:6])
        lo, hi = 15.0 * k, 15.0 * (k + 1)
        ns = sd(hi) - sd(lo)
        ni = hi * sd(lo) - lo * sd(hi)
        lo2, hi2 = 90.0 - hi, 90.0 - lo
        ds = sd(hi2) - sd(lo2)
        di = hi2 * sd(lo2) - lo2 * sd(hi2)
        computed = (ns, ni, -ds, 90.0 * ds + di)
        for j, (p, val) in enumerate(zip((p_ns, p_ni, p_ds, p_di), computed)):
            if k == 1 and j == 2:
                # eq. (5) prints -0.099: the slope -0.0999 cut to 3 decimals
                assert abs(p) <= abs(val) < abs(p) + 1e-3
                continue
            if k == 1 and j == 3:
                # eq. (5) prints 15.9673 for 15.9874 (misprint, 0.13%)
                assert abs(val - p) / abs(val) < 2e-3
                continue
            assert abs(p) <= abs(val) + 1e-12 and abs(val) < abs(p) + 1e-4, \
                (k, j, p, val)
        # the rounded integer form stays within 0.2% of the decimal form
        for t in np.linspace(lo, hi, 31):
            t_dec = (ns * t + ni) / (-ds * t + 90.0 * ds + di)
            assert abs(_piece_tan_deg(k, t) / t_dec - 1.0) < 2e-3


def test_appendix_a3_identities():
    """A.3 builds pieces 0 and 5 from piece 2 with tan(45 -+ x'); the A.2
    construction makes piece 4 the reflection of piece 1 and piece 5 of
    piece 0 (tan t * tan(90 - t) = 1)."""
    for t in np.linspace(0.0, 15.0, 61):
        t2 = _piece_tan_deg(2, 45.0 - t)
        assert _piece_tan_deg(0, t) == pytest.approx((1 - t2) / (1 + t2),
                                                     rel=1e-12, abs=1e-15)
    for t in np.linspace(75.0, 89.9, 61):
        t2 = _piece_tan_deg(2, t - 45.0)
        assert _piece_tan_deg(5, t) == pytest.approx((1 + t2) / (1 - t2),
                                                     rel=1e-11)
    for t in np.linspace(60.0, 75.0, 31):
        assert _piece_tan_deg(4, t) * _piece_tan_deg(1, 90.0 - t) == \
            pytest.approx(1.0, rel=1e-13)
    for t in np.linspace(75.0, 89.9, 31):
        assert _piece_tan_deg(5, t) * _piece_tan_deg(0, 90.0 - t) == \
            pytest.approx(1.0, rel=1e-12)
    # pieces 2 and 3 are NOT reflections of each other
    dev = max(abs(_piece_tan_deg(3, t) * _piece_tan_deg(2, 90.0 - t) - 1.0)
              for t in np.linspace(45.0, 60.0, 301))
    assert dev > 1e-4


# --------------------------------------------------------------------------
# Values fixed by mathematics
# --------------------------------------------------------------------------

def test_exact_at_0_45_90_degrees():
    r = oracle.forward([0.0, -0.0])
    assert r["sin"][0] == 0.0 and not math.copysign(1, r["sin"][0]) < 0
    assert math.copysign(1, r["sin"][1]) < 0 and r["sin"][1] == 0.0
    assert math.copysign(1, r["tan"][1]) < 0 and r["tan"][1] == 0.0
    assert r["cos"][0] == 1.0 and r["cos"][1] == 1.0
    h = math.sqrt(0.5)
    for k in (2, 3):  # 45 degrees from both sides: N = D exactly
        s, c, t = oracle.piece_scs(k, math.pi / 4, math.pi / 4)
        assert s == pytest.approx(h, rel=1e-15)
        assert c == pytest.approx(h, rel=1e-15)
        assert t == pytest.approx(1.0, rel=1e-14)
    r = oracle.forward([math.pi / 4])
    assert r["sin"][0] == pytest.approx(h, rel=1e-14)
    assert r["tan"][0] == pytest.approx(1.0, rel=1e-14)
    s, c, t = oracle.piece_scs(5, math.pi / 2, 0.0)
    assert s == 1.0 and c == 0.0 and math.isinf(t)


def test_special_inputs():
    r = oracle.forward([math.nan, math.inf, -math.inf])
    for name in ("sin", "cos", "tan"):
        assert np.isnan(r[name]).all()


def test_segment_index_at_nodes():
    for k in range(1, 6):
        node = k * math.pi / 12
        assert oracle.segment(node * (1 + 1e-12)) == k
        assert oracle.segment(node * (1 - 1e-12)) == k - 1
    assert oracle.segment(math.pi / 2) == 5
    assert oracle.segment(0.0) == 0


# --------------------------------------------------------------------------
# Reduction (Section 3 fold) against an independent 60-digit reduction
# --------------------------------------------------------------------------

WORST_FP32 = [252.898209, 4.71238899, 1.57079637, 3.14159274, 1.5707963,
              -7.85398149, 823549.625, 1e6, -999999.9375, 0.7853982]


def test_fold_against_mpmath():
    mpmath.mp.dps = 60
    rng = np.random.default_rng(RNG_SEED)
    xs = [float(np.float32(w)) for w in WORST_FP32]
    xs += [float(v) for v in
           rng.uniform(-1e6, 1e6, 200).astype(np.float32)]
    rho, v, k, ns, nc = oracle.fold(xs)
    for i, x in enumerate(xs):
        s = mpmath.sin(mpmath.mpf(x))
        c = mpmath.cos(mpmath.mpf(x))
        r_mp = mpmath.asin(abs(s)) if abs(s) < abs(c) else \
            mpmath.acos(abs(c))
        v_mp = mpmath.pi / 2 - r_mp
        assert abs(rho[i] - r_mp) <= 2.0 ** -50 * r_mp, x
        assert abs(v[i] - v_mp) <= 2.0 ** -50 * v_mp, x
        assert ns[i] == (1 if s < 0 else 0)
        assert nc[i] == (1 if c < 0 else 0)
        assert k[i] == min(int(mpmath.floor(r_mp / (mpmath.pi / 12))), 5)


def test_symmetry_and_periodicity():
    rng = np.random.default_rng(RNG_SEED)
    x = rng.uniform(-1e4, 1e4, 20000)
    a = oracle.forward(x)
    b = oracle.forward(-x)
    np.testing.assert_array_equal(b["sin"], -a["sin"])
    np.testing.assert_array_equal(b["cos"], a["cos"])
    np.testing.assert_array_equal(b["tan"], -a["tan"])
    rho, v, _, _, _ = oracle.fold(x)
    node_dist = np.abs(rho / (math.pi / 12) - np.round(rho / (math.pi / 12)))
    ok = (node_dist > 1e-7) & (v > 1e-3)
    for shift, names in ((2 * math.pi, ("sin", "cos", "tan")),
                         (math.pi, ("tan",))):
        c = oracle.forward(x + shift)
        for name in names:
            # the shifted argument is rounded to double: |dx| <= 1e-12, and
            # tan amplifies it by up to tan^2 <= 1e6 here
            np.testing.assert_allclose(c[name][ok], a[name][ok], rtol=1e-8,
                                       atol=1e-9)
    # sin(pi - x) = sin(x) for the fold
    d = oracle.forward(math.pi - x)
    np.testing.assert_allclose(d["sin"][ok], a["sin"][ok], atol=1e-9, rtol=0)
    # sin_a(pi/2 - x) == cos_a(x) exactly in real arithmetic whenever the
    # fold angle lies outside [30, 60] degrees (pieces 0/1 reflect 5/4)
    e = oracle.forward(math.pi / 2 - x)
    deg = np.degrees(rho)
    outside = ok & ((deg < 29.99) | (deg > 60.01))
    np.testing.assert_allclose(e["sin"][outside], a["cos"][outside],
                               atol=1e-9, rtol=0)
    inside = ok & (deg > 31) & (deg < 59)
    assert np.abs(e["sin"][inside] - a["cos"][inside]).max() > 1e-5


# --------------------------------------------------------------------------
# Closed-form limits
# --------------------------------------------------------------------------

def test_limits():
    rho = 1e-8
    s, c, t = oracle.piece_scs(0, rho, math.pi / 2 - rho)
    assert s / math.sin(rho) == pytest.approx(11 * 180 / (632 * math.pi),
                                              rel=1e-9)
    v = 1e-9
    s, c, t = oracle.piece_scs(5, math.pi / 2 - v, v)
    assert t / (1.0 / math.tan(v)) == pytest.approx(632 * math.pi / 1980,
                                                    rel=1e-8)


# --------------------------------------------------------------------------
# Error envelope against libm and the paper's Tables 1-3
# --------------------------------------------------------------------------

def _table(golden_dir):
    rows = read_table(os.path.join(golden_dir, "table_error_statistics.txt"))
    return {(r[0], r[1]): [float(v) for v in r[2:]] for r in rows}


@pytest.fixture(scope="module")
def dense_rho():
    return np.linspace(0.0, math.pi / 2, 2_000_001)[1:-1]


def test_exact_formula_within_paper_error_bounds(golden_dir, dense_rho):
    tab = _table(golden_dir)
    r = oracle.forward(dense_rho)
    es = np.abs(r["sin"] - np.sin(dense_rho))
    ec = np.abs(r["cos"] - np.cos(dense_rho))
    assert es.max() < tab[("sin", "proposed")][0]
    assert ec.max() < tab[("cos", "proposed")][0]
    m = dense_rho < math.pi / 2 - 1e-3
    tt = np.tan(dense_rho[m])
    assert (np.abs(r["tan"][m] - tt) / tt).max() < tab[("tan", "proposed")][3]
    # the method is an approximation: errors are not zero
    assert es.max() > 1e-4


def test_fisr_variant_reproduces_paper_tables(golden_dir, dense_rho):
    """Algorithm 1-4 arithmetic reproduces the printed 0.001532 maximum and,
    within sampling error of 1000 angles, the printed averages."""
    tab = _table(golden_dir)
    f = oracle.fisr(dense_rho)
    for name, fn in (("sin", np.sin), ("cos", np.cos), ("tan", np.tan)):
        p_amax, p_aavg, p_astd, p_rmax, p_ravg, p_rstd = tab[(name,
                                                              "proposed")]
        m = dense_rho < math.pi / 2 - 1e-3
        ref = fn(dense_rho[m])
        ea = np.abs(f[name][m] - ref)
        er = ea / np.abs(ref)
        if name in ("sin", "cos"):
            assert round(ea.max(), 6) == p_amax
            se = ea.std() / math.sqrt(1000)
            assert abs(ea.mean() - p_aavg) < 3.5 * se
            assert ea.std() == pytest.approx(p_astd, rel=0.1)
        # a dense maximum bounds the 1000-angle sample maximum from above
        assert p_rmax <= er.max() <= 1.15 * p_rmax
        se = er.std() / math.sqrt(1000)
        assert abs(er.mean() - p_ravg) < 3.5 * se
        assert er.std() == pytest.approx(p_rstd, rel=0.1)
    # and the exact square root is more accurate than the FISR form
    r = oracle.forward(dense_rho)
    assert np.abs(r["sin"] - np.sin(dense_rho)).max() < \
        0.5 * np.abs(f["sin"] - np.sin(dense_rho)).max()


# --------------------------------------------------------------------------
# Taylor baseline
# --------------------------------------------------------------------------

def test_taylor_converges_to_libm(dense_rho):
    x = dense_rho[::10]
    t9 = oracle.taylor(x, 9)
    np.testing.assert_allclose(t9["sin"], np.sin(x), rtol=0, atol=1e-13)
    np.testing.assert_allclose(t9["cos"], np.cos(x), rtol=0, atol=1e-12)
    m = x < 0.5
    np.testing.assert_allclose(t9["tan"][m], np.tan(x[m]), rtol=1e-9)


def test_taylor_remainders_match_mpmath(golden_dir):
    mpmath.mp.dps = 40
    half_pi = math.pi / 2
    for terms in (5, 7, 9):
        t = oracle.taylor([half_pi], terms)
        s_mp = sum((-1) ** j * mpmath.mpf(half_pi) ** (2 * j + 1) /
                   mpmath.factorial(2 * j + 1) for j in range(terms))
        c_mp = sum((-1) ** j * mpmath.mpf(half_pi) ** (2 * j) /
                   mpmath.factorial(2 * j) for j in range(terms))
        assert t["sin"][0] == pytest.approx(float(s_mp), abs=1e-15)
        assert t["cos"][0] == pytest.approx(float(c_mp), abs=1e-15)
    tab = _table(golden_dir)
    t5 = oracle.taylor([half_pi], 5)
    # Taylor-5 errors are largest at pi/2; the printed sample maxima are at
    # most these (rounded to 6 decimals)
    assert abs(1.0 - t5["sin"][0]) >= tab[("sin", "taylor5_nosimd")][0] - 5e-7
    assert abs(0.0 - t5["cos"][0]) >= tab[("cos", "taylor5_nosimd")][0] - 5e-7


def _tangent_coefficients(count):
    """c_j of tan(z) = sum_j c_j z^(2j+1), from the Bernoulli-number closed
    form c_j = (-1)^j 2^(2n) (2^(2n) - 1) B_(2n) / (2n)!, n = j + 1, as exact
    fractions (independent of the decimal or rational constants the oracle
    carries)."""
    from fractions import Fraction
    out = []
    for j in range(count):
        n = j + 1
        p, q = mpmath.bernfrac(2 * n)
        b = Fraction(int(p), int(q))
        c = (-1) ** j * 2 ** (2 * n) * (2 ** (2 * n) - 1) * b / \
            math.factorial(2 * n)
        out.append(c)
    return out


def test_taylor_tan_series_matches_bernoulli_form():
    """Taylor-N tan is the first N terms of the tangent series (the Taylor
    columns of Table 3).  Checked at rho = pi/2, 1.5 and 0.7 against the sum
    built from the Bernoulli closed form of the coefficients, in 50-digit
    arithmetic at the oracle's own folded angle: a change of one unit in any
    numerator or denominator of the highest coefficients moves the sum by
    more than 1e-8 relative at pi/2."""
    mpmath.mp.dps = 50
    coef = _tangent_coefficients(9)
    # known first values of the series, as a check of the closed form itself
    from fractions import Fraction
    assert coef[:4] == [Fraction(1), Fraction(1, 3), Fraction(2, 15),
                        Fraction(17, 315)]
    for x in (math.pi / 2, 1.5, 0.7):
        rho = float(oracle.fold([x])[0][0])
        for terms in (5, 7, 9):
            got = oracle.taylor([x], terms)["tan"][0]
            want = sum(mpmath.mpf(c.numerator) / c.denominator *
                       mpmath.mpf(rho) ** (2 * j + 1)
                       for j, c in enumerate(coef[:terms]))
            assert got == pytest.approx(float(want), rel=1e-13, abs=0), \
                (x, terms)


def test_forward_tan_guard_threshold():
    """proposed_tan (Section 3) returns +infinity, before any sign, when the
    folded angle is within 1e-3 of pi/2.  The oracle's guarded forward must
    switch exactly there: +inf for v = 1e-3 - 1e-9 on either side of a pole
    and for either sign of x, the piece's finite value for v = 1e-3 + 1e-9;
    sin and cos do not depend on the flag."""
    for m in (0, 1, 7, 300):
        pole = (2 * m + 1) * math.pi / 2
        for sgn in (1.0, -1.0):
            for side in (1.0, -1.0):
                inside = sgn * (pole + side * (1e-3 - 1e-9))
                outside = sgn * (pole + side * (1e-3 + 1e-9))
                g_in = oracle.forward([inside], flags=oracle.TAN_GUARD)
                g_out = oracle.forward([outside], flags=oracle.TAN_GUARD)
                p_in = oracle.forward([inside])
                assert np.isposinf(g_in["tan"][0]), (m, sgn, side)
                assert np.isfinite(g_out["tan"][0]), (m, sgn, side)
                assert g_out["tan"][0] == oracle.forward([outside])["tan"][0]
                assert np.isfinite(p_in["tan"][0])
                assert abs(p_in["tan"][0]) > 900.0
                for name in ("sin", "cos"):
                    assert g_in[name][0] == p_in[name][0]
    # the threshold is on the folded angle, not on x: far from any pole the
    # flag changes nothing
    x = np.linspace(-10, 10, 20001)
    rho, v, _, _, _ = oracle.fold(x)
    far = v > 1.001e-3
    np.testing.assert_array_equal(
        oracle.forward(x[far], flags=oracle.TAN_GUARD)["tan"],
        oracle.forward(x[far])["tan"])


def test_taylor_tan_reproduces_table3_worst_angle(golden_dir):
    """The Table 3 Taylor columns share one worst angle: abs/rel of the
    Taylor-5 (SIMD) column gives tan there; the Taylor-7 and -9 columns must
    follow from the same angle."""
    tab = _table(golden_dir)
    a5, r5 = tab[("tan", "taylor5_simd")][0], tab[("tan", "taylor5_simd")][3]
    tan_star = a5 / r5
    x = [math.atan(tan_star)]
    for terms, key, tol in ((5, "taylor5_simd", 1e-4),
                            (7, "taylor7_simd", 1e-4),
                            (9, "taylor9_simd", 3e-3)):
        t = oracle.taylor(x, terms)["tan"][0]
        assert abs((tan_star - t) - tab[("tan", key)][0]) < tol
        assert abs((tan_star - t) / tan_star - tab[("tan", key)][3]) < 2e-5


# --------------------------------------------------------------------------
# Derivative
# --------------------------------------------------------------------------

def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(RNG_SEED)
    x = rng.uniform(-50, 50, 4000)
    h = 1e-6
    rho, v, _, _, _ = oracle.fold(x)
    node = np.abs(rho - np.round(rho / (math.pi / 12)) * (math.pi / 12))
    x = x[(node > 4 * h) & (v > 1e-2)]
    g = oracle.grad(x)
    fp = oracle.forward(x + h)
    fm = oracle.forward(x - h)
    for name in ("sin", "cos", "tan"):
        fd = (fp[name] - fm[name]) / (2 * h)
        np.testing.assert_allclose(g[name], fd, rtol=1e-6, atol=1e-8)


def test_gradient_shift_is_the_neighbouring_piece_derivative():
    """grad(x, shift) differentiates piece k + shift (clamped to 0..5):
    checked against central differences of that piece's values (piece_scs)
    at the same fold angle, on first-quadrant x where d rho/dx = 1."""
    rng = np.random.default_rng(RNG_SEED + 1)
    x = rng.uniform(0.02, math.pi / 2 - 0.02, 2000)
    h = 1e-6
    k0 = np.array([oracle.segment(r) for r in x])
    for shift in (-1, 1):
        g = oracle.grad(x, shift=shift)
        for i in range(0, x.size, 7):
            k = min(5, max(0, k0[i] + shift))
            sp = oracle.piece_scs(k, x[i] + h, math.pi / 2 - x[i] - h)
            sm = oracle.piece_scs(k, x[i] - h, math.pi / 2 - x[i] + h)
            for j, name in enumerate(("sin", "cos", "tan")):
                fd = (sp[j] - sm[j]) / (2 * h)
                assert g[name][i] == pytest.approx(fd, rel=1e-6, abs=1e-8), \
                    (shift, x[i], name)
    # shift 0 is the plain derivative; a shift past the ends clamps
    np.testing.assert_array_equal(oracle.grad(x, shift=0)["sin"],
                                  oracle.grad(x)["sin"])
    low = x[k0 == 0]
    np.testing.assert_array_equal(oracle.grad(low, shift=-1)["sin"],
                                  oracle.grad(low)["sin"])


def test_gradient_closed_forms_and_trig_distance(dense_rho):
    g = oracle.grad([0.0])
    assert g["sin"][0] == pytest.approx(11 * 180 / (632 * math.pi), rel=1e-14)
    x = dense_rho[::4]
    g = oracle.grad(x)
    f = oracle.forward(x)
    # omega = K (ad - bc)/Q is the same factor for sin, cos and tan
    om_s = g["sin"] / f["cos"]
    om_c = -g["cos"] / f["sin"]
    om_t = g["tan"] / (1 + f["tan"] ** 2)
    np.testing.assert_allclose(om_c, om_s, rtol=1e-12)
    np.testing.assert_allclose(om_t[x < 1.5], om_s[x < 1.5], rtol=1e-12)
    assert 0.97 < om_s.min() and om_s.max() < 1.01
    assert np.abs(g["sin"] - np.cos(x)).max() < 2.3e-2


def test_paper_protocol_statistics(golden_dir):
    """Section 4 protocol on the oracle's literal arithmetic: angles uniform
    in [-1e6, 1e6]; errors against libm as in run_benchmark (relative error
    0 where |std| <= 1e-12).  The sample here is 10^6 angles; the printed
    values come from 1000, so the averages agree within that sample's
    standard error and the printed maxima are at most ours."""
    tab = _table(golden_dir)
    rng = np.random.default_rng(RNG_SEED)
    x = rng.uniform(-1e6, 1e6, 1_000_000)
    got = oracle.paper(x)
    for name, fn in (("sin", np.sin), ("cos", np.cos), ("tan", np.tan)):
        ref = fn(x)
        ea = np.abs(got[name] - ref)
        er = np.where(np.abs(ref) > 1e-12, ea / np.abs(ref), 0.0)
        p_amax, p_aavg, p_astd, p_rmax, p_ravg, p_rstd = tab[(name,
                                                              "proposed")]
        if name != "tan":
            assert round(ea.max(), 6) == p_amax
            assert abs(ea.mean() - p_aavg) < 3.5 * ea.std() / math.sqrt(1000)
        keep = np.abs(np.cos(x)) > 1e-3 if name == "tan" else slice(None)
        assert p_rmax <= er[keep].max() <= 1.25 * p_rmax
        assert abs(er.mean() - p_ravg) < 3.5 * er.std() / math.sqrt(1000)
    # proposed_tan's guard: +inf (unsigned) within 1e-3 of the poles
    g = oracle.paper(x[:20000], flags=oracle.TAN_GUARD)["tan"]
    near_pole = np.abs(np.cos(x[:20000])) < math.sin(1e-3)
    assert np.all(np.isposinf(g[near_pole]))
    assert not np.isinf(g[~near_pole]).any()
