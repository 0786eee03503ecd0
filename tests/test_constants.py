"""The GPU source's constants against first principles (CPU only): the
reduction constants re-derived from pi with 400-bit mpmath, the 2/pi bit
table, and the per-piece integers against the Appendix A forms printed in the
paper."""
import os
import re

import mpmath
import pytest

from conftest import ROOT, read_table

SRC = os.path.join(ROOT, "paper_2502_10831_amd", "csrc", "ta_math.hpp")


@pytest.fixture(scope="module")
def text():
    return open(SRC).read()


def _const(text, name):
    m = re.search(rf"constexpr double {name} = ([0-9a-fx.p+-]+);", text)
    assert m, name
    return float.fromhex(m.group(1))


def test_reduction_constants(text):
    mpmath.mp.prec = 400
    pi = mpmath.pi
    assert _const(text, "kTwoOverPi") == float(2 / pi)
    hi = _const(text, "kPio2Hi")
    assert hi == float(pi / 2)
    assert _const(text, "kPio2Lo") == float(pi / 2 - mpmath.mpf(hi))
    assert _const(text, "kDegPerRad") == float(180 / pi)
    assert _const(text, "kRoundMagic") == 1.5 * 2.0 ** 52
    assert _const(text, "kPi12") == float(pi / 12)
    # FP64 path: third word of pi/2, the low word of 180/pi
    lo = _const(text, "kPio2Lo")
    assert _const(text, "kPio2Lo2") == float(pi / 2 - mpmath.mpf(hi) -
                                             mpmath.mpf(lo))
    k = _const(text, "kDegPerRad")
    assert _const(text, "kDegPerRadLo") == float(180 / pi - mpmath.mpf(k))
    assert _const(text, "kLargeArg64") == 2.0 ** 29


def _const_f(text, name):
    m = re.search(rf"constexpr float {name} = ([0-9a-fx.p+-]+)f;", text)
    assert m, name
    return mpmath.mpf(float.fromhex(m.group(1)))


def _round24(v, down=False):
    """v > 0 to 24 significant bits: to nearest (ties to even), or down."""
    e = int(mpmath.floor(mpmath.log(v, 2)))
    scaled = v * mpmath.mpf(2) ** (23 - e)
    m = mpmath.floor(scaled) if down else mpmath.nint(scaled)
    return m * mpmath.mpf(2) ** (e - 23)


def test_fp32_reduction_constants(text):
    """The FP32 evaluation (16-bit storage, and FP32 storage under the FP32
    reduction flag): RN24(2/pi), pi/2 as three words rounded down (all
    positive, so -q Ci is -0 for q = 0 and a zero x keeps its sign; the first
    a multiple of 2^-23, so x - q C1 is exact below 2^16), RN24(180/pi)."""
    mpmath.mp.prec = 400
    pi = mpmath.pi
    assert _const_f(text, "kTwoOverPiF") == _round24(2 / pi)
    f1 = _const_f(text, "kPio2F1")
    f2 = _const_f(text, "kPio2F2")
    f3 = _const_f(text, "kPio2F3")
    assert f1 == _round24(pi / 2, down=True)
    assert f2 == _round24(pi / 2 - f1, down=True)
    assert f3 == _round24(pi / 2 - f1 - f2)
    assert f1 > 0 and f2 > 0 and f3 > 0
    assert (f1 * 2 ** 23) == mpmath.floor(f1 * 2 ** 23)
    assert abs(pi / 2 - f1 - f2 - f3) < mpmath.mpf(2) ** -72
    k_hi = _const_f(text, "kDegPerRadF")
    assert k_hi == _round24(180 / pi)
    assert _const_f(text, "kRoundMagicF") == 1.5 * 2 ** 23
    assert _const_f(text, "kSmall16") == 2 ** 16
    # the carried evaluation (FP32 storage under the flag): the low word of
    # 180/pi, the threshold and the 2^-12-degree grid constant
    k_lo = _const_f(text, "kDegPerRadLoF")
    assert k_lo < 0 and -k_lo == _round24(k_hi - 180 / pi)
    assert abs(180 / pi - k_hi - k_lo) < mpmath.mpf(2) ** -44
    assert _const_f(text, "kSmall32") == 2 ** 20
    assert _const_f(text, "kGridT") == 1.5 * 2 ** 11


def test_carried_reduction_exactness_conditions(text):
    """The carried FP32 reduction relies on: the first word of pi/2 a
    multiple of 2^-22 (so x - q C1 is exact for |x| < 2^20, where x is a
    multiple of 2^-22 or q is 0 or +-1); q < 2^22 (the 1.5 2^23 rounding
    gives the integer nearest x 2/pi); q times the truncation of the three
    words below 2^-52; and (t + 1.5 2^11) - 1.5 2^11 a multiple of 2^-12 for
    t in [0, 64), so that s t + i (|s| <= 13, |i| <= 1252 integers) needs at
    most 24 bits."""
    mpmath.mp.prec = 400
    pi = mpmath.pi
    f1 = _const_f(text, "kPio2F1")
    f2 = _const_f(text, "kPio2F2")
    f3 = _const_f(text, "kPio2F3")
    assert f1 * 2 ** 22 == mpmath.floor(f1 * 2 ** 22)
    q_max = int(mpmath.ceil(2 ** 20 * 2 / pi))
    assert q_max < 2 ** 22
    assert q_max * abs(pi / 2 - f1 - f2 - f3) < mpmath.mpf(2) ** -52
    grid = _const_f(text, "kGridT")
    # every sum in [grid, grid + 64) has ulp 2^-12
    assert grid >= 2 ** 11 and grid + 64 < 2 ** 12
    assert (13 * 64 + 1252) * 2 ** 12 < 2 ** 24


def test_two_over_pi_bits(text):
    mpmath.mp.prec = 400
    m = re.search(r"kTwoOverPiBits\[8\] = \{([^}]*)\}", text)
    words = [int(w.strip().rstrip("u"), 16) for w in m.group(1).split(",")]
    x = 2 / mpmath.pi
    for w in words:
        x *= 2 ** 32
        top = int(mpmath.floor(x))
        assert w == top
        x -= top


def test_two_over_pi_bits_fp64(text):
    """Word 0 is zero (bits -31..0); word w holds bits 32(w-1)+1 .. 32w; the
    table must reach the last word the reduction of the largest double
    reads (exponent 971: words up to 31 + 6)."""
    mpmath.mp.prec = 2000
    m = re.search(r"kTwoOverPiBits64\[(\d+)\] = \{([^}]*)\}", text)
    size = int(m.group(1))
    words = [int(w.strip().rstrip("u"), 16) for w in m.group(2).split(",")]
    assert len(words) == size and words[0] == 0
    x = 2 / mpmath.pi
    for w in words[1:]:
        x *= 2 ** 32
        top = int(mpmath.floor(x))
        assert w == top
        x -= top
    e_max = 2046 - 1075
    w0 = (e_max + 30) >> 5
    assert w0 + 6 < size
    assert (-23 + 30) >> 5 >= 0   # smallest exponent on the large path


def test_piece_integers_match_appendix(text, golden_dir):
    rows = read_table(os.path.join(golden_dir, "appendix_a_integer_forms.txt"))
    arrays = {}
    for name in ("kA", "kB", "kC", "kD"):
        m = re.search(rf"constexpr int {name}\[6\] = \{{([^}}]*)\}}", text)
        arrays[name] = [int(v) for v in m.group(1).split(",")]
    for row in rows:
        k = int(row[0])
        a, b, c, d = (int(v) for v in row[4:8])
        assert (arrays["kA"][k], arrays["kB"][k], arrays["kC"][k],
                arrays["kD"][k]) == (a, b, c, d)
