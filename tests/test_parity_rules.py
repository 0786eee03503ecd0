"""CPU checks of the parity rules themselves (tests/ta_check.py): planted
mistakes in oracle-derived values must be caught, legitimate neighbour-piece
values at the jump nodes must be accepted only inside the band."""
import math

import numpy as np
import pytest

import oracle
from paper_2502_10831_amd import workloads as wl
from ta_check import BAND, check_16, check_f32_counted, ulp32


def test_ulp32_definition():
    y = np.array([1.0, 1.5, 0.75, 2.0 ** -126, 2.0 ** -140, 0.0, -3.0])
    np.testing.assert_array_equal(
        ulp32(y), [2.0 ** -23, 2.0 ** -23, 2.0 ** -24, 2.0 ** -149,
                   2.0 ** -149, 2.0 ** -149, 2.0 ** -22])


def test_rule_catches_planted_errors():
    x = wl.small_uniform(4096, seed=5)
    ref = oracle.forward(x.astype(np.float64))["sin"]
    good = ref.astype(np.float32)
    w, r = check_f32_counted("sin", x, good, ref)
    assert w <= 0.5 and r == 0
    bad = good.astype(np.float64).copy()
    bad[17] = ref[17] + 5 * ulp32(ref[17])          # 5 ulp off
    with pytest.raises(AssertionError):
        check_f32_counted("sin", x, bad, ref)
    bad = good.copy()
    bad[3] = -bad[3]                                  # wrong sign
    with pytest.raises(AssertionError):
        check_f32_counted("sin", x, bad, ref)
    bad = good.copy()
    bad[9] = np.nan                                   # NaN where not due
    with pytest.raises(AssertionError):
        check_f32_counted("sin", x, bad, ref)


def test_band_accepts_neighbour_piece_only_near_nodes():
    node = math.pi / 6                                # 30 degrees: a jump
    x_in = np.array([node + 0.5 * BAND, node - 0.5 * BAND])
    x_out = np.array([node + 20 * BAND])
    for x in (x_in, x_out):
        rho, v, k, ns, nc = oracle.fold(x)
        ref = oracle.forward(x)["tan"]
        # the other piece's value (across the node)
        alt = np.array([oracle.piece_scs(int(kk) - 1 if r >= node else
                                         int(kk) + 1, r, vv)[2]
                        for kk, r, vv in zip(k, rho, v)])
        assert np.all(np.abs(alt - ref) > 100 * ulp32(ref))
        if x is x_in:
            w, r = check_f32_counted("tan", x, alt, ref)
            assert r == len(x)
        else:
            with pytest.raises(AssertionError):
                check_f32_counted("tan", x, alt, ref)


def test_16bit_rule():
    raw = wl.all_16bit_patterns()
    x = wl.decode_16(raw, "bf16")
    fin = np.isfinite(x) & (np.abs(x) < 100)
    x = x[fin]
    ref = oracle.forward(x)["cos"]
    got = wl.round_to_16(ref, "bf16")
    check_16("cos", "bf16", got, ref, 4 * ulp32(ref))
    off = got.copy()
    off[100] = off[100] + 1                           # next BF16 value
    with pytest.raises(AssertionError):
        check_16("cos", "bf16", off, ref, 4 * ulp32(ref))
