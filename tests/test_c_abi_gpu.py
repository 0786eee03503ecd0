"""The boundary used from plain C (tests/c_abi/ta_example.c: hipMalloc'd
buffers, a stream of its own, ta_sincos and ta_sin_fwdbwd, the validation
paths), run as a child process; its outputs checked against the oracle by
the same rules as the Python-driven tests."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2502_10831_amd import workloads as wl
from ta_check import U24, check_f32, neighbour_values, ulp32

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BIN = os.path.join(HERE, "c_abi", "ta_example")


def test_c_program_uses_the_abi(tmp_path):
    assert os.path.exists(BIN), \
        "tests/c_abi/ta_example is not built (run __graft_entry__.build())"
    x = wl.small_uniform((1 << 16) + 5, seed=61)
    fin, fout = tmp_path / "x.bin", tmp_path / "y.bin"
    x.astype("<f4").tofile(fin)
    print(f"[gpu] C example n={x.size}", flush=True)
    sys.stdout.flush()
    r = subprocess.run([BIN, str(fin), str(fout)], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "gfx950" in r.stdout
    y = np.fromfile(fout, "<f4").astype(np.float64).reshape(5, x.size)
    x64 = x.astype(np.float64)
    ref = oracle.forward(x64)
    near, alt = neighbour_values(x64)
    for i, name in enumerate(("sin", "cos", "tan")):
        check_f32(f"c-{name}", x, y[i], ref[name], alt, near)
    # ta_sin_fwdbwd with g = 1: the value equals ta_sincos's sin bit for bit
    assert np.array_equal(y[3], y[0])
    g = oracle.grad(x64)["sin"]
    tol = 12 * U24 * np.abs(g) + ulp32(g)
    assert ((np.abs(y[4] - g) <= tol) | near).all()
