"""bench.py pieces that need no GPU: the refusal of --gpus N > 1, the
comment-blind source hash that ties profiles to kernel sources, and the
rocprofv3 trace summary on a synthetic trace."""
import csv
import os
import subprocess
import sys

import pytest

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single" in r.stderr


def test_code_only_drops_comments_keeps_strings():
    src = ('int a = 1; // note\n/* block\n comment */ const char *s = '
           '"// kept /* kept */"; char c = \'/\';  int   b;\n')
    out = bench._code_only(src)
    assert "note" not in out and "block" not in out
    assert '"// kept /* kept */"' in out and "'/'" in out
    assert "int b;" in out
    assert bench._code_only("x = 1; // a") == bench._code_only("x  =  1;")


def test_source_hash_is_stable_and_tracks_code():
    h = bench.source_hash()
    assert len(h) == 16 and h == bench.source_hash()


def _write_trace(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size_X",
                                          "Workgroup_Size_X",
                                          "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        w.writerows(rows)


def test_trace_summary_on_a_synthetic_trace(tmp_path):
    name = ("void ta::map_vec_kernel<ta::F32, ta::FwdOp<7, false, false, "
            "false, false>, 64, 4, false, true, 1, true, true>(ta::IoPtrs, "
            "long, long, long)")
    grid = (1 << 28) // 16   # 64-thread groups, four 16-byte vectors a thread
    rows, t = [], 0
    warm, steps = 1733, bench.HEADLINE_STEPS   # a time-based warm-up count
    copy = "void ta::map_vec_kernel<ta::F32, ta::CopyOp<1, 3>, 64, 1, false, true, 1>"
    for i in range(warm + steps + 10):
        if i == warm + steps:   # the copy ceiling runs next, then more calls
            rows.append({"Kernel_Name": copy, "Grid_Size_X": grid,
                         "Workgroup_Size_X": 64,
                         "Start_Timestamp": t, "End_Timestamp": t + 900_000})
            t += 901_000
        dur = 800_000 if i < warm or i >= warm + steps else 700_000
        rows.append({"Kernel_Name": name, "Grid_Size_X": grid,
                     "Workgroup_Size_X": 64,
                     "Start_Timestamp": t, "End_Timestamp": t + dur})
        t += dur + 1000
    # dispatches of the same kernel at another size are not counted: another
    # grid, or the same grid in 256-thread groups (2^26 elements, one vector
    # a thread)
    rows.append({"Kernel_Name": name, "Grid_Size_X": 1024,
                 "Workgroup_Size_X": 64,
                 "Start_Timestamp": t, "End_Timestamp": t + 5})
    small = name.replace("64, 4, false, true, 1, true, true",
                         "256, 1, false, true, 1, false, false")
    rows.append({"Kernel_Name": small, "Grid_Size_X": grid,
                 "Workgroup_Size_X": 256,
                 "Start_Timestamp": t + 10, "End_Timestamp": t + 150_000})
    _write_trace(str(tmp_path / "trace" / "run_kernel_trace.csv"), rows)
    out = str(tmp_path / "summary.txt")
    bench.summarize(["trace", str(tmp_path / "trace"), out, "cmd"])
    text = open(out).read()
    assert (f"sincos_tan_f32: grid {grid} workgroup 64 "
            f"calls {warm + steps + 10}") in text
    assert (f"sincos_tan_f32_headline_timed: the last {steps} of the first "
            f"{warm + steps} back-to-back dispatches, average_ns 700000") in text
    assert f"source_sha: {bench.source_hash()}" in text


def test_error_helpers_match_the_format_ulps():
    """bench._ulp_of gives the spacing of the binary format at |y| (FP32,
    BF16, FP16 and FP64 parameters against numpy's own spacing), and
    _err_stats reports max |got - ref| and its size in those ulps."""
    import numpy as np
    rng = np.random.default_rng(5)
    y = np.concatenate([rng.uniform(-4, 4, 1000), [1.0, 0.5, 2.0 ** -130]])
    for dt, mant, emin in ((np.float32, 23, -126), (np.float16, 10, -14),
                           (np.float64, 52, -1022)):
        yd = y.astype(dt)
        want = np.spacing(np.abs(yd)).astype(np.float64)
        got = bench._ulp_of(yd.astype(np.float64), mant, emin)
        keep = np.abs(yd) > 0
        np.testing.assert_array_equal(got[keep], want[keep])
    # BF16: 7 stored bits, FP32's exponent range
    assert bench._ulp_of(np.array([1.0, 3.0]), 7, -126).tolist() == [2.0 ** -7, 2.0 ** -6]
    ref = np.array([1.0, -0.75, np.nan, 0.25])
    got = np.array([1.0 + 2.0 ** -22, -0.75, np.nan, 0.25 - 2.0 ** -26])
    st = bench._err_stats(got, ref, 23, -126)
    assert st["max_abs"] == 2.0 ** -22
    assert st["max_ulp"] == 2.0


def test_interleaved_alternates_blocks_and_takes_the_median_ratio():
    """bench.interleaved times its two launch sequences in alternating
    blocks (ten untimed launches, then the timed ones) and returns per-block
    ms per launch and the median of time(b) / time(a)."""
    calls, clock = [], [0.0]

    class FakeEvent:
        def __init__(self, enable_timing=False):
            self.t = None

        def record(self):
            self.t = clock[0]

        def elapsed_time(self, end):
            return end.t - self.t

    class Cuda:
        Event = FakeEvent

        @staticmethod
        def synchronize():
            pass

    class Torch:
        cuda = Cuda

    cost = {"a": [1.0, 1.0, 2.0], "b": [1.25, 1.5, 2.0]}
    rnd = {"a": 0, "b": 0}

    def launcher(name):
        def fn():
            calls.append(name)
            clock[0] += cost[name][rnd[name] // 14]
            rnd[name] += 1
        return fn

    ta_ms, tb_ms, ratio = bench.interleaved(launcher("a"), launcher("b"), 3, 4,
                                            Torch)
    assert calls == (["a"] * 14 + ["b"] * 14) * 3
    assert ta_ms == [1.0, 1.0, 2.0] and tb_ms == [1.25, 1.5, 2.0]
    assert ratio == 1.25   # ratios 1.0, 1.25, 1.5


def test_valu_model_reads_both_summaries(tmp_path, monkeypatch):
    """bench.valu_cycles_per_elem combines the instruction counts of the two
    SQ summaries with the per-class cycle costs: FP32 arithmetic 2 (4 in the
    upper bound), FP64 arithmetic, conversions and INT64 4, FP32
    transcendentals 8, the remaining instructions 3 (2 to 4); summaries of
    other kernel sources give None."""
    sha = bench.source_hash()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / bench.SQ_SUMMARY).write_text(
        f"source_sha: {sha}\n"
        "k_SQ_INSTS_VALU: 1 per_elem 40.00\n"
        "k_SQ_INSTS_VALU_FMA_F64: 1 per_elem 6.00\n"
        "k_SQ_INSTS_VALU_CVT: 1 per_elem 4.00\n")
    classes = {"FMA_F32": 10, "ADD_F32": 2, "MUL_F32": 4, "TRANS_F32": 1,
               "ADD_F64": 1, "MUL_F64": 3, "INT64": 0}
    (prof / bench.SQ_CLASS_SUMMARY).write_text(
        f"source_sha: {sha}\n" + "".join(
            f"k_SQ_INSTS_VALU_{c}: 1 per_elem {v:.2f}\n" for c, v in classes.items()))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: sha)
    # f32 16, trans 1, 4-cycle 6 + 1 + 3 + 4 + 0 = 14, rest 40 - 31 = 9
    mid, lo, hi = bench.valu_cycles_per_elem("k")
    assert (mid, lo, hi) == ((56 + 8 + 32 + 27) / 64, (56 + 8 + 32 + 18) / 64,
                             (56 + 8 + 64 + 36) / 64)
    r = bench.valu_roofline("k", 1e12)
    assert r["bound"] == "alu" and r["valu_per_elem"] == 40.0
    assert r["frac"] == round(1e12 * mid / bench.SIMD_CYCLES_PER_S, 3)
    assert r["frac_range"][0] < r["frac"] < r["frac_range"][1]
    assert bench.valu_cycles_per_elem("other") is None
    monkeypatch.setattr(bench, "source_hash", lambda: "0" * 16)
    assert bench.valu_cycles_per_elem("k") is None


def test_every_profiled_kernel_has_rows_in_the_committed_summaries():
    """Each kernel `bench.py --profile` dispatches is named in every committed
    counter summary: a kernel whose name no longer matches its pattern in
    bench.KERNELS (a renamed storage type, say) would drop out of the
    traffic, instruction and stall summaries without an error."""
    prof = os.path.join(bench.ROOT, "profiles")
    for fname, suffix in (("ta_sincos_tan_f32_2p28_pmc.txt",
                           "_traffic_over_algorithmic:"),
                          (bench.SQ_SUMMARY, "_SQ_INSTS_VALU:"),
                          (bench.SQ_CLASS_SUMMARY, "_SQ_INSTS_VALU_FMA_F32:"),
                          ("ta_kernels_f32_bf16_f64_stall_counters.txt",
                           "_SQ_WAVE_CYCLES:")):
        text = open(os.path.join(prof, fname)).read()
        for key in bench.KERNELS:
            if key == "copy_1to1_f32" and "traffic" in suffix:
                continue   # the calibration copy itself
            assert f"\n{key}{suffix}" in text, (fname, key)
