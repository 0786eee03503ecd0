"""GPU parity: the HIP kernels (through the C ABI) against the FP64 oracle,
element by element on seeded inputs.  Rules in tests/ta_check.py."""
import math
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2502_10831_amd as ta
from paper_2502_10831_amd import workloads as wl
from ta_check import (U24, check_16, check_f32, check_f32_counted, grad_bad,
                      neighbour_grads, neighbour_values, ulp32, ulp_error)

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ta.load()
    return torch.device("cuda:0")


def to_dev(a, dev, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev).view(dtype) \
        if a.dtype == np.uint16 else torch.from_numpy(
            np.ascontiguousarray(a)).to(dev)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def run_forward(x_dev):
    """All forward entry points on one input; returns dict of numpy arrays."""
    out = {}
    for name, fn in (("sin", ta.ta_sin), ("cos", ta.ta_cos),
                     ("tan", ta.ta_tan)):
        y = torch.empty_like(x_dev)
        fn(x_dev, y)
        out[name] = host(y)
    ys, yc, yt = (torch.empty_like(x_dev) for _ in range(3))
    ta.ta_sincos(x_dev, ys, yc, yt)
    out["f3_sin"], out["f3_cos"], out["f3_tan"] = host(ys), host(yc), host(yt)
    ys2, yc2 = torch.empty_like(x_dev), torch.empty_like(x_dev)
    ta.ta_sincos(x_dev, ys2, yc2, None)
    out["f2_sin"], out["f2_cos"] = host(ys2), host(yc2)
    return out


def check_all_f32(x, out, label, quiet=False):
    """Every output in `out` against the oracle; the outputs are checked in
    parallel threads (numpy releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    ref = oracle.forward(x.astype(np.float64))
    keys = [k for k in ("sin", "cos", "tan", "f3_sin", "f3_cos", "f3_tan",
                        "f2_sin", "f2_cos") if k in out]

    def one(key):
        w, r = check_f32_counted(f"{label}:{key}", x, out[key],
                                 ref[key.split("_")[-1]])
        return key, w, r

    with ThreadPoolExecutor(max_workers=4) as pool:
        results = list(pool.map(one, keys))
    worst = {k: w for k, w, _ in results}
    rescued = sum(r for _, _, r in results)
    if not quiet:
        say(f"{label}: max ulp {worst}; inputs that matched only the "
            f"neighbouring piece across a jump node: {rescued}")
    return worst


# ---------------------------------------------------------------------------
# forward, FP32
# ---------------------------------------------------------------------------

def test_forward_small_uniform(dev):
    n = (1 << 20) + 3   # several tiles and a ragged tail
    say(f"forward small uniform n={n}")
    x = wl.small_uniform(n)
    out = run_forward(to_dev(x, dev))
    check_all_f32(x, out, "U[-2pi,2pi]")
    # the fused kernels compute bit-identical values to the single ones
    for k in ("sin", "cos", "tan"):
        assert np.array_equal(out[k].view(np.uint32),
                              out["f3_" + k].view(np.uint32))


def _sweep_bits(dev, hi, flags, label, step=1):
    """Every `step`-th FP32 bit pattern in [0, hi] and its negation through
    the fused sin+cos+tan kernel, every output against the oracle.  2^26
    patterns (2^27 values, 512 MiB) per launch: the full launches run the
    vector body the library uses for inputs above 256 MiB (the grouped
    four-vector form of the default evaluation), the last, partial one the
    body used below."""
    chunk = 1 << 26
    worst = {}
    total = 0
    for start in range(0, int(hi) + 1, chunk * step):
        bits = np.arange(start, min(start + chunk * step, int(hi) + 1), step,
                         dtype=np.uint64).astype(np.uint32)
        x = bits.view(np.float32)
        x = np.concatenate([x, -x])
        say(f"{label}: chunk start=0x{start:08x} n={x.size}")
        xd = to_dev(x, dev)
        ys, yc, yt = (torch.empty_like(xd) for _ in range(3))
        ta.ta_sincos_ex(xd, ys, yc, yt, flags)
        out = {"f3_sin": host(ys), "f3_cos": host(yc), "f3_tan": host(yt)}
        w = check_all_f32(x, out, label, quiet=True)
        for k, v in w.items():
            worst[k] = max(worst.get(k, 0.0), v)
        total += x.size
    say(f"{label}: {total} values, max ulp {worst}")
    return worst


def test_forward_every_fp32_in_0_2pi(dev):
    """The brute-force pin: every FP32 in [0, 2 pi] and its negation (2.2e9
    values), default evaluation.  With TA_EXHAUSTIVE=all, every finite
    FP32 instead."""
    hi = np.float32(2 * math.pi).view(np.uint32)
    if os.environ.get("TA_EXHAUSTIVE", "") == "all":
        hi = np.uint32(0x7F7FFFFF)
    _sweep_bits(dev, hi, 0, "every FP32 in [-2pi, 2pi]")


def test_carried_fp32_every_input_below_2p20(dev):
    """TA_FLAG_FORCE_FP32_REDUCTION (the carried FP32 evaluation, which holds
    below 2^20): every FP32 with |x| < 2^20 (2.5e9 values) within 4 ulp of
    the formula."""
    hi = np.uint32(np.float32(2.0 ** 20).view(np.uint32) - 1)
    _sweep_bits(dev, hi, ta.TA_FLAG_FORCE_FP32_REDUCTION,
                "carried FP32, every |x| < 2^20")


def test_forward_wide_strided_sweep(dev):
    """Every 127th FP32 from 2 pi up to the largest finite float, and the
    negations (~17M values): the two-word and the bit-table reductions."""
    lo = int(np.float32(2 * math.pi).view(np.uint32))
    hi = 0x7F7FFFFF
    step = 127
    chunk = 1 << 24
    worst = {}
    for start in range(lo, hi + 1, chunk * step):
        bits = np.arange(start, min(start + chunk * step, hi + 1), step,
                         dtype=np.uint64).astype(np.uint32)
        x = bits.view(np.float32)
        x = np.concatenate([x, -x])
        say(f"wide sweep chunk start=0x{start:08x} n={x.size}")
        xd = to_dev(x, dev)
        ys, yc, yt = (torch.empty_like(xd) for _ in range(3))
        ta.ta_sincos(xd, ys, yc, yt)
        w = check_all_f32(x, {"f3_sin": host(ys), "f3_cos": host(yc),
                              "f3_tan": host(yt)}, "wide")
        for k, v in w.items():
            worst[k] = max(worst.get(k, 0.0), v)
    say(f"wide sweep max ulp {worst}")


@pytest.mark.parametrize("tdt", [torch.float32, torch.bfloat16, torch.float64])
def test_graph_capture_replays(dev, tdt):
    """The launch is capturable: replay a captured ta_sincos and a fused
    forward+backward several times, with eager work between replays, and
    compare every replay bit for bit with the eager result."""
    x = wl.small_uniform((1 << 16) + 3, seed=101)
    xd = torch.from_numpy(x).to(dev).to(tdt)
    gd = torch.ones_like(xd)
    outs = [torch.empty_like(xd) for _ in range(5)]

    def launch():
        ta.ta_sincos(xd, outs[0], outs[1], outs[2])
        ta.ta_sin_fwdbwd(xd, gd, outs[3], outs[4])

    launch()
    torch.cuda.synchronize()
    eager = [t.clone() for t in outs]
    say(f"graph capture {tdt}")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        launch()
    for rep in range(4):
        for t in outs:
            t.fill_(float(rep + 7))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for t, e in zip(outs, eager):
            assert torch.equal(t, e), (tdt, rep)


def test_concurrent_host_threads(dev):
    """Calls from several host threads on their own streams, FP32, BF16
    and FP64 kernels at once; each result equals the same call made alone."""
    import threading
    dts = [torch.float32, torch.bfloat16, torch.float64, torch.float32]
    xs = [torch.from_numpy(wl.small_uniform(1 << 18, seed=110 + i)).to(dev)
          .to(dts[i]) for i in range(4)]
    alone = []
    for xd in xs:
        y = torch.empty_like(xd)
        ta.ta_sin(xd, y)
        alone.append(y)
    torch.cuda.synchronize()
    outs = [None] * 4
    errors = []

    def work(i):
        try:
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                y = torch.empty_like(xs[i])
                for _ in range(20):
                    ta.ta_sin(xs[i], y)
                stream.synchronize()
                outs[i] = y
        except Exception as e:  # reported below
            errors.append(e)

    say("concurrent host threads")
    threads = [threading.Thread(target=work, args=(i,)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for o, a in zip(outs, alone):
        assert torch.equal(o, a)


def test_forward_throughput_mix_full_size(dev):
    """The benchmark workload (2^28 FP32, 1% near the poles) in the
    benchmark's launch: every element against the oracle in 2^24-element
    chunks, and the identities S^2 + C^2 = 1, T = S/C on every element."""
    n = 1 << 28
    say(f"throughput mix n={n}: generating inputs")
    x = wl.throughput_mix(n)
    xd = to_dev(x, dev)
    ys, yc, yt = (torch.empty_like(xd) for _ in range(3))
    say("ta_sincos with tan")
    ta.ta_sincos(xd, ys, yc, yt)
    torch.cuda.synchronize()
    chunk = 1 << 24
    worst = {}
    for lo in range(0, n, chunk):
        sl = slice(lo, lo + chunk)
        w = check_all_f32(x[sl], {"f3_sin": host(ys[sl]),
                                  "f3_cos": host(yc[sl]),
                                  "f3_tan": host(yt[sl])}, f"mix[{lo}:]")
        worst = {k: max(v, worst.get(k, 0.0)) for k, v in w.items()}
    say(f"throughput mix, every element: max ulp {worst}")
    s64, c64, t64 = ys.double(), yc.double(), yt.double()
    # |S|,|C| <= 1 and each within 4 ulp of the formula: S^2 + C^2 - 1 is at
    # most 2*(4+4) * 2^-24 in magnitude
    dev_id = (s64 * s64 + c64 * c64 - 1.0).abs().max().item()
    assert dev_id < 16 * U24, dev_id
    rel = ((t64 - s64 / c64).abs() / (s64 / c64).abs().clamp_min(1e-30)).max()
    assert rel.item() < 24 * U24, rel.item()
    del s64, c64, t64


@pytest.mark.parametrize("flags", [0, ta.TA_FLAG_FORCE_FP32_REDUCTION])
def test_forward_log_magnitude(dev, flags):
    """2^26 FP32 with |x| = 10^U[0,6] and random sign (the precision
    workload that exercises the reduction of large arguments): every element
    of the fused sin+cos+tan output against the oracle in 2^24-element
    chunks, with the default evaluation and with the carried FP32 one."""
    n = 1 << 26
    say(f"log magnitude n={n} flags={flags}")
    x = wl.log_magnitude(n)
    xd = to_dev(x, dev)
    ys, yc, yt = (torch.empty_like(xd) for _ in range(3))
    ta.ta_sincos_ex(xd, ys, yc, yt, flags)
    torch.cuda.synchronize()
    worst = {}
    chunk = 1 << 24
    for lo in range(0, n, chunk):
        sl = slice(lo, lo + chunk)
        w = check_all_f32(x[sl], {"f3_sin": host(ys[sl]),
                                  "f3_cos": host(yc[sl]),
                                  "f3_tan": host(yt[sl])}, "log-magnitude")
        for k, v in w.items():
            worst[k] = max(worst.get(k, 0.0), v)
    say(f"log magnitude flags={flags}: every element, max ulp {worst}")


def _closest_to_multiples_of_half_pi(count=64):
    """FP32 values in (1, 2^20) closest to multiples of pi/2 (brute force
    over the quotients, in FP64 then refined with the oracle's fold)."""
    q = np.arange(1, 667544, dtype=np.float64)
    c = q * (math.pi / 2)
    f = c.astype(np.float32)
    cand = np.concatenate([f, np.nextafter(f, np.float32(np.inf)),
                           np.nextafter(f, np.float32(0))])
    rho, v, _, _, _ = oracle.fold(cand.astype(np.float64))
    d = np.minimum(rho, v)
    return cand[np.argsort(d)[:count]]


def test_forward_hard_inputs(dev):
    """Worst-case reductions, node neighbourhoods, specials, subnormals."""
    worst = _closest_to_multiples_of_half_pi()
    nodes = (np.arange(-400, 400)[:, None] * (math.pi / 2) +
             np.array([k * math.pi / 12 for k in range(1, 6)])[None, :]).ravel()
    nf = nodes.astype(np.float32)
    near_nodes = np.concatenate([nf, np.nextafter(nf, np.float32(np.inf)),
                                 np.nextafter(nf, np.float32(-np.inf))])
    specials = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-45, -1e-45,
                         1e-40, -3e-39, 1.1754942e-38, 1e-30, -1e-20,
                         3.4028235e38, -3.4028235e38, 0.7853982, 0.7853981,
                         1.5707964, 1.5707963, 3.1415927, 4.712389,
                         252.898209, 2.0 ** 29, -(2.0 ** 29), 2.0 ** 29 - 32,
                         1e6, -1e6], np.float32)
    rng = np.random.default_rng(5)
    big = rng.integers(0x4e000000, 0x7f800000, 200000,
                       dtype=np.uint64).astype(np.uint32).view(np.float32)
    big = np.concatenate([big, -big])
    x = np.concatenate([worst, -worst, near_nodes, specials, big])
    say(f"hard inputs n={x.size}")
    out = run_forward(to_dev(x, dev))
    check_all_f32(x, out, "hard")


def test_alignment_tails_and_canaries(dev):
    rng = np.random.default_rng(3)
    base = rng.uniform(-50, 50, 5000).astype(np.float32)
    ref = oracle.forward(base.astype(np.float64))
    xd_all = to_dev(base, dev)
    sentinel = 12345.0
    for n in (0, 1, 2, 3, 4, 5, 7, 8, 9, 31, 33, 1023, 1025, 4097):
        for xo in (0, 1, 2, 3):
            for yo in (0, 1, 3):
                say(f"align n={n} xoff={xo} yoff={yo}")
                y_all = torch.full((n + 16,), sentinel, device=dev)
                xs = xd_all[xo:xo + n]
                ys = y_all[4 + yo:4 + yo + n]
                ta.ta_sin(xs, ys)
                y = host(y_all)
                assert np.all(y[:4 + yo] == sentinel)
                assert np.all(y[4 + yo + n:] == sentinel)
                if n:
                    err = ulp_error(y[4 + yo:4 + yo + n], ref["sin"][xo:xo + n])
                    assert err.max() <= 4.0


def test_in_place(dev):
    x = wl.small_uniform(10001, seed=9)
    ref = oracle.forward(x.astype(np.float64))
    for name, fn in (("sin", ta.ta_sin), ("cos", ta.ta_cos),
                     ("tan", ta.ta_tan)):
        say(f"in place {name}")
        xd = to_dev(x, dev)
        fn(xd, xd)
        assert ulp_error(host(xd), ref[name]).max() <= 4.0


def test_tan_guard(dev):
    x = wl.throughput_mix(1 << 16, seed=13)
    xd = to_dev(x, dev)
    say("tan guard")
    y0, y1 = torch.empty_like(xd), torch.empty_like(xd)
    ta.ta_tan_ex(xd, y0, 0)
    ta.ta_tan_ex(xd, y1, ta.TA_FLAG_TAN_GUARD)
    ref = oracle.forward(x.astype(np.float64), flags=oracle.TAN_GUARD)["tan"]
    g0, g1 = host(y0), host(y1)
    guarded = np.isinf(ref)
    assert guarded.sum() > 100
    assert np.all(np.isposinf(g1[guarded]))
    assert np.array_equal(g1[~guarded].view(np.uint32),
                          g0[~guarded].view(np.uint32))
    ys, yc, yt = (torch.empty_like(xd) for _ in range(3))
    ta.ta_sincos_ex(xd, ys, yc, yt, ta.TA_FLAG_TAN_GUARD)
    assert np.array_equal(host(yt).view(np.uint32), g1.view(np.uint32))


# ---------------------------------------------------------------------------
# forward, 16-bit storage: every pattern
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_forward_16bit_exhaustive(dev, kind):
    tdt = torch.float16 if kind == "f16" else torch.bfloat16
    raw = wl.all_16bit_patterns()
    x64 = wl.decode_16(raw, kind)
    say(f"16-bit exhaustive {kind}")
    xd = torch.from_numpy(raw.view(np.int16)).to(dev).view(tdt)
    ref = oracle.forward(x64)
    near, alt = neighbour_values(x64)
    outs = {}
    for name, fn in (("sin", ta.ta_sin), ("cos", ta.ta_cos),
                     ("tan", ta.ta_tan)):
        y = torch.empty_like(xd)
        fn(xd, y)
        outs[name] = host(y.view(torch.int16)).view(np.uint16)
    ys, yc, yt = (torch.empty_like(xd) for _ in range(3))
    ta.ta_sincos(xd, ys, yc, yt)
    for name, t in (("sin", ys), ("cos", yc), ("tan", yt)):
        fused = host(t.view(torch.int16)).view(np.uint16)
        assert np.array_equal(fused, outs[name])
        check_16(name, kind, outs[name], ref[name], 4 * ulp32(ref[name]),
                 alt, near)


@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_forward_16bit_full_size(dev, kind):
    """2^29 16-bit inputs U[-pi, pi] in the benchmark launch: every output
    equals the exhaustive table entry of its input pattern."""
    tdt = torch.float16 if kind == "f16" else torch.bfloat16
    table_in = torch.from_numpy(
        wl.all_16bit_patterns().view(np.int16)).to(dev).view(tdt)
    tabs, tabc, tabt = (torch.empty_like(table_in) for _ in range(3))
    ta.ta_sincos(table_in, tabs, tabc, tabt)
    n = 1 << 29
    say(f"16-bit full size {kind} n={n}")
    gen = torch.Generator(device=dev).manual_seed(wl.SEED)
    x = (torch.rand(n, device=dev, generator=gen, dtype=torch.float64)
         * (2 * math.pi) - math.pi).to(tdt)
    ys, yc, yt = (torch.empty_like(x) for _ in range(3))
    ta.ta_sincos(x, ys, yc, yt)
    idx = x.view(torch.int16).long() & 0xFFFF
    for out, tab in ((ys, tabs), (yc, tabc), (yt, tabt)):
        expect = tab.view(torch.int16)[idx]
        assert torch.equal(out.view(torch.int16), expect)
    torch.cuda.synchronize()


def test_max_size_beyond_2_31_elements(dev):
    """n = 2^31 + 123 BF16 (4 GiB per array): element indices past 2^31 use
    the 64-bit paths; every output equals the exhaustive table entry of its
    input pattern.  Then n = 2^31 + 3 FP32 with the scalar tail: the last
    elements and a random sample against the oracle."""
    n = (1 << 31) + 123
    say(f"max size BF16 n={n}")
    table_in = torch.from_numpy(
        wl.all_16bit_patterns().view(np.int16)).to(dev).view(torch.bfloat16)
    tab = torch.empty_like(table_in)
    ta.ta_sin(table_in, tab)
    gen = torch.Generator(device=dev).manual_seed(131)
    raw = torch.randint(-32768, 32768, (n,), device=dev, generator=gen,
                        dtype=torch.int16)
    x = raw.view(torch.bfloat16)
    y = torch.empty_like(x)
    ta.ta_sin(x, y)
    for lo in range(0, n, 1 << 30):   # check in 1 Gi-element slices
        hi = min(n, lo + (1 << 30))
        idx = raw[lo:hi].long() & 0xFFFF
        assert torch.equal(y[lo:hi].view(torch.int16),
                           tab.view(torch.int16)[idx]), (lo, hi)
        del idx
    del raw, x, y
    torch.cuda.synchronize()
    n = (1 << 31) + 3
    say(f"max size FP32 n={n}")
    x = torch.rand(n, device=dev, generator=gen) * 200.0 - 100.0
    y = torch.empty_like(x)
    ta.ta_sin(x, y)
    torch.cuda.synchronize()
    sample = np.concatenate([np.arange(n - 4096, n),
                             np.random.default_rng(5).integers(0, n, 1 << 16)])
    it = torch.from_numpy(sample).to(dev)
    xs, ys = host(x[it]), host(y[it])
    check_f32("max-size:sin", xs, ys, oracle.forward(xs.astype(np.float64))["sin"])
    del x, y


@pytest.mark.parametrize("kind", ["f32", "bf16", "f64"])
def test_single_output_load_policy_threshold(dev, kind):
    """Inputs of at most 256 MiB in all are read with plain loads, larger
    ones with the shape's nontemporal loads (and FP32 sin+cos+tan in the
    grouped four-vector kernel): on both sides of that
    size, ta_sin, ta_cos and ta_tan, and ta_sincos without tan, give the
    bits of the sin, cos and tan outputs of ta_sincos on the same input
    (the same arithmetic), and the Taylor sine, the two- and three-input
    backward and the fused forward and backward give the same bits below
    and above the size for a shared prefix."""
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f64": torch.float64}[kind]
    iv = {"f32": torch.int32, "bf16": torch.int16, "f64": torch.int64}[kind]
    esz = torch.tensor([], dtype=tdt).element_size()
    limit = (256 << 20) // esz
    gen = torch.Generator(device=dev).manual_seed(977)
    big = (torch.rand(limit + 37, device=dev, generator=gen, dtype=torch.float64)
           * 2e3 - 1e3).to(tdt)
    tay = {}
    for n in (limit - 5, limit, limit + 37):
        say(f"load policy {kind} n={n}")
        x = big[:n]
        ys, yc, yt = (torch.empty_like(x) for _ in range(3))
        ta.ta_sincos(x, ys, yc, yt)
        for fn, ref in ((ta.ta_sin, ys), (ta.ta_cos, yc), (ta.ta_tan, yt)):
            y = torch.empty_like(x)
            fn(x, y)
            torch.cuda.synchronize()
            assert torch.equal(y.view(iv), ref.view(iv)), (kind, n, fn.__name__)
        ys2, yc2 = torch.empty_like(x), torch.empty_like(x)
        ta.ta_sincos(x, ys2, yc2, None)
        torch.cuda.synchronize()
        assert torch.equal(ys2.view(iv), ys.view(iv)), (kind, n, "sin of two")
        assert torch.equal(yc2.view(iv), yc.view(iv)), (kind, n, "cos of two")
        if kind == "f32":   # the tan guard through the fused kernels too
            yg = torch.empty_like(x)
            ta.ta_tan_ex(x, yg, ta.TA_FLAG_TAN_GUARD)
            ta.ta_sincos_ex(x, ys2, yc2, yt, ta.TA_FLAG_TAN_GUARD)
            torch.cuda.synchronize()
            assert torch.equal(yt.view(iv), yg.view(iv)), (kind, n, "guard")
            assert torch.equal(ys2.view(iv), ys.view(iv)), (kind, n, "guard sin")
            del yg
        del ys2, yc2
        yt5 = torch.empty_like(x)
        ta.ta_taylor_sin(x, yt5, 5)
        tay[n] = yt5[: limit - 5]
        del ys, yc, yt
    assert torch.equal(tay[limit - 5].view(iv), tay[limit + 37].view(iv))
    assert torch.equal(tay[limit].view(iv), tay[limit + 37].view(iv))
    del tay
    # two and three inputs: the size counts all of them; the backward of a
    # prefix gives the same bits below and above it
    g1 = (torch.rand(limit + 37, device=dev, generator=gen,
                     dtype=torch.float64) * 2 - 1).to(tdt)
    g2 = g1.flip(0)
    for nin, fn, args in ((2, ta.ta_sin_bwd, (g1,)), (3, ta.ta_sincos_bwd, (g1, g2))):
        lim = limit // nin
        outs = {}
        for n in (lim - 5, lim + 37):
            say(f"load policy {kind} {nin} inputs n={n}")
            gx = torch.empty(n, device=dev, dtype=tdt)
            fn(big[:n], *(a[:n] for a in args), gx)
            outs[n] = gx
        torch.cuda.synchronize()
        assert torch.equal(outs[lim - 5].view(iv), outs[lim + 37][: lim - 5].view(iv)), nin
    # the fused forward and backward (two inputs, two outputs; 16-bit
    # storage changes its access width at the size): the same bits below
    # and above it
    lim = limit // 2
    fb = {}
    for n in (lim - 5, lim + 37):
        say(f"load policy {kind} fused forward+backward n={n}")
        y, gx = (torch.empty(n, device=dev, dtype=tdt) for _ in range(2))
        ta.ta_sin_fwdbwd(big[:n], g1[:n], y, gx)
        fb[n] = (y, gx)
    torch.cuda.synchronize()
    for a, b in zip(fb[lim - 5], fb[lim + 37]):
        assert torch.equal(a.view(iv), b[: lim - 5].view(iv)), "fwdbwd"
    del big, g1, g2, fb


@pytest.mark.parametrize("off", [1, 3])
def test_grouped_kernel_shared_misalignment(dev, off):
    """FP32 sin+cos+tan on more than 256 MiB of input runs the grouped
    four-vector kernel.  With the input and the outputs (of sin+cos+tan,
    and of sin+cos) all `off` elements past a 16-byte boundary (a scalar
    head of 4 - off elements, the 16-byte body ending in a partial
    workgroup, a scalar tail), every element equals that of the same call
    on aligned buffers (and sin+cos those of sin+cos+tan), and the ends
    plus 2^20 elements spread over the array are within the FP32 rule of
    the oracle."""
    n = (256 << 20) // 4 + 1037
    gen = torch.Generator(device=dev).manual_seed(979)
    x = (torch.rand(n, device=dev, generator=gen, dtype=torch.float64)
         * 2e3 - 1e3).to(torch.float32)
    say(f"grouped kernel shared misalignment off={off} n={n}")

    def at_offset(t=None):
        buf = torch.empty(n + off, device=dev)
        assert buf.data_ptr() % 16 == 0
        if t is not None:
            buf[off:].copy_(t)
        return buf[off:]

    ref = [torch.empty_like(x) for _ in range(3)]
    ta.ta_sincos(x, *ref)
    outs = [at_offset() for _ in range(3)]
    ta.ta_sincos(at_offset(x), *outs)
    torch.cuda.synchronize()
    for a, b in zip(ref, outs):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32)), off
    two = [at_offset() for _ in range(2)]
    ta.ta_sincos(at_offset(x), two[0], two[1], None)
    torch.cuda.synchronize()
    for a, b in zip(ref, two):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32)), (off, 2)
    del two
    idx = np.unique(np.concatenate([
        np.arange(4096), np.arange(n - 4096, n),
        np.linspace(0, n - 1, 1 << 20).astype(np.int64)]))
    got = {k: host(t)[idx] for k, t in zip(("f3_sin", "f3_cos", "f3_tan"), outs)}
    check_all_f32(host(x)[idx], got, f"grouped off={off}")
    del x, ref, outs


# ---------------------------------------------------------------------------
# Taylor baseline
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("terms", [5, 7, 9])
def test_taylor(dev, terms):
    """Taylor-5/7/9 on the 2^20-element U[-2pi, 2pi] workload, every
    element, plus a ragged tail of 5."""
    x = np.concatenate([wl.small_uniform(1 << 20),
                        wl.small_uniform(5, seed=21)])
    xd = to_dev(x, dev)
    say(f"taylor terms={terms}")
    ref = oracle.taylor(x.astype(np.float64), terms)
    for name, fn in (("sin", ta.ta_taylor_sin), ("cos", ta.ta_taylor_cos),
                     ("tan", ta.ta_taylor_tan)):
        y = torch.empty_like(xd)
        fn(xd, y, terms)
        g = host(y).astype(np.float64)
        # FP32 Horner on rho^2 with rho rounded once: error bound
        # (4N + 2) u * sum|terms|  (u = 2^-24), plus the output rounding
        tol = (4 * terms + 2) * U24 * ref["abs_" + name] + ulp32(ref[name])
        bad = np.abs(g - ref[name]) > tol
        assert not bad.any(), (name, x[bad][:3], g[bad][:3], ref[name][bad][:3])


# ---------------------------------------------------------------------------
# backward and fused forward+backward
# ---------------------------------------------------------------------------

# FP32 storage: omega (4 roundings), the output (2.5 ulp) and g; a host build
# of the arithmetic over every FP32 in [2^-31, 2^16) and a 1/101 sample
# above peaks at 7.5 u (relative) before the product with g.
GRAD_ULPS = 12
# 16-bit storage: the unrefined inverse square root and reciprocal (each
# within an FP32 ulp) enter omega = kdet y^2 twice and the output once; a
# host build of the arithmetic over every FP16 and BF16 input, with the
# estimates pushed an ulp either way, peaks at 12.6 u (relative) before the
# product with g (0.5 u more) and the rounding to 16 bits.
GRAD_ULPS_16 = 14


def _grad_case(n, sigma, seed):
    x, g = wl.normal_pair((n,), sigma, seed=seed)
    return x, g


def _check_grad(name, x, g, gx, ref_grad, grad_near=None):
    """gx = g * d f/dx within GRAD_ULPS FP32 roundings of its size (plus
    one ulp); in the jump-node band the derivative of either neighbouring
    piece."""
    g64 = g.astype(np.float64)
    ref = g64 * ref_grad
    near, alt_grad = grad_near or neighbour_grads(x.astype(np.float64))
    alt = g64 * alt_grad[name]
    bad = grad_bad(gx, ref, GRAD_ULPS * U24 * np.abs(ref) + ulp32(ref), near,
                   alt, GRAD_ULPS * U24 * np.abs(alt) + ulp32(alt))
    assert not bad.any(), (name, x[bad][:3], gx[bad][:3], ref[bad][:3])


def test_backward_f32(dev):
    n = (1 << 20) + 7
    x, g = _grad_case(n, 3.0, 31)
    say(f"backward f32 n={n}")
    xd, gd = to_dev(x, dev), to_dev(g, dev)
    rg = oracle.grad(x.astype(np.float64))
    rf = oracle.forward(x.astype(np.float64))
    grad_near = neighbour_grads(x.astype(np.float64))
    for name, bwd, fb in (("sin", ta.ta_sin_bwd, ta.ta_sin_fwdbwd),
                          ("cos", ta.ta_cos_bwd, ta.ta_cos_fwdbwd),
                          ("tan", ta.ta_tan_bwd, ta.ta_tan_fwdbwd)):
        gx = torch.empty_like(xd)
        bwd(xd, gd, gx)
        gxh = host(gx)
        _check_grad(name, x, g, gxh, rg[name], grad_near)
        y2, gx2 = torch.empty_like(xd), torch.empty_like(xd)
        fb(xd, gd, y2, gx2)
        assert np.array_equal(host(gx2).view(np.uint32), gxh.view(np.uint32))
        near, alt = neighbour_values(x.astype(np.float64))
        check_f32(f"fwdbwd-y:{name}", x, host(y2), rf[name], alt, near)
    # sincos backward: gx = gs dsin + gc dcos
    gs, gc = g, wl.normal_pair((n,), 1.0, seed=32)[1]
    gsd, gcd = to_dev(gs, dev), to_dev(gc, dev)
    near, ag = grad_near
    for label, ws, wc in (("both", 1.0, 1.0), ("gs", 1.0, 0.0),
                          ("gc", 0.0, 1.0)):
        a = gsd if ws else None
        b = gcd if wc else None
        ref = ws * gs * rg["sin"] + wc * gc * rg["cos"]
        alt = ws * gs * ag["sin"] + wc * gc * ag["cos"]
        tol = GRAD_ULPS * U24 * (np.abs(ws * gs * rg["sin"]) +
                                 np.abs(wc * gc * rg["cos"])) + ulp32(ref)
        tol_a = GRAD_ULPS * U24 * (np.abs(ws * gs * ag["sin"]) +
                                   np.abs(wc * gc * ag["cos"])) + ulp32(alt)
        gx = torch.empty_like(xd)
        ta.ta_sincos_bwd(xd, a, b, gx)
        bad = grad_bad(host(gx), ref, tol, near, alt, tol_a)
        assert not bad.any(), (label, x[bad][:3])


@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_backward_16bit(dev, kind):
    tdt = torch.float16 if kind == "f16" else torch.bfloat16
    n = 1 << 16
    x, g = _grad_case(n, 3.0, 41)
    xr, gr = wl.round_to_16(x, kind), wl.round_to_16(g, kind)
    x64, g64 = wl.decode_16(xr, kind), wl.decode_16(gr, kind)
    say(f"backward {kind}")
    xd = torch.from_numpy(xr.view(np.int16)).to(dev).view(tdt)
    gd = torch.from_numpy(gr.view(np.int16)).to(dev).view(tdt)
    rg = oracle.grad(x64)
    near, ag = neighbour_grads(x64)
    for name, bwd in (("sin", ta.ta_sin_bwd), ("cos", ta.ta_cos_bwd),
                      ("tan", ta.ta_tan_bwd)):
        gx = torch.empty_like(xd)
        bwd(xd, gd, gx)
        raw = host(gx.view(torch.int16)).view(np.uint16)
        ref = g64 * rg[name]
        alt = np.where(near, g64 * ag[name], ref)
        # the band's neighbour may differ in size by the jump: the larger
        # of the two sizes sets the tolerance
        size = np.maximum(np.abs(ref), np.abs(alt))
        tol = GRAD_ULPS_16 * U24 * size + ulp32(size)
        check_16(f"bwd-{name}", kind, raw, ref, tol, {name: alt}, near)
        say(f"backward {kind} {name}: band elements {int(near.sum())}")


def test_gradient_vs_finite_differences_and_trig(dev):
    """Central differences of the FP64 oracle (h = 1e-3) at 10^4 points away
    from the piece boundaries and the folds; and the distance to the
    exact-trig gradient."""
    rng = np.random.default_rng(51)
    x = (rng.standard_normal(40000) * 3.0).astype(np.float32)
    h = 1e-3
    x64 = x.astype(np.float64)
    rho, v, _, _, _ = oracle.fold(x64)
    nodes = np.arange(1, 6) * (math.pi / 12)
    dist = np.abs(rho[:, None] - nodes[None, :]).min(axis=1)
    # the fold makes the approximation C^1 but not C^2 at rho = 0 and
    # rho = pi/2 (D's slope in x flips sign with |r|): keep 2h away too
    keep = (dist > 2 * h) & (v > 2 * h) & (rho > 2 * h)
    x = x[keep][:10000]
    x64 = x.astype(np.float64)
    say(f"finite differences n={x.size}")
    xd = to_dev(x, dev)
    ones = torch.ones_like(xd)
    fp = oracle.forward(x64 + h)
    fm = oracle.forward(x64 - h)
    t0 = oracle.forward(x64)["tan"]
    for name, bwd in (("sin", ta.ta_sin_bwd), ("cos", ta.ta_cos_bwd),
                      ("tan", ta.ta_tan_bwd)):
        gx = torch.empty_like(xd)
        bwd(xd, ones, gx)
        gpu = host(gx).astype(np.float64)
        fd = (fp[name] - fm[name]) / (2 * h)
        # central-difference truncation h^2/6 |f'''| with the trig third
        # derivative as the size (sin/cos: <= 1.1; tan: 2 sec^2 (3 tan^2 + 1))
        if name == "tan":
            sec2 = 1.0 + t0 * t0
            trunc = h * h / 6 * 2 * sec2 * (3 * t0 * t0 + 1) * 1.5
            keep_t = np.abs(t0) < 20.0
        else:
            trunc = np.full_like(fd, h * h / 6 * 1.1 * 1.5)
            keep_t = np.ones_like(fd, bool)
        tol = 1e-5 + 8 * ulp32(fd) + trunc + 2 * GRAD_ULPS * U24 * np.abs(fd)
        bad = (np.abs(gpu - fd) > tol) & keep_t
        assert not bad.any(), (name, x[bad][:3], gpu[bad][:3], fd[bad][:3])
    gx = torch.empty_like(xd)
    ta.ta_sin_bwd(xd, ones, gx)
    d = np.abs(host(gx).astype(np.float64) - np.cos(x64))
    say(f"|d sin_a/dx - cos x|: max {d.max():.4g} mean {d.mean():.4g}")
    assert d.max() < 2.3e-2


def test_autograd_functions(dev):
    x, g = _grad_case(4099, 3.0, 61)
    xd = to_dev(x, dev).requires_grad_(True)
    gd = to_dev(g, dev)
    say("autograd functions")
    for fn, bwd, fwd in ((ta.SinFn, ta.ta_sin_bwd, ta.ta_sin),
                         (ta.CosFn, ta.ta_cos_bwd, ta.ta_cos),
                         (ta.TanFn, ta.ta_tan_bwd, ta.ta_tan)):
        xd.grad = None
        y = fn.apply(xd)
        y.backward(gd)
        yref, gref = torch.empty_like(gd), torch.empty_like(gd)
        fwd(xd.detach(), yref)
        bwd(xd.detach(), gd, gref)
        assert torch.equal(y.detach(), yref)
        assert torch.equal(xd.grad, gref)
    xd.grad = None
    s, c = ta.SinCosFn.apply(xd)
    (s * gd + c * 2.0).sum().backward()
    gref = torch.empty_like(gd)
    ta.ta_sincos_bwd(xd.detach(), gd, torch.full_like(gd, 2.0), gref)
    assert torch.equal(xd.grad, gref)


def test_fused_fwdbwd_full_size(dev):
    """[128, 8192, 512] FP32 activation, x ~ N(0, 10^2): the fused kernel in
    the benchmark launch, every element against the oracle in 2^24-element
    chunks."""
    shape = (128, 8192, 512)
    n = int(np.prod(shape))
    say(f"fused fwd+bwd full size n={n}: generating")
    gen = torch.Generator(device=dev).manual_seed(wl.SEED)
    x = torch.randn(n, device=dev, generator=gen) * 10.0
    g = torch.randn(n, device=dev, generator=gen)
    y, gx = torch.empty_like(x), torch.empty_like(x)
    ta.ta_sin_fwdbwd(x, g, y, gx)
    torch.cuda.synchronize()
    chunk = 1 << 24
    for lo in range(0, n, chunk):
        sl = slice(lo, lo + chunk)
        xs, gs = host(x[sl]), host(g[sl])
        ys, gxs = host(y[sl]), host(gx[sl])
        x64 = xs.astype(np.float64)
        ref_f = oracle.forward(x64, want=("sin",))["sin"]
        near, alt = neighbour_values(x64)
        check_f32("fwdbwd-y:sin", xs, ys, ref_f, alt, near)
        rg = oracle.grad(x64)["sin"]
        g64 = gs.astype(np.float64)
        ref = g64 * rg
        gnear, ag = neighbour_grads(x64)
        alt = g64 * ag["sin"]
        bad = grad_bad(gxs, ref, GRAD_ULPS * U24 * np.abs(ref) + ulp32(ref),
                       gnear, alt, GRAD_ULPS * U24 * np.abs(alt) + ulp32(alt))
        assert not bad.any(), (lo, xs[bad][:3], gxs[bad][:3], ref[bad][:3])
        if lo % (1 << 27) == 0:
            say(f"fused fwd+bwd: elements {lo}.. ok")
    del x, g, y, gx


@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_activation_every_element(dev, kind):
    """[64, 4096, 256] activation, x ~ N(0, 3^2), g ~ N(0, 1) (BF16: both
    rounded to nearest even): forward, backward and the fused kernel on the
    whole tensor, every element checked against the oracle in 2^24-element
    chunks; the fused kernel's outputs equal the separate calls' bits."""
    tdt = torch.float32 if kind == "f32" else torch.bfloat16
    n = 64 * 4096 * 256
    say(f"activation {kind} n={n}: generating")
    gen = torch.Generator(device=dev).manual_seed(wl.SEED)
    x = (torch.randn(n, device=dev, generator=gen) * 3.0).to(tdt)
    g = torch.randn(n, device=dev, generator=gen).to(tdt)
    y1, gx1 = torch.empty_like(x), torch.empty_like(x)
    y2, gx2 = torch.empty_like(x), torch.empty_like(x)
    ta.ta_sin(x, y1)
    ta.ta_sin_bwd(x, g, gx1)
    ta.ta_sin_fwdbwd(x, g, y2, gx2)
    torch.cuda.synchronize()
    iv = torch.int32 if kind == "f32" else torch.int16
    assert torch.equal(y1.view(iv), y2.view(iv))
    assert torch.equal(gx1.view(iv), gx2.view(iv))
    chunk = 1 << 24
    for lo in range(0, n, chunk):
        sl = slice(lo, lo + chunk)
        xs = x[sl].double().cpu().numpy()
        gs = g[sl].double().cpu().numpy()
        ref_f = oracle.forward(xs, want=("sin",))["sin"]
        ref_g = gs * oracle.grad(xs)["sin"]
        near, alt = neighbour_values(xs)
        gnear, ag = neighbour_grads(xs)
        alt_g = gs * ag["sin"]
        tol = GRAD_ULPS * U24 * np.abs(ref_g) + ulp32(ref_g)
        tol_a = GRAD_ULPS * U24 * np.abs(alt_g) + ulp32(alt_g)
        if kind == "f32":
            check_f32("act-y:sin", xs, host(y2[sl]), ref_f, alt, near)
            gxs = host(gx2[sl]).astype(np.float64)
        else:
            raw = host(y2[sl].view(torch.int16)).view(np.uint16)
            check_16("act-y:sin", "bf16", raw, ref_f, 4 * ulp32(ref_f), alt,
                     near)
            # the 16-bit gradient: RNE16 of a value within tol of the oracle
            # (in the band, of the neighbouring piece's)
            alt16 = np.where(gnear, alt_g, ref_g)
            size = np.maximum(np.abs(ref_g), np.abs(alt16))
            tol = GRAD_ULPS_16 * U24 * size + ulp32(size)
            graw = host(gx2[sl].view(torch.int16)).view(np.uint16)
            check_16("act-gx:sin", "bf16", graw, ref_g, tol, {"sin": alt16},
                     gnear)
            say(f"activation {kind}: elements {lo}..{lo + chunk} ok")
            continue
        bad = grad_bad(gxs, ref_g, tol, gnear, alt_g, tol_a)
        assert not bad.any(), (kind, lo, xs[bad][:3], gxs[bad][:3],
                               ref_g[bad][:3])
        say(f"activation {kind}: elements {lo}..{lo + chunk} ok")
    del x, g, y1, y2, gx1, gx2


# ---------------------------------------------------------------------------
# multi-frequency encoding
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [(1 << 18) + 4, 1000003])   # vector / scalar
def test_encode_f32(dev, n):
    nfreq = 8
    x = wl.small_uniform(n, seed=121)
    x[:3] = [0.0, -0.0, 1.5707964]
    xd = to_dev(x, dev)
    y = torch.empty(2 * nfreq * n, device=dev)
    say(f"encode n={n} nfreq={nfreq}")
    ta.ta_sincos_encode(xd, y, nfreq)
    yh = host(y).reshape(2 * nfreq, n)
    worst = 0.0
    for j in range(nfreq):
        xj = x.astype(np.float64) * 2.0 ** j
        ref = oracle.forward(xj)
        worst = max(worst,
                    check_f32(f"enc{j}:sin", xj, yh[2 * j], ref["sin"]),
                    check_f32(f"enc{j}:cos", xj, yh[2 * j + 1], ref["cos"]))
    say(f"encode max ulp {worst}")
    # frequency 0 is bit-identical to ta_sincos
    ys, yc = torch.empty_like(xd), torch.empty_like(xd)
    ta.ta_sincos(xd, ys, yc, None)
    assert np.array_equal(host(ys).view(np.uint32), yh[0].view(np.uint32))
    assert np.array_equal(host(yc).view(np.uint32), yh[1].view(np.uint32))


@pytest.mark.parametrize("kind,off", [("f32", 1), ("f32", 3), ("bf16", 1),
                                      ("f16", 5)])
def test_map_shared_misalignment(dev, kind, off):
    """Inputs and outputs that all sit `off` elements past a 16-byte boundary
    take a scalar head, then the 16-byte body, then a scalar tail; every
    element equals that of the same call on 16-byte aligned buffers (whose
    parity with the oracle the other tests check)."""
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16,
           "f16": torch.float16}[kind]
    n = (1 << 16) + 37
    gen = torch.Generator().manual_seed(123)
    x = (torch.rand(n, generator=gen, dtype=torch.float64) * 20 - 10).to(tdt)
    g = torch.randn(n, generator=gen).to(tdt)
    say(f"shared misalignment {kind} off={off} n={n}")

    def at_offset(t):
        buf = torch.empty(n + off, dtype=tdt, device=dev)
        assert buf.data_ptr() % 16 == 0
        buf[off:].copy_(t)
        return buf[off:]

    results = []
    for xs, gs in ((x.to(dev), g.to(dev)), (at_offset(x), at_offset(g))):
        o = [at_offset(torch.zeros(n, dtype=tdt)) if xs.data_ptr() % 16
             else torch.zeros(n, dtype=tdt, device=dev) for _ in range(7)]
        ta.ta_sin(xs, o[0])
        ta.ta_sincos(xs, o[1], o[2], o[3])
        ta.ta_sin_bwd(xs, gs, o[4])
        ta.ta_sin_fwdbwd(xs, gs, o[5], o[6])
        results.append([host(t.view(torch.int16) if t.element_size() == 2
                             else t) for t in o])
    for k, (u, v) in enumerate(zip(*results)):
        assert u.tobytes() == v.tobytes(), (kind, off, k)


def test_encode_f32_shared_misalignment(dev):
    """x and y both 4 bytes past a 16-byte boundary: the 16-byte body starts
    at element 3 of every plane, with a scalar head of 3 and tail of 1."""
    n, nfreq = (1 << 18) + 8, 8
    x = wl.small_uniform(n, seed=122)
    xbuf = torch.empty(n + 1, device=dev)
    ybuf = torch.empty(2 * nfreq * n + 1, device=dev)
    assert xbuf.data_ptr() % 16 == 0 and ybuf.data_ptr() % 16 == 0
    xd, y = xbuf[1:], ybuf[1:]
    xd.copy_(torch.from_numpy(x))
    say(f"encode shared misalignment n={n} nfreq={nfreq}")
    ta.ta_sincos_encode(xd, y, nfreq)
    yh = host(y).reshape(2 * nfreq, n)
    for j in range(nfreq):
        xj = x.astype(np.float64) * 2.0 ** j
        ref = oracle.forward(xj)
        check_f32(f"encm{j}:sin", xj, yh[2 * j], ref["sin"])
        check_f32(f"encm{j}:cos", xj, yh[2 * j + 1], ref["cos"])


@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_encode_16bit_exhaustive(dev, kind):
    tdt = torch.float16 if kind == "f16" else torch.bfloat16
    raw = wl.all_16bit_patterns()
    x64 = wl.decode_16(raw, kind)
    nfreq = 4
    say(f"encode 16-bit exhaustive {kind}")
    xd = torch.from_numpy(raw.view(np.int16)).to(dev).view(tdt)
    y = ta.encode(xd, nfreq)
    got = host(y.view(torch.int16)).view(np.uint16)
    for j in range(nfreq):
        with np.errstate(invalid="ignore"):   # the NaN patterns
            xj = x64 * 2.0 ** j
        fin = np.abs(xj) < 3.0e38   # 2^j x stays finite in FP32
        ref = oracle.forward(xj[fin])
        for k, name in ((2 * j, "sin"), (2 * j + 1, "cos")):
            check_16(f"enc{j}-{name}", kind, got[k][fin], ref[name],
                     4 * ulp32(ref[name]))


# ---------------------------------------------------------------------------
# comparators and the copy ceiling kernel (not the method)
# ---------------------------------------------------------------------------

def test_comparators_and_copy(dev):
    x = wl.small_uniform(1 << 16, seed=81)
    xd = to_dev(x, dev)
    say("comparators")
    x64 = x.astype(np.float64)
    for kind, tol in ((0, 4e-7), (1, 2e-3), (2, 4e-7)):
        ys, yc, yt = (torch.empty_like(xd) for _ in range(3))
        ta.ta_builtin_sincos(xd, ys, yc, yt, kind=kind)
        assert np.abs(host(ys) - np.sin(x64)).max() < tol
        assert np.abs(host(yc) - np.cos(x64)).max() < tol
    outs = [torch.empty_like(xd) for _ in range(3)]
    ta.ta_copy([xd], outs)
    for o in outs:
        assert torch.equal(o, xd)
    # the copy shapes of the ceilings (1 -> 1, 2 -> 2) with ragged sizes,
    # an unaligned start and canaries after the end
    for n in ((1 << 20) + 5, 1000003):
        a = torch.randn(n + 1, device=dev)[1:]
        b = torch.randn(n, device=dev, dtype=torch.float64).float()
        ya = torch.full((n + 8,), 7.0, device=dev)
        yb = torch.full((n + 8,), 7.0, device=dev)
        ta.ta_copy([a], [ya[:n]])
        assert torch.equal(ya[:n], a) and bool((ya[n:] == 7.0).all())
        ya.fill_(7.0)
        ta.ta_copy([a, b], [ya[:n], yb[:n]])
        assert torch.equal(ya[:n], a) and torch.equal(yb[:n], b)
        assert bool((ya[n:] == 7.0).all()) and bool((yb[n:] == 7.0).all())


def test_builtin_comparators_all_shapes(dev):
    """The built-in comparators of every timed shape: single-output FP32,
    FP16/BF16 single and three outputs, and the fused forward+backward, each
    against FP64 libm within the function's own accuracy."""
    x = wl.small_uniform((1 << 16) + 3, seed=82)
    x64 = x.astype(np.float64)
    xd = to_dev(x, dev)
    say("builtin comparators")
    for kind, tol in ((0, 4e-7), (1, 2e-3), (2, 4e-7)):
        ys = torch.empty_like(xd)
        ta.ta_builtin_sincos(xd, ys, kind=kind)
        assert np.abs(host(ys) - np.sin(x64)).max() < tol, kind
    for tdt, ulp16 in ((torch.bfloat16, 2.0 ** -8), (torch.float16, 2.0 ** -11)):
        xh = xd.to(tdt)
        xh64 = xh.double().cpu().numpy()
        for kind, tol in ((0, 4e-7), (1, 2e-3)):
            one = torch.empty_like(xh)
            ta.ta_builtin_sincos(xh, one, kind=kind)
            a, b, c = (torch.empty_like(xh) for _ in range(3))
            ta.ta_builtin_sincos(xh, a, b, c, kind=kind)
            torch.cuda.synchronize()
            assert torch.equal(one.view(torch.int16), a.view(torch.int16))
            for t, ref in ((a, np.sin(xh64)), (b, np.cos(xh64))):
                err = np.abs(t.double().cpu().numpy() - ref)
                assert (err <= tol + ulp16 * np.abs(ref)).all(), (tdt, kind)
            tr = np.tan(xh64)
            ok = np.abs(np.cos(xh64)) > 1e-2
            rel = np.abs(c.double().cpu().numpy() - tr)[ok] / np.abs(tr[ok])
            assert rel.max() < (3e-2 if kind == 1 else 2 * ulp16), (tdt, kind)
    g = wl.normal_pair((x.size,), 1.0, seed=83)[1]
    gd = to_dev(g, dev)
    for tdt in (torch.float32, torch.bfloat16):
        xt, gt = xd.to(tdt), gd.to(tdt)
        xt64, gt64 = xt.double().cpu().numpy(), gt.double().cpu().numpy()
        for kind, tol in ((0, 4e-7), (1, 2e-3)):
            y, gx = torch.empty_like(xt), torch.empty_like(xt)
            ta.ta_builtin_sin_fwdbwd(xt, gt, y, gx, kind=kind)
            torch.cuda.synchronize()
            rel16 = 2.0 ** -8 if tdt == torch.bfloat16 else 0.0
            ey = np.abs(y.double().cpu().numpy() - np.sin(xt64))
            eg = np.abs(gx.double().cpu().numpy() - gt64 * np.cos(xt64))
            assert (ey <= tol + rel16 * np.abs(np.sin(xt64))).all()
            assert (eg <= (tol + rel16) * np.abs(gt64) + 1e-30).all()


def test_stream_probes(dev):
    """The bandwidth probes stream what they claim: the write probe stores
    the vector index in the first word of each 16-byte vector and zeros in
    the others, the copy probe copies, the read probe runs; every valid flag
    combination (device scope only with nontemporal stores)."""
    n = (1 << 20) + 4096
    x = torch.randn(n, device=dev)
    sink = torch.zeros(1024, dtype=torch.int32, device=dev)
    idx = torch.arange(n // 4, device=dev, dtype=torch.int64).to(torch.int32)
    for flags in range(16):
        if (flags & ta.TA_PROBE_DEVICE_SCOPE) and not (flags & ta.TA_PROBE_NT_STORE):
            continue
        outs = [torch.full((n,), 7.0, device=dev) for _ in range(3)]
        ta.ta_stream_probe(0, x, [sink.view(torch.float32)], flags)
        for k in (1, 2, 3):
            ta.ta_stream_probe(1, x, outs[:k], flags)
            torch.cuda.synchronize()
            for o in outs[:k]:
                w = o.view(torch.int32).view(-1, 4)
                assert torch.equal(w[:, 0], idx)
                assert bool((w[:, 1:] == 0).all())
            ta.ta_stream_probe(2, x, outs[:k], flags)
            torch.cuda.synchronize()
            for o in outs[:k]:
                assert torch.equal(o, x)
    say("stream probes ok")


def test_force_fp32_reduction_flag(dev):
    """TA_FLAG_FORCE_FP32_REDUCTION on FP32 storage: the FP32 evaluation with
    the reduction residual carried, within 4 ulp of the formula on a strided
    sweep of every binade below 2^20, large arguments (the FP64 fold above
    2^20) and the FP32 values closest to multiples of pi/2.  On 16-bit
    storage the flag changes no bit; flags 0 give the bits of the plain
    calls."""
    flag = ta.TA_FLAG_FORCE_FP32_REDUCTION
    pos = np.arange(0, 0x49800000, 251, dtype=np.uint32).view(np.float32)
    rng = np.random.default_rng(5)
    parts = [pos, -pos, wl.log_magnitude(1 << 20, seed=6),
             _closest_to_multiples_of_half_pi(),
             rng.uniform(-1e30, 1e30, 4096).astype(np.float32)]
    x = np.concatenate(parts).astype(np.float32)
    say(f"force fp32 reduction n={x.size}")
    xd = to_dev(x, dev)
    out = {}
    for name, fn in (("sin", ta.ta_sin_ex), ("cos", ta.ta_cos_ex),
                     ("tan", ta.ta_tan_ex)):
        y = torch.empty_like(xd)
        fn(xd, y, flag)
        out[name] = host(y)
    ys, yc, yt = (torch.empty_like(xd) for _ in range(3))
    ta.ta_sincos_ex(xd, ys, yc, yt, flag)
    out["f3_sin"], out["f3_cos"], out["f3_tan"] = host(ys), host(yc), host(yt)
    ref = oracle.forward(x.astype(np.float64))
    near, alt = neighbour_values(x.astype(np.float64))
    worst = {}
    for key, got in out.items():
        fn = key.split("_")[-1]
        worst[key] = check_f32(f"fp32red:{key}", x, got, ref[fn], alt, near)
    for k in ("sin", "cos", "tan"):
        assert np.array_equal(out[k].view(np.uint32),
                              out["f3_" + k].view(np.uint32))
    say(f"force fp32 reduction: max ulp {worst}")
    # flags 0 on the _ex calls give the plain calls' bits
    xs = xd[: 1 << 16]
    for plain, ex in ((ta.ta_sin, ta.ta_sin_ex), (ta.ta_cos, ta.ta_cos_ex),
                      (ta.ta_tan, ta.ta_tan_ex)):
        a, b = torch.empty_like(xs), torch.empty_like(xs)
        plain(xs, a)
        ex(xs, b, 0)
        torch.cuda.synchronize()
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    # 16-bit storage always evaluates in FP32 (without the carried residual)
    for tdt in (torch.bfloat16, torch.float16):
        h = torch.from_numpy(wl.throughput_mix(1 << 16, seed=78)).to(dev)
        h = h.clamp(-6e4, 6e4).to(tdt)
        a = [torch.empty_like(h) for _ in range(3)]
        b = [torch.empty_like(h) for _ in range(3)]
        ta.ta_sincos_ex(h, *a, 0)
        ta.ta_sincos_ex(h, *b, flag)
        torch.cuda.synchronize()
        for u, v in zip(a, b):
            assert torch.equal(u.view(torch.int16), v.view(torch.int16))


def test_force_fp64_reduction_flag_changes_nothing(dev):
    """The flag is accepted and every reduction is FP64 already: identical
    bits with and without it, FP32 and FP64 storage, forward and paper."""
    for dt in (torch.float32, torch.float64):
        x = torch.from_numpy(wl.throughput_mix(1 << 16, seed=77)).to(dev).to(dt)
        a = [torch.empty_like(x) for _ in range(3)]
        b = [torch.empty_like(x) for _ in range(3)]
        ta.ta_sincos_ex(x, *a, 0)
        ta.ta_sincos_ex(x, *b, ta.TA_FLAG_FORCE_FP64_REDUCTION)
        p = [torch.empty_like(x) for _ in range(3)]
        q = [torch.empty_like(x) for _ in range(3)]
        ta.ta_paper_sincos(x, *p, ta.TA_FLAG_LITERAL_DIVISOR)
        ta.ta_paper_sincos(x, *q, ta.TA_FLAG_LITERAL_DIVISOR |
                           ta.TA_FLAG_FORCE_FP64_REDUCTION)
        torch.cuda.synchronize()
        for u, v in zip(a + p, b + q):
            assert torch.equal(u.view(torch.uint8), v.view(torch.uint8))
