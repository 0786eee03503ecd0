"""GPU parity of the FP64 path (TA_F64) against the extended-precision
oracle: forward (fused and single-output), backward, Taylor, the paper's
literal arithmetic, the encoding, the comparators and autograd.

Tolerance: 6 FP64 ulp of the exact value for the method (sin/cos at most
5.5 u relative by the error analysis of the FP64 stages, tan 4.5 u, with
u = 2^-53); inputs whose fold angle lies within 2^-40 rad of a jump of the
approximation (15, 30, 60, 75 degrees) may take either neighbouring piece.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2502_10831_amd as ta
from paper_2502_10831_amd import workloads as wl

pytestmark = pytest.mark.gpu

ULP_FWD = 6.0
ULP_BWD = 16.0
PI12 = math.pi / 12
NAMES = ("sin", "cos", "tan")


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ta.load()
    return torch.device("cuda:0")


def _ulp(ref):
    r = np.abs(np.asarray(ref, np.longdouble)).astype(np.float64)
    return np.spacing(r)


def _near_jump(x):
    rho, _, _ = oracle.fold_ld(x)
    q = rho / np.longdouble(PI12)
    k = np.round(q)
    return (np.abs(q - k) * np.longdouble(PI12) < 2.0 ** -40) & \
        np.isin(k, [1, 2, 4, 5])


def _compare(name, got, ref, tol_ulp, scale=None):
    """Per-element |got - ref| in ulp of `scale` (default ref); NaN must
    match NaN, infinities must be equal."""
    g = np.asarray(got, np.float64)
    r = np.asarray(ref, np.longdouble)
    both_nan = np.isnan(g) & np.isnan(r.astype(np.float64))
    same_inf = np.isinf(g) & (g == r.astype(np.float64))
    s = r if scale is None else scale
    with np.errstate(invalid="ignore", divide="ignore"):   # inf - inf, NaN
        err = np.abs(g.astype(np.longdouble) - r)
        e_ulp = (err / _ulp(s)).astype(np.float64)
    ok = both_nan | same_inf | (e_ulp <= tol_ulp)
    e_ulp = np.where(both_nan | same_inf, 0.0, e_ulp)
    return ok, e_ulp


def check_forward(x, outs, label, flags=0):
    """outs: dict name -> GPU tensor (FP64) for any subset of NAMES."""
    ref = oracle.forward_ld(x, flags)
    near = _near_jump(x)
    worst = {}
    for name, t in outs.items():
        g = t.cpu().numpy()
        ok, e = _compare(name, g, ref[name], ULP_FWD)
        bad = ~ok
        if bad.any():
            # a rounding-distance neighbour of a jump may use either piece
            idx = np.flatnonzero(bad & near)
            for sh in (-1, 1):
                if idx.size == 0:
                    break
                alt = oracle.forward_ld(x[idx], flags, shift=sh)[name]
                ok2, _ = _compare(name, g[idx], alt, ULP_FWD)
                ok[idx[ok2]] = True
                idx = idx[~ok2]
        assert ok.all(), (label, name, x[~ok][:4], g[~ok][:4],
                          ref[name][~ok][:4])
        worst[name] = float(e[~near].max()) if (~near).any() else 0.0
    say(f"{label}: n={x.size} max ulp {worst}; near a jump {int(near.sum())}")
    return worst


def _gpu(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).to(dev)


def _sincos3(xd, flags=0):
    ys, yc, yt = (torch.empty_like(xd) for _ in range(3))
    ta.ta_sincos_ex(xd, ys, yc, yt, flags)
    torch.cuda.synchronize()
    return {"sin": ys, "cos": yc, "tan": yt}


HARD = [6381956970095103.0 * 2.0 ** 797, 5.319372648326541e+255, 1e22, 355.0,
        2.0 ** 29, float(np.nextafter(2.0 ** 29, 0)), 2.0 ** 52, 2.0 ** 53,
        1.7976931348623157e308, 2.2250738585072014e-308, 5e-324, 1e-300,
        float.fromhex("0x1.921fb54442d18p+0"), float.fromhex("0x1.921fb54442d18p-1")]


def _edge_inputs():
    xs = list(HARD)
    rng = np.random.default_rng(11)
    ks = list(range(1, 2001, 2)) + [int(v) * 2 + 1 for v in
                                    rng.integers(1, 1 << 29, 1000)]
    for k in ks:  # nearest doubles to odd multiples of pi/4 (quadrant ties)
        v = math.pi / 4 * k
        xs += [v, float(np.nextafter(v, 0)), float(np.nextafter(v, np.inf))]
    xs += [math.pi / 2 * k for k in range(1, 2000)]  # tiny |r|
    xs = np.array(xs)
    return np.concatenate([xs, -xs])


def test_f64_mixed_parity(dev):
    x = np.concatenate([wl.uniform(1 << 18, -2 * math.pi, 2 * math.pi, 31,
                                   np.float64),
                        wl.protocol_f64((1 << 18) + 5, seed=32),
                        wl.log_magnitude_f64(1 << 18, seed=33)])
    xd = _gpu(x, dev)
    outs = _sincos3(xd)
    check_forward(x, outs, "f64 mixed")
    # the single-output kernels run the same arithmetic: identical bits
    for name, fn in (("sin", ta.ta_sin), ("cos", ta.ta_cos), ("tan", ta.ta_tan)):
        y = torch.empty_like(xd)
        fn(xd, y)
        torch.cuda.synchronize()
        assert torch.equal(y.view(torch.int64), outs[name].view(torch.int64)), name
    ys, yc = torch.empty_like(xd), torch.empty_like(xd)
    ta.ta_sincos(xd, ys, yc, None)
    torch.cuda.synchronize()
    assert torch.equal(ys.view(torch.int64), outs["sin"].view(torch.int64))
    assert torch.equal(yc.view(torch.int64), outs["cos"].view(torch.int64))


def test_f64_every_exponent(dev):
    x = wl.exponent_sweep_f64(32, seed=34)
    say(f"f64 exponent sweep n={x.size}")
    check_forward(x, _sincos3(_gpu(x, dev)), "f64 exponents")


def test_f64_reduction_edges_and_specials(dev):
    x = _edge_inputs()
    check_forward(x, _sincos3(_gpu(x, dev)), "f64 reduction edges")
    sp = np.array([0.0, -0.0, math.inf, -math.inf, math.nan])
    o = {k: v.cpu().numpy() for k, v in _sincos3(_gpu(sp, dev)).items()}
    assert o["sin"][0] == 0 and not np.signbit(o["sin"][0])
    assert o["sin"][1] == 0 and np.signbit(o["sin"][1])
    assert o["tan"][1] == 0 and np.signbit(o["tan"][1])
    assert o["cos"][0] == 1 and o["cos"][1] == 1
    for k in NAMES:
        assert np.isnan(o[k][2:]).all()


def test_f64_tan_guard(dev):
    x = wl.protocol_f64(1 << 16, seed=35)
    # plus points within 1e-3 of odd multiples of pi/2
    m = np.random.default_rng(36).integers(-1000, 1000, 4096)
    near = (2 * m + 1) * (math.pi / 2) + \
        np.random.default_rng(37).uniform(-2e-3, 2e-3, 4096)
    x = np.concatenate([x, near])
    outs = _sincos3(_gpu(x, dev), ta.TA_FLAG_TAN_GUARD)
    check_forward(x, {"tan": outs["tan"]}, "f64 tan guard",
                  flags=oracle.TAN_GUARD)
    assert np.isposinf(outs["tan"].cpu().numpy()).sum() > 1000


def test_f64_alignment_and_in_place(dev):
    x = wl.protocol_f64((1 << 16) + 3, seed=38)
    xd = _gpu(x, dev)
    ref = oracle.forward_ld(x, 0, want=("sin",))["sin"]
    # shared offset of one element (8 bytes): scalar head, then vectors
    buf = torch.empty(x.size + 1, dtype=torch.float64, device=dev)
    buf[1:].copy_(xd)
    out = torch.empty_like(buf)
    ta.ta_sin(buf[1:], out[1:])
    # different offsets: the scalar kernel
    out2 = torch.empty(x.size + 1, dtype=torch.float64, device=dev)
    ta.ta_sin(xd, out2[1:])
    # in place
    xi = xd.clone()
    ta.ta_sin(xi, xi)
    torch.cuda.synchronize()
    for t in (out[1:], out2[1:], xi):
        ok, _ = _compare("sin", t.cpu().numpy(), ref, ULP_FWD)
        near = _near_jump(x)
        assert (ok | near).all()
    assert torch.equal(out[1:], xi) and torch.equal(out2[1:], xi)


def test_f64_full_size(dev):
    """2^27 FP64 inputs U[-1e6, 1e6] (the benchmark's FP64 workload): every
    element of the fused sin+cos+tan output against the long-double oracle,
    in 2^24-element chunks."""
    n = 1 << 27
    say(f"f64 full size n={n}: generating inputs")
    x = wl.protocol_f64(n, seed=39)
    xd = _gpu(x, dev)
    outs = _sincos3(xd)
    torch.cuda.synchronize()
    chunk = 1 << 24
    for lo in range(0, n, chunk):
        sl = slice(lo, lo + chunk)
        check_forward(x[sl], {k: v[sl] for k, v in outs.items()},
                      f"f64 2^27 elements {lo}..")


def _grad_ref(x, g, which, shift=0):
    d = oracle.grad_ld(x, shift)[which]
    return d * np.asarray(g, np.longdouble)


def _check_grad(x, g, got, which, label):
    ref = _grad_ref(x, g, which)
    ok, e = _compare(which, got, ref, ULP_BWD)
    near = _near_jump(x)
    idx = np.flatnonzero(~ok & near)
    for sh in (-1, 1):
        if idx.size == 0:
            break
        alt = _grad_ref(x[idx], g[idx], which, sh)
        ok2, _ = _compare(which, got[idx], alt, ULP_BWD)
        ok[idx[ok2]] = True
        idx = idx[~ok2]
    assert ok.all(), (label, x[~ok][:4], got[~ok][:4], ref[~ok][:4])
    say(f"{label}: max ulp {float(e[~near].max()):.3f}")


def test_f64_backward_and_fused(dev):
    x = np.concatenate([wl.protocol_f64(1 << 17, seed=41),
                        wl.uniform(1 << 17, -10, 10, 42, np.float64)])
    g = np.random.default_rng(43).standard_normal(x.size)
    xd, gd = _gpu(x, dev), _gpu(g, dev)
    fwd = oracle.forward_ld(x)
    for which, bwd, fb in (("sin", ta.ta_sin_bwd, ta.ta_sin_fwdbwd),
                           ("cos", ta.ta_cos_bwd, ta.ta_cos_fwdbwd),
                           ("tan", ta.ta_tan_bwd, ta.ta_tan_fwdbwd)):
        gx = torch.empty_like(xd)
        bwd(xd, gd, gx)
        y2, gx2 = torch.empty_like(xd), torch.empty_like(xd)
        fb(xd, gd, y2, gx2)
        torch.cuda.synchronize()
        _check_grad(x, g, gx.cpu().numpy(), which, f"f64 {which} backward")
        assert torch.equal(gx.view(torch.int64), gx2.view(torch.int64))
        ok, _ = _compare(which, y2.cpu().numpy(), fwd[which], ULP_FWD)
        assert (ok | _near_jump(x)).all()
    # sincos backward: gs d sin + gc d cos (cancellation: scale by the sum
    # of the magnitudes of the two terms)
    gc = np.random.default_rng(44).standard_normal(x.size)
    gx = torch.empty_like(xd)
    ta.ta_sincos_bwd(xd, gd, _gpu(gc, dev), gx)
    torch.cuda.synchronize()
    d = oracle.grad_ld(x)
    a = d["sin"] * np.asarray(g, np.longdouble)
    b = d["cos"] * np.asarray(gc, np.longdouble)
    got = gx.cpu().numpy()
    err = np.abs(got.astype(np.longdouble) - (a + b))
    tol = ULP_BWD * _ulp(np.abs(a) + np.abs(b))
    assert ((err <= tol) | _near_jump(x)).all()


def test_f64_taylor(dev):
    x = np.concatenate([wl.protocol_f64(1 << 16, seed=45),
                        wl.uniform(1 << 16, -3, 3, 46, np.float64)])
    xd = _gpu(x, dev)
    eps = 2.0 ** -53
    for terms in (5, 7, 9):
        ref = oracle.taylor(x, terms)
        for name, fn in (("sin", ta.ta_taylor_sin), ("cos", ta.ta_taylor_cos),
                         ("tan", ta.ta_taylor_tan)):
            y = torch.empty_like(xd)
            fn(xd, y, terms)
            torch.cuda.synchronize()
            g = y.cpu().numpy()
            tol = 4 * terms * eps * ref["abs_" + name] + np.spacing(np.abs(ref[name]))
            err = np.abs(g - ref[name])
            assert (err <= tol).all(), (terms, name, x[err > tol][:3])
    say("f64 Taylor 5/7/9 within 4 N u sum|terms|")


def test_f64_paper_variant(dev):
    x = np.concatenate([wl.protocol_f64(1 << 17, seed=47),
                        wl.uniform(1 << 16, -2 * math.pi, 2 * math.pi, 48,
                                   np.float64)])
    xd = _gpu(x, dev)
    for divisor, flags in ((PI12, 0), (0.261, ta.TA_FLAG_LITERAL_DIVISOR)):
        ys, yc, yt = (torch.empty_like(xd) for _ in range(3))
        ta.ta_paper_sincos(xd, ys, yc, yt, flags)
        torch.cuda.synchronize()
        ref = oracle.paper(x, divisor=divisor)
        rho, v, _, _, _ = oracle.fold(x)
        q = rho / divisor
        off_node = np.abs(q - np.round(q)) * divisor >= 1e-12
        for name, t in (("sin", ys), ("cos", yc), ("tan", yt)):
            g = t.cpu().numpy()
            r = ref[name]
            tol = 1e-14 * np.abs(r) + np.spacing(np.abs(r))
            if name in ("cos", "tan"):
                tol = tol + np.abs(r) * 2.0 ** -51 / np.maximum(v, 1e-300)
            bad = (np.abs(g - r) > tol) & off_node
            assert not bad.any(), (divisor, name, x[bad][:3], g[bad][:3], r[bad][:3])
        # Tables 1-3: the literal arithmetic's maximum error on sin
        if flags == 0:
            e = np.abs(ys.cpu().numpy() - np.sin(x))
            say(f"f64 paper variant max |sin error| {e.max():.6f}")
            assert abs(e.max() - 1.532e-3) < 2e-6


def test_f64_encode(dev):
    x = wl.uniform((1 << 15) + 2, -50, 50, 49, np.float64)
    xd = _gpu(x, dev)
    y = ta.encode(xd, 8).cpu().numpy()
    for j in range(8):
        xj = x * 2.0 ** j
        ref = oracle.forward_ld(xj, want=("sin", "cos"))
        near = _near_jump(xj)
        for p, name in ((2 * j, "sin"), (2 * j + 1, "cos")):
            ok, _ = _compare(name, y[p], ref[name], ULP_FWD)
            assert (ok | near).all(), (j, name)


def test_f64_comparators(dev):
    x = wl.protocol_f64(1 << 16, seed=50)
    xd = _gpu(x, dev)
    for kind in (0, 2):
        ys, yc, yt = (torch.empty_like(xd) for _ in range(3))
        ta.ta_builtin_sincos(xd, ys, yc, yt, kind)
        torch.cuda.synchronize()
        for t, f in ((ys, np.sin), (yc, np.cos), (yt, np.tan)):
            err = np.abs(t.cpu().numpy() - f(x)) / np.spacing(np.abs(f(x)))
            assert err.max() <= 4, (kind, err.max())
    with pytest.raises(ta.TaError):
        ta.ta_builtin_sincos(xd, torch.empty_like(xd), torch.empty_like(xd),
                             None, 1)


def test_f64_autograd_gradcheck(dev):
    x = wl.uniform(64, -3, 3, 51, np.float64)
    rho, v, _, _, _ = oracle.fold(x)
    q = rho / PI12
    x = x[(np.abs(q - np.round(q)) > 1e-3) & (v > 0.05)]
    xt = torch.from_numpy(x).to(dev).requires_grad_(True)
    for fn in (ta.SinFn.apply, ta.CosFn.apply, ta.TanFn.apply):
        assert torch.autograd.gradcheck(fn, (xt,), eps=1e-7, atol=1e-6,
                                        rtol=1e-5)
    assert torch.autograd.gradcheck(lambda t: ta.SinCosFn.apply(t), (xt,),
                                    eps=1e-7, atol=1e-6, rtol=1e-5)
