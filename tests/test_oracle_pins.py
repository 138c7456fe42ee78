"""Pins of the CPU oracle against facts fixed by mathematics and by library
routines -- not against the oracle itself.

Each operation of the chain (Sections VI-F and VI-J: Crop -> Resize ->
ColorConvert -> Multiply -> Subtract -> Divide -> Split; Section VI-B:
Mul/Add chains) is pinned by at least one closed form, invariant, special
case or independent library computation, chosen so that a dropped term, a
wrong sign or index, or a transposed operand fails one of them.
"""
import math

import numpy as np
import pytest
import torch

import datagen
import oracle


def resize_only(C=3, ow=8, oh=8, dtype="u8", layout="packed", ops=None, out_dtype="f32"):
    return {"read": {"kind": "crop_resize", "dtype": dtype, "channels": C, "out_w": ow, "out_h": oh},
            "ops": ops or [], "write": {"dtype": out_dtype, "layout": layout}}


def plain(C=3, dtype="u8", layout="packed", ops=None, out_dtype="f32"):
    return {"read": {"kind": "plain", "dtype": dtype, "channels": C, "out_w": 0, "out_h": 0},
            "ops": ops or [], "write": {"dtype": out_dtype, "layout": layout}}


def item(x, y, w, h, ow=None, oh=None, frame=0):
    return {"frame": frame, "x": x, "y": y, "w": w, "h": h,
            "out_w": w if ow is None else ow, "out_h": h if oh is None else oh}


# --------------------------------------------------------------- resize --

def test_resize_same_size_is_identity():
    g = datagen.rng(1)
    fr = datagen.frame(g, 41, 57, 3)
    it = item(5, 3, 29, 21, 29, 21)
    out = oracle.run_chain(resize_only(ow=29, oh=21), [fr], [it])[0]["out"]
    np.testing.assert_array_equal(out, fr[3:24, 5:34].astype(np.float32))


@pytest.mark.parametrize("src,dst", [((100, 60), (37, 91)), ((13, 7), (64, 128)), ((600, 599), (64, 128))])
def test_resize_constant_image_stays_constant(src, dst):
    fr = np.full((700, 700, 3), 77, np.uint8)
    it = item(11, 17, src[0], src[1], dst[0], dst[1])
    out = oracle.run_chain(resize_only(ow=dst[0], oh=dst[1]), [fr], [it])[0]["out"]
    assert np.all(out == 77.0)


@pytest.mark.parametrize("w,h,ow,oh", [(200, 150, 64, 128), (60, 90, 224, 224), (256, 31, 17, 250),
                                       (255, 255, 255, 200)])
def test_resize_linear_ramp_is_source_coordinate(w, h, ow, oh):
    """A ramp P[x] = x is reproduced exactly by linear interpolation, so the
    output is the (clamped) half-pixel source coordinate itself:
    clamp((o + 0.5) * in / out - 0.5, 0, in - 1).  Channel 0 ramps in x and
    channel 1 in y, so a transposed axis fails."""
    fr = datagen.index_coded_frame(h, w, 3)  # ch0 = x, ch1 = y (both < 256)
    out = oracle.run_chain(resize_only(ow=ow, oh=oh), [fr], [item(0, 0, w, h, ow, oh)])[0]["out"]
    ex = np.clip((np.arange(ow) + 0.5) * w / ow - 0.5, 0, w - 1)
    ey = np.clip((np.arange(oh) + 0.5) * h / oh - 0.5, 0, h - 1)
    np.testing.assert_allclose(out[:, :, 0], np.broadcast_to(ex[None, :], (oh, ow)), rtol=0, atol=2e-4)
    np.testing.assert_allclose(out[:, :, 1], np.broadcast_to(ey[:, None], (oh, ow)), rtol=0, atol=2e-4)


@pytest.mark.parametrize("f", [2, 4])
def test_resize_integer_downscale_is_box_mean(f):
    """Scale f (2 or 4): source coordinate f*o + (f-1)/2 falls midway between
    pixels f*o + f/2 - 1 and f*o + f/2, so each output is the exact mean of
    that 2x2 block."""
    g = datagen.rng(2)
    fr = datagen.frame(g, 64, 96, 3)
    w, h = 96, 64
    out = oracle.run_chain(resize_only(ow=w // f, oh=h // f), [fr], [item(0, 0, w, h, w // f, h // f)])[0]["out"]
    p = fr.astype(np.float64)
    a = f // 2 - 1
    blk = (p[a::f, a::f] + p[a::f, a + 1::f] + p[a + 1::f, a::f] + p[a + 1::f, a + 1::f]) / 4.0
    np.testing.assert_array_equal(out.astype(np.float64), blk)


def test_resize_2x_upscale_weights_quarter_three_quarters():
    g = datagen.rng(3)
    fr = datagen.frame(g, 10, 12, 1)
    out = oracle.run_chain(resize_only(C=1, ow=24, oh=20), [fr], [item(0, 0, 12, 10, 24, 20)])[0]["out"][:, :, 0]
    p = fr[:, :, 0].astype(np.float64)

    def taps(n_out, n_in):
        # output 2j sits at j - 1/4, output 2j+1 at j + 1/4 (clamped to [0, n_in - 1])
        i0, i1, a = [], [], []
        for o in range(n_out):
            j = o // 2
            if o % 2 == 0:
                lo, wt = (j - 1, 0.75) if j > 0 else (0, 0.0)
            else:
                lo, wt = (j, 0.25) if j < n_in - 1 else (n_in - 1, 0.0)
            i0.append(lo); i1.append(min(lo + 1, n_in - 1)); a.append(wt)
        return np.array(i0), np.array(i1), np.array(a)

    x0, x1, ax = taps(24, 12)
    y0, y1, ay = taps(20, 10)
    top = p[y0][:, x0] * (1 - ax) + p[y0][:, x1] * ax
    bot = p[y1][:, x0] * (1 - ax) + p[y1][:, x1] * ax
    exp = top * (1 - ay[:, None]) + bot * ay[:, None]
    np.testing.assert_array_equal(out.astype(np.float64), exp)


@pytest.mark.parametrize("seed", range(4))
def test_resize_matches_torch_bilinear(seed):
    """Against torch's bilinear interpolation (align_corners=False, no
    antialias) in fp64: the same half-pixel convention, differing only by
    the fp32 rounding of coordinates."""
    g = datagen.rng(100 + seed)
    fr = datagen.frame(g, 700, 900, 3)
    w, h = int(g.integers(8, 600)), int(g.integers(8, 600))
    x, y = int(g.integers(0, 900 - w)), int(g.integers(0, 700 - h))
    ow, oh = int(g.integers(4, 300)), int(g.integers(4, 300))
    out = oracle.run_chain(resize_only(ow=ow, oh=oh), [fr], [item(x, y, w, h, ow, oh)])[0]["out"]
    t = torch.from_numpy(fr[y:y + h, x:x + w].astype(np.float64)).permute(2, 0, 1)[None]
    ref = torch.nn.functional.interpolate(t, size=(oh, ow), mode="bilinear", align_corners=False,
                                          antialias=False)[0].permute(1, 2, 0).numpy()
    err = np.abs(out.astype(np.float64) - ref)
    assert err.max() < 0.1, err.max()


# -------------------------------------------- crop, swap, split, write --

@pytest.mark.parametrize("layout", ["packed", "planar"])
@pytest.mark.parametrize("kind", ["plain", "crop_resize"])
def test_crop_swap_split_index_coded(layout, kind):
    """Every output element decodes to its own source coordinate and
    channel: crop offset, BGR->RGB order and the planar/packed layout are
    checked exhaustively."""
    H, W = 300, 520
    fr = datagen.index_coded_frame(H, W, 3)
    x, y, w, h = 213, 37, 301, 263
    ops = [{"kind": "swap", "k": []}, {"kind": "cvt", "k": []}, {"kind": "mul", "k": [1.0]},
           {"kind": "sub", "k": [0.0, 0.0, 0.0]}, {"kind": "div", "k": [1.0]}]
    ch = plain(layout=layout, ops=ops) if kind == "plain" else resize_only(ow=w, oh=h, layout=layout, ops=ops)
    out = oracle.run_chain(ch, [fr], [item(x, y, w, h, w, h)])[0]["out"]
    if layout == "planar":
        out = np.transpose(out, (1, 2, 0))
    assert out.shape == (h, w, 3)
    o = out.astype(np.int64)
    # after the swap: channel 0 = original channel 2, channel 2 = original channel 0
    xs = o[:, :, 2] | ((o[:, :, 0] & 7) << 8)
    ys = o[:, :, 1] | ((o[:, :, 0] >> 3) << 8)
    jj, ii = np.mgrid[0:h, 0:w]
    np.testing.assert_array_equal(xs, x + ii)
    np.testing.assert_array_equal(ys, y + jj)


@pytest.mark.parametrize("C", [1, 3, 4])
def test_swap_semantics_per_channel_count(C):
    fr = datagen.index_coded_frame(5, 7, C)
    ops = [{"kind": "swap", "k": []}]
    out = oracle.run_chain(plain(C=C, ops=ops), [fr], [item(0, 0, 7, 5)])[0]["out"]
    perm = {1: [0], 3: [2, 1, 0], 4: [2, 1, 0, 3]}[C]
    np.testing.assert_array_equal(out, fr[:, :, perm].astype(np.float32))
    # two swaps cancel
    out2 = oracle.run_chain(plain(C=C, ops=ops * 2), [fr], [item(0, 0, 7, 5)])[0]["out"]
    np.testing.assert_array_equal(out2, fr.astype(np.float32))


def test_per_channel_constants_follow_swapped_positions():
    fr = datagen.index_coded_frame(6, 9, 3)
    ops = [{"kind": "swap", "k": []}, {"kind": "add", "k": [1000.0, 2000.0, 3000.0]}]
    out = oracle.run_chain(plain(ops=ops), [fr], [item(0, 0, 9, 6)])[0]["out"]
    f = fr.astype(np.float32)
    np.testing.assert_array_equal(out[:, :, 0], f[:, :, 2] + 1000)
    np.testing.assert_array_equal(out[:, :, 1], f[:, :, 1] + 2000)
    np.testing.assert_array_equal(out[:, :, 2], f[:, :, 0] + 3000)


# ----------------------------------------------------------- arithmetic --

def test_normalise_chain_is_per_op_ieee_fp32():
    """The normalise ops after the resize are single IEEE fp32 operations in
    chain order: numpy float32 arithmetic (one rounding per op) on the
    resized values gives the same bits, and fp64 stays within a few ulps."""
    cfg = datagen.config0(seed=5, frame_hw=(300, 400), crop=(17, 29, 250, 190), out=(96, 64))
    it = cfg["items"][0]
    res = oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"])[0]
    resized = oracle.run_chain(resize_only(ow=96, oh=64), cfg["frames"], cfg["items"])[0]["out"]
    v = resized[:, :, ::-1]  # BGR -> RGB
    k = np.float32(datagen.NORM_SCALE)
    mean = np.array(datagen.NORM_MEAN, np.float32)
    std = np.array(datagen.NORM_STD, np.float32)
    exp32 = ((v * k) - mean) / std
    np.testing.assert_array_equal(res["out"], np.transpose(exp32, (2, 0, 1)))
    exp64 = ((v.astype(np.float64) / 255.0) - np.array([0.485, 0.456, 0.406])) / np.array([0.229, 0.224, 0.225])
    err = np.abs(np.transpose(exp64, (2, 0, 1)) - res["out"])
    assert err.max() < 1e-5, err.max()
    assert it["out_w"] == 96


@pytest.mark.parametrize("n_ops", [1, 4, 16, 64])
def test_muladd_chain_matches_affine_closed_form(n_ops):
    """Alternating Mul/Add with scalar constants is an affine map
    v -> A v + B, A = product of the multipliers; the fp32 chain stays within
    the fp32 rounding bound of that closed form (evaluated in fp64), and the
    oracle's fp64 shadow equals it to fp64 rounding."""
    cfg = datagen.config1(n_ops, seed=7, frame_hw=(23, 31))
    res = oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"])[0]
    A, B = 1.0, 0.0
    for op in cfg["chain"]["ops"]:
        if op["kind"] == "mul":
            A *= op["k"][0]; B *= op["k"][0]
        elif op["kind"] == "add":
            B += op["k"][0]
    x = cfg["frames"][0].astype(np.float64)
    exact = A * x + B
    # first-order fp32 error bound: one half-ulp per op, magnified by later multipliers
    u = 2.0 ** -24
    ops = [op for op in cfg["chain"]["ops"] if op["kind"] in ("mul", "add")]
    bound = np.zeros_like(x)
    v = x.copy()
    for i, op in enumerate(ops):
        v = v * op["k"][0] if op["kind"] == "mul" else v + op["k"][0]
        gain = np.prod([o["k"][0] for o in ops[i + 1:] if o["kind"] == "mul"]) if i + 1 < len(ops) else 1.0
        bound += u * np.abs(v) * gain
    assert np.all(np.abs(res["out"] - exact) <= 1.01 * bound + 1e-30)
    np.testing.assert_allclose(res["v64"], exact, rtol=1e-12, atol=1e-12)
    assert np.all(res["smax"] >= np.abs(res["out"]))


def _loop_body(g, C):
    body = []
    for kind in ("mul", "sub", "div", "add"):
        lo, hi = (0.5, 1.5) if kind in ("mul", "div") else (-1.0, 1.0)
        body.append({"kind": kind, "k": [datagen.f32(g.uniform(lo, hi)) for _ in range(C)]})
    return body


@pytest.mark.parametrize("span,count", [(1, 5), (3, 4), (4, 3), (2, 1)])
def test_loop_equals_unrolled_body(span, count):
    """A loop op is its body written out `count` times (Section VI-B's repeat
    op): same results bit for bit, with ops before and after the loop and a
    swap in between so per-channel constants keep their positions."""
    g = datagen.rng(span * 10 + count)
    fr = datagen.frame(g, 9, 11, 3)
    body = _loop_body(g, 3)[:span]
    head = [{"kind": "cvt", "k": []}, {"kind": "mul", "k": [0.75, 1.25, 1.5]}, {"kind": "swap", "k": []}]
    tail = [{"kind": "swap", "k": []}, {"kind": "sub", "k": [0.5, -0.25, 0.125]}]
    looped = plain(ops=head + body + [{"kind": "loop", "span": span, "count": count}] + tail)
    unrolled = plain(ops=head + body * count + tail)
    it = [item(1, 2, 8, 6)]
    a = oracle.run_chain(looped, [fr], it)[0]
    b = oracle.run_chain(unrolled, [fr], it)[0]
    np.testing.assert_array_equal(a["out"].view(np.uint32), b["out"].view(np.uint32))
    np.testing.assert_array_equal(a["v64"], b["v64"])
    if count == 1:  # a loop that runs once is no op at all
        c = oracle.run_chain(plain(ops=head + body + tail), [fr], it)[0]
        np.testing.assert_array_equal(a["out"].view(np.uint32), c["out"].view(np.uint32))


@pytest.mark.parametrize("pairs", [1, 7, 1000])
def test_loop_chain_matches_affine_closed_form(pairs):
    """v -> m v + a repeated P times is v -> m^P v + a (1 - m^P) / (1 - m):
    the fp64 shadow equals it to fp64 rounding and the fp32 result stays
    within the first-order bound of one half-ulp per op, each damped by the
    multipliers that follow it."""
    cfg = datagen.loop_batch(pairs, seed=pairs, batch=2, hw=(5, 7), channels=1)
    ch = cfg["chain"]
    m, a = ch["ops"][1]["k"][0], ch["ops"][2]["k"][0]
    res = oracle.run_chain(ch, cfg["frames"], cfg["items"][1:])[0]
    x = cfg["frames"][0][5:10].astype(np.float64)
    mp = m ** pairs
    exact = mp * x + a * (1.0 - mp) / (1.0 - m)
    np.testing.assert_allclose(res["v64"], exact, rtol=1e-11, atol=1e-11)
    u = 2.0 ** -24
    v = x.copy()
    bound = np.zeros_like(x)
    for p in range(pairs):
        rest = m ** (pairs - 1 - p)  # multipliers after this pair's add
        v = v * m
        bound += u * np.abs(v) * m * rest
        v = v + a
        bound += u * np.abs(v) * rest
    assert np.all(np.abs(res["out"] - exact) <= 1.01 * bound + 1e-30)
    assert np.all(res["smax"] >= np.abs(res["out"]))


@pytest.mark.parametrize("ops", [
    [{"kind": "loop", "span": 1, "count": 2}],                                    # nothing before it
    [{"kind": "mul", "k": [2.0]}, {"kind": "loop", "span": 2, "count": 2}],       # span past the start
    [{"kind": "mul", "k": [2.0]}, {"kind": "loop", "span": 1, "count": 0}],       # count < 1
    [{"kind": "swap", "k": []}, {"kind": "mul", "k": [2.0]}, {"kind": "loop", "span": 2, "count": 2}],
    [{"kind": "cvt", "k": []}, {"kind": "loop", "span": 1, "count": 2}],
    [{"kind": "mul", "k": [2.0]}, {"kind": "loop", "span": 1, "count": 2},
     {"kind": "loop", "span": 2, "count": 2}],                                    # nested
])
def test_bad_loops_are_rejected(ops):
    fr = np.zeros((4, 4, 3), np.uint8)
    assert oracle.validate(plain(ops=ops), [fr], [item(0, 0, 4, 4)]) < 0


def test_division_is_true_division_not_reciprocal():
    fr = np.full((1, 4, 1), 1, np.uint8)
    fr[0, :, 0] = [3, 7, 11, 13]
    k = 3.0
    out = oracle.run_chain(plain(C=1, ops=[{"kind": "div", "k": [k]}]), [fr], [item(0, 0, 4, 1)])[0]["out"]
    np.testing.assert_array_equal(out.ravel(), np.array([3, 7, 11, 13], np.float32) / np.float32(3))
    assert out.ravel()[0] == 1.0  # 3/3 exactly; 3 * fl(1/3) would not be exactly 1


def test_scalar_and_per_channel_constants_agree_when_equal():
    g = datagen.rng(9)
    fr = datagen.frame(g, 8, 8, 3)
    a = oracle.run_chain(plain(ops=[{"kind": "mul", "k": [0.37]}]), [fr], [item(0, 0, 8, 8)])[0]["out"]
    b = oracle.run_chain(plain(ops=[{"kind": "mul", "k": [0.37] * 3}]), [fr], [item(0, 0, 8, 8)])[0]["out"]
    np.testing.assert_array_equal(a, b)


# ---------------------------------------------------------------- fp16 --

def test_half_to_float_all_patterns_match_numpy():
    bits = np.arange(65536, dtype=np.uint16)
    got = oracle.half_to_float(bits)
    exp = bits.view(np.float16).astype(np.float32)
    nan = np.isnan(exp)
    np.testing.assert_array_equal(np.isnan(got), nan)
    np.testing.assert_array_equal(got[~nan].view(np.uint32), exp[~nan].view(np.uint32))


def test_float_to_half_round_to_nearest_even_matches_numpy():
    g = datagen.rng(11)
    specials = np.array([0.0, -0.0, 65504.0, 65519.99, 65520.0, 65536.0, 1e-8, 2.0 ** -24, 2.0 ** -25,
                         3 * 2.0 ** -26, 2.0 ** -14, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, np.inf, -np.inf,
                         -2.0 ** -25, 0.1, 255.0, 1.0 / 3.0], np.float32)
    vals = np.concatenate([specials,
                           g.uniform(-70000, 70000, 3000).astype(np.float32),
                           (g.standard_normal(3000) * 2.0 ** g.integers(-30, 16, 3000)).astype(np.float32)])
    got = oracle.float_to_half(vals)
    exp = vals.astype(np.float16).view(np.uint16)
    np.testing.assert_array_equal(got, exp)


def test_fp16_output_is_rne_of_fp32_result():
    g = datagen.rng(12)
    fr = datagen.frame(g, 9, 11, 3)
    ops = [{"kind": "mul", "k": [0.3]}, {"kind": "add", "k": [-20.5]}]
    r32 = oracle.run_chain(plain(ops=ops), [fr], [item(0, 0, 11, 9)])[0]["out"]
    r16 = oracle.run_chain(plain(ops=ops, out_dtype="f16"), [fr], [item(0, 0, 11, 9)])[0]["out"]
    np.testing.assert_array_equal(r16.view(np.uint16), r32.astype(np.float16).view(np.uint16))


@pytest.mark.parametrize("dt", ["f16", "f32"])
def test_float_inputs_read_exactly(dt):
    g = datagen.rng(13)
    fr = datagen.frame(g, 6, 10, 4, dtype=dt)
    out = oracle.run_chain(plain(C=4, dtype=dt), [fr], [item(1, 2, 8, 3)])[0]["out"]
    np.testing.assert_array_equal(out, fr[2:5, 1:9].astype(np.float32))


# ---------------------------------------------------------- validation --

@pytest.mark.parametrize("bad", [dict(x=-1), dict(y=-1), dict(w=0), dict(h=0), dict(x=101),
                                 dict(w=141), dict(y=51, h=50), dict(out_w=0), dict(out_h=-3)])
def test_invalid_items_are_rejected(bad):
    fr = np.zeros((100, 150, 3), np.uint8)
    good = item(10, 10, 50, 50, 20, 20)
    assert oracle.validate(resize_only(ow=20, oh=20), [fr], [good]) == 0
    good.update(bad)
    assert oracle.validate(resize_only(ow=20, oh=20), [fr], [good]) < 0


def test_bad_constant_counts_are_rejected():
    fr = np.zeros((10, 10, 3), np.uint8)
    ch = plain(ops=[{"kind": "mul", "k": [1.0, 2.0]}])
    assert oracle.validate(ch, [fr], [item(0, 0, 10, 10)]) < 0
    with pytest.raises(ValueError):
        oracle.run_chain(ch, [fr], [item(0, 0, 10, 10)])


def test_shadow_bounds_the_fp32_result():
    cfg = datagen.config0(seed=3, frame_hw=(200, 300), crop=(5, 6, 150, 120), out=(64, 128))
    r = oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"])[0]
    scale = np.maximum(np.abs(r["v64"]), r["smax"])
    assert np.all(np.abs(r["out"] - r["v64"]) <= 8 * 2.0 ** -24 * np.maximum(scale, 1.0))
    assert math.isfinite(float(r["out"].sum()))
