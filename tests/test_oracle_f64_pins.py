"""Pins of the oracle's double-precision chains (the data-type experiment,
Section VI-I: float->double and double->double compute in double).  A chain
with an fp64 write runs every op as one IEEE fp64 operation; the pins
compare each element with exact rational arithmetic rounded once per op to
the nearest double (Python's Fraction -> float conversion rounds correctly,
ties to even), so a chain computed in fp32, a dropped or reordered op, or a
constant not taken exactly as its fp32 value fails.  CPU only."""
from fractions import Fraction

import numpy as np
import pytest

import datagen
import oracle


def chain(in_dtype, ops, layout="packed", channels=1, out="f64"):
    return {"read": {"kind": "plain", "dtype": in_dtype, "channels": channels, "out_w": 0, "out_h": 0},
            "ops": ops, "write": {"dtype": out, "layout": layout}}


def exact_chain(x, ops, c=0):
    """The chain on one value: each op exact in rationals, then rounded to the
    nearest double."""
    v = float(x)
    for op in ops:
        if op["kind"] in ("cvt", "swap"):
            continue
        k = op["k"][0] if len(op["k"]) == 1 else op["k"][c]
        a, b = Fraction(v), Fraction(float(np.float32(k)))
        r = {"mul": a * b, "add": a + b, "sub": a - b, "div": a / b}[op["kind"]]
        v = float(r)
    return v


NORM_OPS = [{"kind": "cvt", "k": []}, {"kind": "mul", "k": [datagen.f32(1.0 / 3.0)]},
            {"kind": "sub", "k": [datagen.f32(0.1)]}, {"kind": "div", "k": [datagen.f32(0.7)]}]


@pytest.mark.parametrize("in_dtype", ["u8", "f16", "f32", "f64"])
def test_each_op_rounds_once_to_double(in_dtype):
    g = datagen.rng(41)
    fr = datagen.frame(g, 12, 17, 1, dtype=in_dtype)
    if in_dtype == "f64":
        fr = fr + g.uniform(0, 1e-6, size=fr.shape)  # use the low mantissa bits too
    it = {"frame": 0, "x": 2, "y": 3, "w": 13, "h": 7}
    out = oracle.run_chain(chain(in_dtype, NORM_OPS), [fr], [it])[0]["out"]
    assert out.dtype == np.float64
    roi = fr[3:10, 2:15, 0]
    for (j, i), x in np.ndenumerate(roi):
        want = exact_chain(float(x), NORM_OPS)
        assert out[j, i, 0] == want, (in_dtype, j, i, x, out[j, i, 0], want)


def test_double_chain_differs_from_the_fp32_chain():
    """The same chain with an fp32 write (every op rounded to fp32) differs
    from the fp64 write in most elements: the write's type sets the
    arithmetic type."""
    g = datagen.rng(42)
    fr = datagen.frame(g, 8, 8, 1, dtype="f32")
    it = {"frame": 0, "x": 0, "y": 0, "w": 8, "h": 8}
    d = oracle.run_chain(chain("f32", NORM_OPS), [fr], [it])[0]["out"]
    f = oracle.run_chain(chain("f32", NORM_OPS, out="f32"), [fr], [it])[0]["out"]
    assert np.mean(d != f.astype(np.float64)) > 0.5
    assert np.max(np.abs(d - f) / np.abs(d)) < 1e-6


def test_identity_chain_keeps_every_double():
    vals = np.array([0.0, -0.0, 5e-324, -2.2250738585072014e-308, 1.7976931348623157e308, np.inf,
                     -np.inf, 1.0 / 3.0, np.pi, -123456789.123456789, 2.0 ** -1074 * 3, 1e-300],
                    np.float64).reshape(3, 4, 1)
    it = {"frame": 0, "x": 0, "y": 0, "w": 4, "h": 3}
    out = oracle.run_chain(chain("f64", [{"kind": "cvt", "k": []}]), [vals], [it])[0]["out"]
    assert np.array_equal(out.view(np.uint64), vals.view(np.uint64))


def test_planar_split_swap_and_per_channel_constants_in_double():
    """An fp64 frame holding each element's linear index: the planar write
    puts channel c of pixel (x, y) at plane c (after the swap of channels 0
    and 2), and per-channel constants follow the swapped positions."""
    H, W, C = 5, 6, 3
    fr = np.arange(H * W * C, dtype=np.float64).reshape(H, W, C)
    ops = [{"kind": "swap", "k": []}, {"kind": "mul", "k": [2.0, 4.0, 8.0]}, {"kind": "add", "k": [0.5]}]
    it = {"frame": 0, "x": 1, "y": 2, "w": 4, "h": 3}
    out = oracle.run_chain(chain("f64", ops, layout="planar", channels=3), [fr], [it])[0]["out"]
    assert out.shape == (3, 3, 4)
    for c in range(3):
        for y in range(3):
            for x in range(4):
                src = fr[2 + y, 1 + x, 2 - c]
                assert out[c, y, x] == src * [2.0, 4.0, 8.0][c] + 0.5


def test_loop_in_double_is_the_unrolled_chain():
    g = datagen.rng(43)
    fr = datagen.frame(g, 4, 5, 1, dtype="f64")
    body = [{"kind": "mul", "k": [datagen.f32(1.01)]}, {"kind": "add", "k": [datagen.f32(-0.3)]}]
    looped = [{"kind": "cvt", "k": []}] + body + [{"kind": "loop", "k": [], "span": 2, "count": 7}]
    unrolled = [{"kind": "cvt", "k": []}] + body * 7
    it = {"frame": 0, "x": 0, "y": 0, "w": 5, "h": 4}
    a = oracle.run_chain(chain("f64", looped), [fr], [it])[0]["out"]
    b = oracle.run_chain(chain("f64", unrolled), [fr], [it])[0]["out"]
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    for (j, i), x in np.ndenumerate(fr[:, :, 0]):
        assert a[j, i, 0] == exact_chain(x, unrolled)


@pytest.mark.parametrize("bad", [
    {"read": "crop_resize", "in": "f32", "out": "f64", "layout": "planar"},   # fp64 chains: plain reads only
    {"read": "plain", "in": "f64", "out": "f32", "layout": "packed"},         # fp64 frame needs an fp64 write
    {"read": "plain", "in": "f64", "out": "f64", "layout": "stats"},          # the stats write reduces fp32 values
])
def test_rejected_double_chains(bad):
    c = chain(bad["in"], [{"kind": "cvt", "k": []}], layout=bad["layout"], out=bad["out"])
    c["read"]["kind"] = bad["read"]
    fr = np.zeros((4, 4, 1), datagen.DTYPES[bad["in"]])
    it = {"frame": 0, "x": 0, "y": 0, "w": 4, "h": 4, "out_w": 2, "out_h": 2}
    assert oracle.validate(c, [fr], [it]) != 0
