"""Pins of the oracle's stats write (per channel min, max, sum, mean of the
chain's fp32 values from one read; the reduction pattern of Section IV-C)
against closed forms on coordinate-coded frames, numpy's min/max and an
exactly rounded sum (math.fsum), and NaN/inf special cases."""
import math

import numpy as np
import pytest

import datagen
import oracle


def stats_chain(C=3, kind="plain", dtype="u8", ops=None, ow=0, oh=0):
    return {"read": {"kind": kind, "dtype": dtype, "channels": C, "out_w": ow, "out_h": oh},
            "ops": ops or [], "write": {"dtype": "f64", "layout": "stats"}}


def image_chain(ch):
    return dict(ch, write={"dtype": "f32", "layout": "packed"})


def coord_frame(H=300, W=280):
    """Channel 0 = x mod 256, channel 1 = y mod 256, channel 2 = 7."""
    fr = np.zeros((H, W, 3), np.uint8)
    fr[:, :, 0] = (np.arange(W) % 256)[None, :]
    fr[:, :, 1] = (np.arange(H) % 256)[:, None]
    fr[:, :, 2] = 7
    return fr


@pytest.mark.parametrize("roi", [(0, 0, 1, 1), (3, 5, 17, 9), (10, 40, 200, 150), (255, 0, 1, 256)])
def test_stats_of_coordinate_ramps_are_closed_forms(roi):
    x0, y0, w, h = roi
    fr = coord_frame()
    out = oracle.run_chain(stats_chain(), [fr], [{"frame": 0, "x": x0, "y": y0, "w": w, "h": h}])[0]["out"]
    n = w * h
    sx = h * w * (2 * x0 + w - 1) / 2  # sum over the ROI of x, exact in fp64 at these sizes
    sy = w * h * (2 * y0 + h - 1) / 2
    want = np.array([[x0, x0 + w - 1, sx, sx / n],
                     [y0, y0 + h - 1, sy, sy / n],
                     [7, 7, 7 * n, 7.0]])
    np.testing.assert_array_equal(out, want)


def test_stats_follow_ops_and_swap():
    """swap then *2 then +0.5: every value stays exact, so closed forms hold;
    the swap moves channel 2 (constant 7) to position 0."""
    fr = coord_frame()
    ops = [{"kind": "swap", "k": []}, {"kind": "cvt", "k": []},
           {"kind": "mul", "k": [2.0]}, {"kind": "add", "k": [0.5]}]
    x0, y0, w, h = 4, 6, 30, 20
    out = oracle.run_chain(stats_chain(ops=ops), [fr], [{"frame": 0, "x": x0, "y": y0, "w": w, "h": h}])[0]["out"]
    n = w * h
    sx = h * w * (2 * x0 + w - 1) / 2
    sy = w * h * (2 * y0 + h - 1) / 2
    want = np.array([[14.5, 14.5, 14.5 * n, 14.5],
                     [2 * y0 + 0.5, 2 * (y0 + h - 1) + 0.5, 2 * sy + 0.5 * n, (2 * sy + 0.5 * n) / n],
                     [2 * x0 + 0.5, 2 * (x0 + w - 1) + 0.5, 2 * sx + 0.5 * n, (2 * sx + 0.5 * n) / n]])
    np.testing.assert_array_equal(out, want)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_stats_match_numpy_and_exactly_rounded_sum(seed):
    """Random crop+resize chains with arithmetic: min/max equal numpy's over
    the chain's image; the fp64 running sum is within (n - 1) u sum|x| of the
    exactly rounded sum (u = 2^-53); mean = sum / n."""
    g = datagen.rng(seed)
    C = [1, 3, 4][seed]
    fr = datagen.frame(g, 90, 130, C)
    ops = [{"kind": "cvt", "k": []}, {"kind": "mul", "k": [datagen.f32(g.uniform(-1.5, 1.5))]},
           {"kind": "sub", "k": [datagen.f32(g.uniform(-50, 50)) for _ in range(C)]},
           {"kind": "div", "k": [datagen.f32(g.uniform(0.5, 3.0))]}]
    ch = stats_chain(C=C, kind="crop_resize", ops=ops, ow=57, oh=33)
    it = [{"frame": 0, "x": 11, "y": 7, "w": 101, "h": 70, "out_w": 57, "out_h": 33}]
    st = oracle.run_chain(ch, [fr], it)[0]["out"]
    img = oracle.run_chain(image_chain(ch), [fr], it, shadow=False)[0]["out"].reshape(-1, C)
    n = img.shape[0]
    for c in range(C):
        v = img[:, c].astype(np.float64)
        assert st[c, 0] == v.min() and st[c, 1] == v.max()
        exact = math.fsum(v)
        assert abs(st[c, 2] - exact) <= (n - 1) * 2.0 ** -53 * np.abs(v).sum()
        assert st[c, 3] == st[c, 2] / n


def test_stats_skip_nan_in_min_max_and_propagate_into_sum():
    fr = np.array([[[1.0, 5.0], [np.nan, -2.0], [3.0, np.inf]]], np.float32)  # 1 x 3 x 2
    out = oracle.run_chain(stats_chain(C=1, dtype="f32"), [fr[:, :, :1].copy()],
                           [{"frame": 0, "x": 0, "y": 0, "w": 3, "h": 1}])[0]["out"]
    assert out[0, 0] == 1.0 and out[0, 1] == 3.0
    assert np.isnan(out[0, 2]) and np.isnan(out[0, 3])
    out = oracle.run_chain(stats_chain(C=1, dtype="f32"), [fr[:, :, 1:].copy()],
                           [{"frame": 0, "x": 0, "y": 0, "w": 3, "h": 1}])[0]["out"]
    assert out[0, 0] == -2.0 and out[0, 1] == np.inf and out[0, 2] == np.inf


def test_stats_write_requires_f64_and_f64_images_need_a_plain_read():
    """The stats write produces fp64 only; an fp64 image write is a
    double-precision chain, which only the plain read takes."""
    fr = np.zeros((4, 4, 3), np.uint8)
    it = [{"frame": 0, "x": 0, "y": 0, "w": 4, "h": 4, "out_w": 2, "out_h": 2}]
    assert oracle.validate(stats_chain(), [fr], it) == 0
    bad = stats_chain()
    bad["write"]["dtype"] = "f32"
    assert oracle.validate(bad, [fr], it) < 0
    dbl = image_chain(stats_chain())
    dbl["write"]["dtype"] = "f64"
    assert oracle.validate(dbl, [fr], it) == 0
    bad = image_chain(stats_chain(kind="crop_resize", ow=2, oh=2))
    bad["write"]["dtype"] = "f64"
    assert oracle.validate(bad, [fr], it) < 0
