"""Pins of the oracle's other read ops: the nearest-neighbour resize and the
NV12 read (BT.601 limited-range YUV -> BGR) with and without a bilinear
resize, against closed forms, the BT.601 colour table, torch's
nearest-exact and bilinear interpolation, and structural invariants."""
import numpy as np
import pytest
import torch

import datagen
import oracle


def chain(kind, C=3, dtype="u8", ow=0, oh=0, ops=None):
    return {"read": {"kind": kind, "dtype": dtype, "channels": C, "out_w": ow, "out_h": oh},
            "ops": ops or [], "write": {"dtype": "f32", "layout": "packed"}}


def item(x, y, w, h, ow=None, oh=None):
    return {"frame": 0, "x": x, "y": y, "w": w, "h": h,
            "out_w": w if ow is None else ow, "out_h": h if oh is None else oh}


def run(ch, fr, it):
    return oracle.run_chain(ch, [fr], [it])[0]["out"]


# ------------------------------------------------------------- nearest --

def test_nearest_same_size_is_the_crop():
    g = datagen.rng(0)
    fr = datagen.frame(g, 40, 50, 3)
    out = run(chain("crop_nearest"), fr, item(3, 4, 30, 20, 30, 20))
    np.testing.assert_array_equal(out, fr[4:24, 3:33].astype(np.float32))


@pytest.mark.parametrize("f", [2, 3, 4])
def test_nearest_integer_upscale_replicates(f):
    g = datagen.rng(f)
    fr = datagen.frame(g, 9, 11, 1)
    out = run(chain("crop_nearest", C=1), fr, item(0, 0, 11, 9, 11 * f, 9 * f))
    want = np.repeat(np.repeat(fr, f, axis=0), f, axis=1).astype(np.float32)
    np.testing.assert_array_equal(out, want)


@pytest.mark.parametrize("f", [2, 3, 5])
def test_nearest_integer_downscale_takes_centre_pixel(f):
    """Output o covers source pixels f*o .. f*o + f - 1; its centre lies in
    pixel f*o + floor(f / 2)."""
    g = datagen.rng(10 + f)
    fr = datagen.frame(g, 7 * f, 6 * f, 3)
    out = run(chain("crop_nearest"), fr, item(0, 0, 6 * f, 7 * f, 6, 7))
    np.testing.assert_array_equal(out, fr[f // 2::f, f // 2::f].astype(np.float32))


@pytest.mark.parametrize("src,dst", [((37, 53), (64, 29)), ((100, 61), (224, 224)), ((480, 640), (128, 64))])
def test_nearest_matches_torch_nearest_exact_off_boundaries(src, dst):
    """torch's nearest-exact picks floor((o + 0.5) * in / out) in floating
    point; the oracle's exact integer form agrees wherever the centre does
    not fall exactly on a pixel boundary."""
    (h, w), (oh, ow) = src, dst
    fr = np.arange(h * w, dtype=np.float32).reshape(h, w, 1)
    out = run(chain("crop_nearest", C=1, dtype="f32"), fr, item(0, 0, w, h, ow, oh))[:, :, 0]
    t = torch.nn.functional.interpolate(torch.from_numpy(fr[:, :, 0]).double()[None, None], size=(oh, ow),
                                        mode="nearest-exact")[0, 0].numpy()
    oy = np.arange(oh)[:, None]
    ox = np.arange(ow)[None, :]
    on_edge = (((2 * oy + 1) * h) % (2 * oh) == 0) | (((2 * ox + 1) * w) % (2 * ow) == 0)
    np.testing.assert_array_equal(out[~on_edge], t[~on_edge])


# ---------------------------------------------------------------- NV12 --

def nv12_const(h, w, Y, U, V):
    fr = np.empty((h * 3 // 2, w), np.uint8)
    fr[:h] = Y
    fr[h:, 0::2] = U
    fr[h:, 1::2] = V
    return fr


# BT.601 limited-range YCbCr of the 100% colours, with their RGB
BT601 = [((16, 128, 128), (0, 0, 0)), ((235, 128, 128), (255, 255, 255)),
         ((81, 90, 240), (255, 0, 0)), ((145, 54, 34), (0, 255, 0)), ((41, 240, 110), (0, 0, 255)),
         ((210, 16, 146), (255, 255, 0)), ((170, 166, 16), (0, 255, 255)), ((106, 202, 222), (255, 0, 255))]


@pytest.mark.parametrize("yuv,rgb", BT601)
def test_nv12_bt601_colour_table(yuv, rgb):
    """Each standard colour comes back within 2 levels (the table's 8-bit
    rounding and the matrix's 3-4 digit coefficients); channels are B, G, R."""
    out = run(chain("nv12"), nv12_const(4, 6, *yuv), item(0, 0, 6, 4))
    bgr = np.array(rgb[::-1], np.float32)
    assert np.all(np.abs(out - bgr) <= 2.0), (yuv, out[0, 0])


def test_nv12_grey_has_equal_channels_and_is_linear_in_luma():
    fr = nv12_const(2, 256, 0, 128, 128)
    fr[0, :] = np.arange(256)
    fr[1, :] = np.arange(256)
    out = run(chain("nv12"), fr, item(0, 0, 256, 2))
    assert np.array_equal(out[..., 0], out[..., 1]) and np.array_equal(out[..., 1], out[..., 2])
    d = np.diff(out[0, :, 0].astype(np.float64))
    np.testing.assert_allclose(d, 1.164, atol=1e-4)  # one luma level = 1.164 levels
    assert out[0, 16, 0] == 0.0


def test_nv12_chroma_pair_serves_a_2x2_block():
    """Constant luma, chroma different at every chroma site: the four pixels
    of each 2x2 block agree, and neighbouring blocks differ."""
    g = datagen.rng(5)
    h, w = 8, 12
    fr = nv12_const(h, w, 120, 0, 0)
    fr[h:] = g.integers(0, 256, size=(h // 2, w), dtype=np.uint8)
    out = run(chain("nv12"), fr, item(0, 0, w, h))
    blocks = out.reshape(h // 2, 2, w // 2, 2, 3)
    assert np.all(blocks == blocks[:, :1, :, :1])
    # every block has its own chroma site: neighbours along x and y differ
    assert np.all(np.any(np.diff(blocks[:, 0, :, 0], axis=1) != 0, axis=-1))
    assert np.all(np.any(np.diff(blocks[:, 0, :, 0], axis=0) != 0, axis=-1))


def test_nv12_crop_uses_absolute_chroma_sites():
    """An ROI at odd offsets reads the same pixels as the full frame."""
    g = datagen.rng(6)
    fr = datagen.nv12_frame(g, 20, 30)
    full = run(chain("nv12"), fr, item(0, 0, 30, 20))
    crop = run(chain("nv12"), fr, item(3, 5, 17, 11))
    np.testing.assert_array_equal(crop, full[5:16, 3:20])


def test_nv12_resize_same_size_is_nv12_crop_and_matches_torch_bilinear():
    g = datagen.rng(7)
    fr = datagen.nv12_frame(g, 60, 80)
    crop = run(chain("nv12"), fr, item(7, 9, 41, 33))
    same = run(chain("nv12_resize", ow=41, oh=33), fr, item(7, 9, 41, 33, 41, 33))
    np.testing.assert_array_equal(same, crop)
    out = run(chain("nv12_resize", ow=64, oh=48), fr, item(7, 9, 41, 33, 64, 48))
    src = torch.from_numpy(crop.astype(np.float64)).permute(2, 0, 1)[None]
    t = torch.nn.functional.interpolate(src, size=(48, 64), mode="bilinear", align_corners=False,
                                        antialias=False)[0].permute(1, 2, 0).numpy()
    np.testing.assert_allclose(out, t, atol=2e-3)


def test_nv12_requires_u8_three_channels_and_even_frames():
    fr = nv12_const(4, 6, 100, 128, 128)
    assert oracle.validate(chain("nv12"), [fr], [item(0, 0, 6, 4)]) == 0
    assert oracle.validate(chain("nv12", C=1), [fr], [item(0, 0, 6, 4)]) < 0
    odd = np.zeros((6, 5), np.uint8)  # 4 x 5 luma: odd width
    assert oracle.validate(chain("nv12"), [odd], [item(0, 0, 5, 4)]) < 0
