"""The other read ops on the GPU, through the C ABI, against the oracle:
nearest-neighbour crop+resize (u8/fp16/fp32 frames, 1/3/4 channels) and
NV12 reads (BT.601 limited range to BGR) with and without a bilinear
resize.  Strict plans are bit-exact; default plans within
|g - r| <= 1e-5 * max(|r|, s)."""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_2508_07071_amd as fk
from fkhelpers import Plan, assert_bitexact, assert_close, host, to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def norm_ops(C):
    return [{"kind": "swap", "k": []}, {"kind": "cvt", "k": []},
            {"kind": "mul", "k": [datagen.NORM_SCALE]},
            {"kind": "sub", "k": (datagen.NORM_MEAN + [0.5])[:C] if C > 1 else [0.45]},
            {"kind": "div", "k": (datagen.NORM_STD + [0.25])[:C] if C > 1 else [0.226]}]


def both_modes(chain, frames, items, what, unfused=False):
    refs = oracle.run_chain(chain, frames, items)
    dframes = to_dev(frames)
    for strict in (True, False):
        with Plan(chain, len(items), strict=strict) as p:
            outs = host(p.run(dframes, items))
            uouts = host(p.run_unfused(dframes, items)) if (unfused and strict) else None
        for b, (g, r) in enumerate(zip(outs, refs)):
            if strict:
                assert_bitexact(g, r["out"], f"{what} strict item {b}")
                if uouts is not None:
                    assert_bitexact(uouts[b], r["out"], f"{what} unfused item {b}")
            else:
                assert_close(g, r, what=f"{what} item {b}")


@pytest.mark.parametrize("dtype", ["u8", "f16", "f32"])
@pytest.mark.parametrize("C", [1, 3, 4])
def test_nearest_crops_match_oracle(dtype, C):
    say("nearest", dtype, C)
    g = datagen.rng(C * 7 + len(dtype))
    fr = datagen.frame(g, 300, 410, C, dtype=dtype)
    items = datagen.random_crops(g, 9, 410, 300, lo=3, hi=290, out=(61, 37))
    items += [{"frame": 0, "x": 5, "y": 6, "w": 20, "h": 10, "out_w": 160, "out_h": 30},   # upscale
              {"frame": 0, "x": 0, "y": 0, "w": 410, "h": 300, "out_w": 7, "out_h": 5},  # strong downscale
              {"frame": 0, "x": 100, "y": 100, "w": 1, "h": 1, "out_w": 9, "out_h": 3}]  # one pixel
    for layout in ("packed", "planar"):
        ch = {"read": {"kind": "crop_nearest", "dtype": dtype, "channels": C, "out_w": 0, "out_h": 0},
              "ops": norm_ops(C), "write": {"dtype": "f32", "layout": layout}}
        both_modes(ch, [fr], items, f"nearest {dtype}x{C} {layout}", unfused=layout == "planar")


@pytest.mark.parametrize("kind", ["nv12", "nv12_resize"])
@pytest.mark.parametrize("out_dtype,layout", [("f32", "planar"), ("f16", "packed"), ("f32", "packed")])
def test_nv12_reads_match_oracle(kind, out_dtype, layout):
    say(kind, out_dtype, layout)
    g = datagen.rng(11 if kind == "nv12" else 12)
    fr = datagen.nv12_frame(g, 480, 640)
    if kind == "nv12":
        items = [{"frame": 0, "x": x, "y": y, "w": w, "h": h, "out_w": w, "out_h": h}
                 for x, y, w, h in ((0, 0, 640, 480), (3, 5, 17, 11), (101, 77, 254, 133), (639, 479, 1, 1))]
    else:
        items = datagen.random_crops(g, 6, 640, 480, lo=2, hi=400, out=(64, 128))
        items.append({"frame": 0, "x": 1, "y": 1, "w": 9, "h": 7, "out_w": 224, "out_h": 224})
    ch = {"read": {"kind": kind, "dtype": "u8", "channels": 3, "out_w": 0, "out_h": 0},
          "ops": norm_ops(3), "write": {"dtype": out_dtype, "layout": layout}}
    both_modes(ch, [fr], items, f"{kind} {out_dtype} {layout}", unfused=out_dtype == "f32")


def test_nv12_dword_units_and_byte_units():
    """The 1:1 NV12 read takes a whole unit as one luma and one chroma dword
    when the frame base, pitch and ROI column are multiples of 4, byte by
    byte otherwise: ROIs at columns 0, 4, 8, 636 (dwords) and 1, 2, 6
    (bytes), odd and even first rows, ragged widths; a batch of equal-sized
    crops (the compact kernel-argument form) mixing both; and a frame base
    2 bytes past a dword boundary (bytes everywhere)."""
    say("nv12 dword and byte units")
    g = datagen.rng(19)
    fr = datagen.nv12_frame(g, 60, 640)
    ch = {"read": {"kind": "nv12", "dtype": "u8", "channels": 3, "out_w": 0, "out_h": 0},
          "ops": norm_ops(3), "write": {"dtype": "f32", "layout": "planar"}}
    rois = [(0, 0, 640, 60), (4, 3, 21, 9), (8, 1, 100, 50), (636, 59, 4, 1), (1, 2, 33, 7), (2, 5, 64, 4),
            (6, 7, 11, 13)]
    items = [{"frame": 0, "x": x, "y": y, "w": w, "h": h, "out_w": w, "out_h": h} for x, y, w, h in rois]
    both_modes(ch, [fr], items, "nv12 mixed", unfused=True)
    same = [{"frame": 0, "x": x, "y": y, "w": 24, "h": 6, "out_w": 24, "out_h": 6}
            for x, y in ((0, 0), (4, 1), (5, 2), (12, 9), (600, 54), (3, 3))]
    both_modes(ch, [fr], same, "nv12 compact")
    # a frame 2 bytes past a dword boundary
    buf = torch.zeros(fr.size + 64, dtype=torch.uint8, device="cuda:0")
    buf[2:2 + fr.size] = torch.from_numpy(fr.reshape(-1)).to("cuda:0")
    dfr = buf[2:2 + fr.size].view(fr.shape)
    refs = oracle.run_chain(ch, [fr], items[:3])
    with Plan(ch, 3, strict=True) as p:
        outs = host(p.run([dfr], items[:3]))
    for b, (o, r) in enumerate(zip(outs, refs)):
        assert_bitexact(o, r["out"], f"nv12 offset base item {b}")


def test_nv12_frame_with_row_padding():
    """An NV12 frame whose rows are padded (pitch 704 for 640 pixels): both
    planes follow the pitch."""
    say("nv12 padded rows")
    g = datagen.rng(13)
    dense = datagen.nv12_frame(g, 96, 640)
    padded = np.zeros((144, 704), np.uint8)
    padded[:, :640] = dense
    items = [{"frame": 0, "x": 13, "y": 9, "w": 300, "h": 70, "out_w": 64, "out_h": 128}]
    ch = {"read": {"kind": "nv12_resize", "dtype": "u8", "channels": 3, "out_w": 0, "out_h": 0},
          "ops": norm_ops(3), "write": {"dtype": "f32", "layout": "planar"}}
    ref = oracle.run_chain(ch, [dense], items)[0]
    dfr = torch.from_numpy(padded).cuda()[:, :640]  # a strided view: pitch 704 bytes
    with Plan(ch, 1, strict=True) as p:
        out = host(p.run([dfr], items))[0]
    assert_bitexact(out, ref["out"], "padded nv12")


def test_stats_over_nearest_and_nv12_reads():
    say("stats over nearest / nv12")
    g = datagen.rng(14)
    cases = [({"kind": "crop_nearest", "dtype": "u8", "channels": 3}, datagen.frame(g, 200, 300, 3)),
             ({"kind": "nv12_resize", "dtype": "u8", "channels": 3}, datagen.nv12_frame(g, 200, 300)),
             ({"kind": "nv12", "dtype": "u8", "channels": 3}, datagen.nv12_frame(g, 200, 300))]
    for read, fr in cases:
        read = dict(read, out_w=0, out_h=0)
        items = datagen.random_crops(g, 5, 300, 200, lo=10, hi=180, out=(50, 70))
        if read["kind"] == "nv12":
            # 1:1 reads: ROIs at dword columns (whole units as dwords) and not
            one = []
            for b, it in enumerate(items):
                x = it["x"] & ~3 if b % 2 else it["x"] | 1
                w = min(it["w"], 300 - x)
                one.append(dict(it, x=x, w=w, out_w=w, out_h=it["h"]))
            items = one
        img = {"read": read, "ops": norm_ops(3), "write": {"dtype": "f32", "layout": "packed"}}
        st = dict(img, write={"dtype": "f64", "layout": "stats"})
        imgs = oracle.run_chain(img, [fr], items)
        sts = oracle.run_chain(st, [fr], items)
        with Plan(st, len(items), strict=True) as p:
            outs = host(p.run(to_dev([fr]), items))
        for b, (o, s_, im) in enumerate(zip(outs, sts, imgs)):
            v = im["out"].reshape(-1, 3).astype(np.float64)
            n = v.shape[0]
            np.testing.assert_array_equal(o[:, :2], s_["out"][:, :2])
            bound = 2 * (n - 1) * 2.0 ** -53 * np.abs(v).sum(0)
            assert np.all(np.abs(o[:, 2] - s_["out"][:, 2]) <= bound), (read["kind"], b)


@pytest.mark.parametrize("kind,dtype,C,out_dtype", [
    ("crop_nearest", "u8", 3, "f32"), ("crop_nearest", "f16", 1, "f16"), ("crop_nearest", "f32", 4, "f32"),
    ("crop_resize", "u8", 3, "f16"), ("crop_resize", "f16", 3, "f32"), ("crop_resize", "f32", 1, "f32"),
    ("nv12", "u8", 3, "f32"), ("nv12_resize", "u8", 3, "f16")])
def test_large_planar_gathers_match_oracle(kind, dtype, C, out_dtype):
    """Launches of at least 2^20 output pixels with a planar write: the
    bilinear reads take the pixel-strided layout (run-time op list), the
    others keep 4-pixel units; the same bits as the oracle in the strict
    mode, within tolerance otherwise, for a large crop and a batch."""
    say("large planar gather", kind, dtype, C, out_dtype)
    g = datagen.rng(31 + C + len(kind) + len(dtype))
    if kind.startswith("nv12"):
        fr = datagen.nv12_frame(g, 832, 1280)
        fh, fw = 832, 1280
    else:
        fh, fw = 700, 900
        fr = datagen.frame(g, fh, fw, C, dtype=dtype)
    if kind == "nv12":
        items = [{"frame": 0, "x": 0, "y": 0, "w": 1280, "h": 832, "out_w": 1280, "out_h": 832},
                 {"frame": 0, "x": 7, "y": 3, "w": 333, "h": 101, "out_w": 333, "out_h": 101}]
    else:
        items = [{"frame": 0, "x": 11, "y": 5, "w": fw - 30, "h": fh - 21, "out_w": 1100, "out_h": 960}]
        items += datagen.random_crops(g, 5, fw, fh, lo=3, hi=500, out=(97, 61))
    ch = {"read": {"kind": kind, "dtype": dtype, "channels": C, "out_w": 0, "out_h": 0},
          "ops": norm_ops(C), "write": {"dtype": out_dtype, "layout": "planar"}}
    assert sum(it["out_w"] * it["out_h"] for it in items) >= 1 << 20
    both_modes(ch, [fr], items, f"large {kind} {dtype}x{C} -> {out_dtype}")
