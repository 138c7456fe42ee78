"""Chains with no compute op (read -> write): every read kind, input dtype
and channel count, into planar fp32, packed fp16 and the stats write, on a
ragged ROI, against the oracle.  Without ops the read's value (the
element, the resized fp32 value or the converted NV12 value) is what the
write stores, rounded to its type."""
import pytest

import datagen
import oracle
from fkhelpers import Plan, assert_bitexact, host, to_dev
from test_gpu_stats import check, image_of, stats_of

pytestmark = pytest.mark.gpu

CASES = [(k, d, c) for k in ("plain", "crop_resize", "crop_nearest") for d in ("u8", "f16", "f32")
         for c in (1, 3, 4)] + [("nv12", "u8", 3), ("nv12_resize", "u8", 3)]


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("kind,dtype,C", CASES)
def test_chain_without_ops_matches_oracle(kind, dtype, C):
    say("no ops", kind, dtype, C)
    g = datagen.rng(400 + CASES.index((kind, dtype, C)))
    nv12 = kind.startswith("nv12")
    fr = datagen.nv12_frame(g, 42, 66) if nv12 else datagen.frame(g, 41, 67, C, dtype=dtype)
    one_to_one = kind in ("plain", "nv12")
    items = [{"frame": 0, "x": 3, "y": 5, "w": 37, "h": 19,
              "out_w": 37 if one_to_one else 29, "out_h": 19 if one_to_one else 31},
             {"frame": 0, "x": 0, "y": 0, "w": 1, "h": 1,
              "out_w": 1 if one_to_one else 5, "out_h": 1 if one_to_one else 3}]
    read = {"kind": kind, "dtype": dtype, "channels": C, "out_w": 0, "out_h": 0}
    dframes = to_dev([fr])
    for write in ({"dtype": "f32", "layout": "planar"}, {"dtype": "f16", "layout": "packed"}):
        ch = {"read": read, "ops": [], "write": write}
        refs = oracle.run_chain(ch, [fr], items)
        with Plan(ch, len(items), strict=True) as p:
            outs = host(p.run(dframes, items))
        for b, (o, r) in enumerate(zip(outs, refs)):
            assert_bitexact(o, r["out"], f"{kind} {dtype}x{C} -> {write} item {b}")
    ch = {"read": read, "ops": [], "write": {"dtype": "f32", "layout": "packed"}}
    st = [r["out"] for r in oracle.run_chain(stats_of(ch), [fr], items)]
    ims = oracle.run_chain(image_of(ch), [fr], items)
    with Plan(stats_of(ch), len(items), strict=True) as p:
        outs = host(p.run(dframes, items))
    for b, o in enumerate(outs):
        check(o, st[b], ims[b], True, f"{kind} {dtype}x{C} stats item {b}")
