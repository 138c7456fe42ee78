"""Every launch configuration against the oracle.  Coarsened threads take
their units through registers in groups (fewer units than K where the
whole tile would spill): 4 of 3 channels, 2 of 4, half that for the
run-time op list into planar fp32, 1 for fp32 plain reads into planar
fp32.  Run-time op lists, the depth sweep's compile-time chains and the
normalise chain run at all 20 configurations (K = 1, 2, 4, 8 at every
block size), on frames whose rows end in a partial unit and whose items
span several tiles, and give the oracle's bits in the strict mode."""
import pytest

import datagen
import oracle
import paper_2508_07071_amd as fk
from fkhelpers import Plan, assert_bitexact, assert_close, host, to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


CASES = [
    # (read kind, input dtype, channels, output dtype, layout)
    ("plain", "u8", 3, "f32", "planar"),   # groups of 2
    ("plain", "f32", 3, "f32", "planar"),  # groups of 1
    ("plain", "f32", 4, "f32", "planar"),  # groups of 1
    ("plain", "u8", 4, "f16", "packed"),   # groups of 2
    ("plain", "f16", 3, "f32", "packed"),  # groups of 4
    ("plain", "u8", 1, "f32", "packed"),   # whole K
    ("crop_resize", "f32", 3, "f32", "packed"),
    ("crop_nearest", "u8", 4, "f32", "planar"),
]


@pytest.mark.parametrize("read,din,C,dout,layout", CASES)
def test_random_op_list_at_every_config_matches_oracle(read, din, C, dout, layout):
    say("unit groups", read, din, C, dout, layout)
    g = datagen.rng(700 + len(read) * 7 + C * 3 + len(din) + len(layout))
    ops = []
    for _ in range(int(g.integers(4, 12))):
        kind = datagen.OP_KINDS[int(g.integers(0, len(datagen.OP_KINDS)))]
        k = []
        if kind in ("mul", "div", "add", "sub"):
            lo, hi = (0.5, 1.5) if kind in ("mul", "div") else (-1.0, 1.0)
            k = [datagen.f32(g.uniform(lo, hi)) for _ in range(1 if g.uniform() < 0.5 else C)]
        ops.append({"kind": kind, "k": k})
    chain = {"read": {"kind": read, "dtype": din, "channels": C, "out_w": 0, "out_h": 0},
             "ops": ops, "write": {"dtype": dout, "layout": layout}}
    fh, fw = 67, 157  # rows of 157 pixels: 39 whole units and a partial one
    frames = [datagen.frame(g, fh, fw, C, dtype=din) for _ in range(2)]
    if read == "plain":
        items = [{"frame": 0, "x": 0, "y": 0, "w": fw, "h": fh},
                 {"frame": 1, "x": 5, "y": 3, "w": 131, "h": 41}]
    else:
        items = [{"frame": 0, "x": 2, "y": 1, "w": 150, "h": 60, "out_w": 133, "out_h": 47},
                 {"frame": 1, "x": 9, "y": 4, "w": 40, "h": 30, "out_w": 97, "out_h": 71}]
    refs = oracle.run_chain(chain, frames, items)
    dframes = to_dev(frames)
    with Plan(chain, len(items), strict=True, tier=fk.FK_TIER_RUNTIME) as p:
        assert fk.fk_plan_get_tier(p.h) == 0
        for c in fk.fk_autotune_space():
            p.set_config(c.block_threads, c.coarsen)
            outs = host(p.run(dframes, items))
            for b, (o, r) in enumerate(zip(outs, refs)):
                assert_bitexact(o, r["out"], f"{c} item {b}")


@pytest.mark.parametrize("n_ops", [16, 64, 256])
def test_compile_time_depth_chains_at_every_config_match_oracle(n_ops):
    """The depth sweep's compile-time chains (groups of 4 units at K = 8)
    at all 20 configurations, both modes: strict bits against the oracle,
    contracted results within tolerance."""
    say("compile-time chain, every config", n_ops)
    cfg = datagen.config1(n_ops, seed=3, frame_hw=(37, 301))
    chain, frames, items = cfg["chain"], cfg["frames"], cfg["items"]
    refs = oracle.run_chain(chain, frames, items)
    dframes = to_dev(frames)
    for strict in (True, False):
        with Plan(chain, 1, strict=strict) as p:
            assert fk.fk_plan_get_tier(p.h) == 1
            for c in fk.fk_autotune_space():
                p.set_config(c.block_threads, c.coarsen)
                out = host(p.run(dframes, items))[0]
                if strict:
                    assert_bitexact(out, refs[0]["out"], f"{c}")
                else:
                    assert_close(out, refs[0], what=f"{c}")


def test_normalize_chain_at_every_config_matches_oracle():
    """The hot chain (crop+resize, swap, cvt, mul, sub, div, planar fp32) at
    all 20 configurations in the strict mode, items of 4-pixel units (below
    2^20 output pixels)."""
    say("normalise chain, every config")
    cfg = datagen.config2(9, seed=5)
    refs = oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"])
    dframes = to_dev(cfg["frames"])
    with Plan(cfg["chain"], 9, strict=True) as p:
        for c in fk.fk_autotune_space():
            p.set_config(c.block_threads, c.coarsen)
            outs = host(p.run(dframes, cfg["items"]))
            for b, (o, r) in enumerate(zip(outs, refs)):
                assert_bitexact(o, r["out"], f"{c} item {b}")
