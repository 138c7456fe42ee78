"""Double-precision chains on the GPU (the data-type experiment's float->
double and double->double pairs, Section VI-I): a plain read with an fp64
write runs the op list in fp64.  Strict plans match the oracle bit for bit,
contracted plans (Mul+Add/Sub as one fp64 FMA) within 1e-13 relative to
max(|r|, s), and the unfused baseline gives the strict bits; every launch
configuration, the table path and graph replays give the same bits."""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_2508_07071_amd as fk
from fkhelpers import Plan, alloc_outs, assert_bitexact, assert_close, host, to_dev

pytestmark = pytest.mark.gpu
REL64 = 1e-13


def say(*a):
    print("[case]", *a, flush=True)


def chain3(din, layout):
    return {"read": {"kind": "plain", "dtype": din, "channels": 3, "out_w": 0, "out_h": 0},
            "ops": [{"kind": "swap", "k": []}, {"kind": "cvt", "k": []},
                    {"kind": "mul", "k": [datagen.f32(1 / 255), datagen.f32(1 / 127), datagen.f32(1 / 63)]},
                    {"kind": "sub", "k": [datagen.f32(0.485), datagen.f32(0.456), datagen.f32(0.406)]},
                    {"kind": "div", "k": [datagen.f32(0.229), datagen.f32(0.224), datagen.f32(0.225)]}],
            "write": {"dtype": "f64", "layout": layout}}


def check(chain, frames, items, what, cfgs=((256, 1),), unfused=True):
    refs = oracle.run_chain(chain, frames, items)
    dframes = to_dev(frames)
    for cfg in cfgs:
        for strict in (True, False):
            with Plan(chain, len(items), strict=strict) as p:
                assert fk.fk_plan_get_tier(p.h) == 0  # the run-time op list
                p.set_config(*cfg)
                got = host(p.run(dframes, items))
                if strict and unfused and cfg == cfgs[0]:
                    ung = host(p.run_unfused(dframes, items))
            for b, (g, r) in enumerate(zip(got, refs)):
                assert g.dtype == np.float64
                if strict:
                    assert_bitexact(g, r["out"], f"{what} {cfg} strict item {b}")
                else:
                    assert_close(g, r, rel=REL64, what=f"{what} {cfg} item {b}")
            if strict and unfused and cfg == cfgs[0]:
                for b, (g, r) in enumerate(zip(ung, refs)):
                    assert_bitexact(g, r["out"], f"{what} unfused item {b}")


@pytest.mark.parametrize("din", ["u8", "f16", "f32", "f64"])
def test_cast_chain_batch50_to_double(din):
    say("data types", din, "-> f64, batch 50")
    c = datagen.cast_chain_batch(50, din, "f64", seed=5)
    check(c["chain"], c["frames"], c["items"], f"{din}->f64")


@pytest.mark.parametrize("layout", ["packed", "planar"])
@pytest.mark.parametrize("din", ["u8", "f64"])
def test_three_channels_swap_ragged_rows_every_config(din, layout):
    """Per-channel constants after a swap, rows of 37 pixels (not whole
    4-pixel units), an ROI inside a wider frame, all 20 launch configs."""
    say("f64 chain C=3", din, layout)
    g = datagen.rng(51)
    fr = datagen.frame(g, 45, 70, 3, dtype=din)
    items = [{"frame": 0, "x": 5, "y": 3, "w": 37, "h": 29}, {"frame": 0, "x": 0, "y": 0, "w": 70, "h": 45},
             {"frame": 0, "x": 69, "y": 44, "w": 1, "h": 1}]
    cfgs = [(c.block_threads, c.coarsen) for c in fk.fk_autotune_space()]
    check(chain3(din, layout), [fr], items, f"{din} C=3 {layout}", cfgs=cfgs)


def test_pitched_f64_frame_and_loop_op():
    say("f64 pitched frame, loop op")
    g = datagen.rng(52)
    img = datagen.frame(g, 20, 33, 1, dtype="f64")
    big = torch.zeros((20, 40), dtype=torch.float64, device="cuda:0")
    big[:, :33] = torch.from_numpy(img[:, :, 0]).to("cuda:0")
    dview = big[:, :33].unsqueeze(2)
    chain = {"read": {"kind": "plain", "dtype": "f64", "channels": 1, "out_w": 0, "out_h": 0},
             "ops": [{"kind": "mul", "k": [datagen.f32(1.001)]}, {"kind": "add", "k": [datagen.f32(-0.25)]},
                     {"kind": "loop", "k": [], "span": 2, "count": 100}],
             "write": {"dtype": "f64", "layout": "packed"}}
    items = [{"frame": 0, "x": 2, "y": 1, "w": 30, "h": 18}]
    refs = oracle.run_chain(chain, [img], items)
    for strict in (True, False):
        with Plan(chain, 1, strict=strict) as p:
            o = host(p.run([dview], items))[0]
        if strict:
            assert_bitexact(o, refs[0]["out"], "pitched loop strict")
        else:
            assert_close(o, refs[0], rel=REL64, what="pitched loop")


def test_table_path_many_frames_and_graph():
    """40 items over 8 frames (the device run table) and graph replays."""
    say("f64 table path and graph")
    g = datagen.rng(53)
    frames = [datagen.frame(g, 60, 50, 1, dtype="f32") for _ in range(8)]
    items = [{"frame": b % 8, "x": b % 7, "y": b % 5, "w": 40, "h": 50} for b in range(40)]
    chain = datagen.cast_chain_batch(1, "f32", "f64", seed=6)["chain"]
    refs = oracle.run_chain(chain, frames, items)
    dframes = to_dev(frames)
    for graph in (False, True):
        with Plan(chain, 40, strict=True, use_graph=graph) as p:
            for _ in range(2):
                got = host(p.run(dframes, items))
                for b, (o, r) in enumerate(zip(got, refs)):
                    assert_bitexact(o, r["out"], f"graph={graph} item {b}")


def test_refused_double_chains():
    c = datagen.normalize_chain(64, 128)
    c["write"]["dtype"] = "f64"  # crop+resize with an fp64 image write
    with pytest.raises(fk.FKError) as e:
        fk.fk_plan_create(fk.chain_desc(c), 1, fk.plan_opts())
    assert e.value.status == fk.FK_ERR_UNSUPPORTED
    c = datagen.cast_chain_batch(1, "f64", "f32", seed=0)["chain"]  # fp64 frame, fp32 write
    with pytest.raises(fk.FKError) as e:
        fk.fk_plan_create(fk.chain_desc(c), 1, fk.plan_opts())
    assert e.value.status == fk.FK_ERR_UNSUPPORTED
    cfg = datagen.cast_chain_batch(2, "f32", "f64", seed=0)
    dframes = to_dev(cfg["frames"])
    with Plan(cfg["chain"], 2) as p:
        arr = fk.make_items(cfg["chain"], dframes, cfg["items"], alloc_outs(cfg["chain"], cfg["items"]))
        with pytest.raises(fk.FKError) as e:
            fk.fk_model_features(p.h, arr, 2)
        assert e.value.status == fk.FK_ERR_UNSUPPORTED


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_double_chains_match_oracle(seed):
    """Random op lists (up to 48 ops of swap, cvt, mul, add, sub, div, scalar
    or per-channel constants) on plain reads of every input type with an fp64
    write, packed or planar, 1-4 frames of 16-200 px sides."""
    say("random fp64 chains, seed", seed)
    g = datagen.rng(900 + seed)
    for k in range(8):
        spec = datagen.random_chain_spec(g, max_ops=48, side=(16, 200), max_batch=4)
        ch = spec["chain"]
        ch["read"].update(kind="plain", dtype=["u8", "f16", "f32", "f64"][k % 4], out_w=0, out_h=0)
        ch["write"]["dtype"] = "f64"
        fh, fw = spec["frame_hw"]
        frames = [datagen.frame(g, fh, fw, ch["read"]["channels"], dtype=ch["read"]["dtype"])
                  for _ in range(spec["batch"])]
        items = []
        for b in range(spec["batch"]):
            # odd items read a random sub-rectangle of their frame
            w = int(g.integers(1, fw + 1)) if b % 2 else fw
            h = int(g.integers(1, fh + 1)) if b % 2 else fh
            items.append({"frame": b, "x": int(g.integers(0, fw - w + 1)),
                          "y": int(g.integers(0, fh - h + 1)), "w": w, "h": h})
        refs = oracle.run_chain(ch, frames, items)
        dframes = to_dev(frames)
        for strict in (True, False):
            with Plan(ch, len(items), strict=strict) as p:
                outs = host(p.run(dframes, items))
            for b, (o, r) in enumerate(zip(outs, refs)):
                what = (f"chain {k} item {b} ({ch['read']['dtype']}x{ch['read']['channels']} "
                        f"{len(ch['ops'])} ops -> f64 {ch['write']['layout']})")
                if strict:
                    assert_bitexact(o, r["out"], what)
                else:
                    assert_close(o, r, rel=REL64, what=what)
