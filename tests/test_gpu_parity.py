"""Parity of the fused HIP path (through the C ABI) with the CPU oracle.

Strict plans (no contraction) must be bit-exact with the oracle; default
plans (Mul+Add/Sub contracted into FMA) must be within 1e-5 relative,
|g - r| <= 1e-5 * max(|r|, s), s = 1 for the normalise chain and the
oracle's largest intermediate magnitude otherwise.
"""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_2508_07071_amd as fk
from fkhelpers import Plan, alloc_outs, assert_bitexact, assert_close, host, to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def check_both_modes(chain, frames, items, refs, s_floor=None, what="", **plan_kw):
    dframes = to_dev(frames)
    for strict in (True, False):
        with Plan(chain, len(items), strict=strict, **plan_kw) as p:
            outs = host(p.run(dframes, items))
        for b, (g, r) in enumerate(zip(outs, refs)):
            if strict:
                assert_bitexact(g, r["out"], f"{what} strict item {b}")
            else:
                assert_close(g, r, s_floor=s_floor, what=f"{what} item {b}")


# ------------------------------------------------------------- config 0 --

def test_config0_hot_chain_full_size():
    say("config0 1920x1080 crop 512^2 -> 224^2")
    cfg = datagen.config0(seed=0)
    refs = oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"])
    check_both_modes(cfg["chain"], cfg["frames"], cfg["items"], refs, s_floor=1.0, what="config0")


@pytest.mark.parametrize("strict", [True, False])
def test_static_and_runtime_tiers_agree_bitwise(strict):
    """The compile-time normalise kernel and the run-time op list compute
    the same operations: bit-identical in the strict mode, and in the
    contracted mode too (both fuse Mul+Sub into one FMA, then divide)."""
    say("config0 static vs runtime tier, strict", strict)
    cfg = datagen.config0(seed=1, frame_hw=(300, 500), crop=(7, 9, 333, 201), out=(100, 60))
    dframes = to_dev(cfg["frames"])
    res = {}
    for tier in (fk.FK_TIER_AUTO, fk.FK_TIER_RUNTIME):
        with Plan(cfg["chain"], 1, strict=strict, tier=tier) as p:
            assert fk.fk_plan_get_tier(p.h) == (1 if tier == fk.FK_TIER_AUTO else 0)
            res[tier] = host(p.run(dframes, cfg["items"]))[0]
    assert_bitexact(res[fk.FK_TIER_AUTO], res[fk.FK_TIER_RUNTIME], "tiers")


# ------------------------------------------------------------- config 1 --

@pytest.mark.parametrize("n_ops", [1, 4, 16, 64, 256])
def test_config1_muladd_depth_small_frame(n_ops):
    say("config1 small frame, N =", n_ops)
    cfg = datagen.config1(n_ops, seed=3, frame_hw=(72, 136))
    refs = oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"])
    check_both_modes(cfg["chain"], cfg["frames"], cfg["items"], refs, what=f"config1 N={n_ops}")
    check_both_modes(cfg["chain"], cfg["frames"], cfg["items"], refs, what=f"config1 N={n_ops} rt",
                     tier=fk.FK_TIER_RUNTIME)


@pytest.mark.parametrize("n_ops", [16, 256])
def test_config1_full_4k_frame_sampled_rows(n_ops):
    """Full 3840x2160 frame in the launch shape the benchmark uses; the
    oracle checks sampled row bands (first, middle, last)."""
    say("config1 4K frame, N =", n_ops)
    cfg = datagen.config1(n_ops, seed=0)
    fr = cfg["frames"][0]
    dframes = to_dev(cfg["frames"])
    for strict in (True, False):
        with Plan(cfg["chain"], 1, strict=strict) as p:
            out = host(p.run(dframes, cfg["items"]))[0]
        for y0 in (0, 1071, 2144):
            band = np.ascontiguousarray(fr[y0:y0 + 16])
            ref = oracle.run_chain(cfg["chain"], [band], [datagen.whole_frame_item(band)])[0]
            g = out[y0:y0 + 16]
            if strict:
                assert_bitexact(g, ref["out"], f"rows {y0}")
            else:
                assert_close(g, ref, what=f"rows {y0}")


# ------------------------------------------------------------- config 2 --

@pytest.mark.parametrize("batch", [1, 8, 50])
def test_config2_uneven_crops_batch(batch):
    say("config2 4K frame, B =", batch)
    cfg = datagen.config2(batch, seed=0)
    refs = oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"])
    check_both_modes(cfg["chain"], cfg["frames"], cfg["items"], refs, s_floor=1.0, what=f"config2 B={batch}")


@pytest.mark.parametrize("strict", [True, False])
def test_config2_batch256_one_tensor_all_items(strict):
    """B = 256 into one contiguous [B][3][128][64] tensor, in the launch
    form the benchmark times (one compact kernel-argument launch, pixel-
    strided lanes); every item checked against the oracle (bit-exact in the
    strict mode, within 1e-5 relative with s = 1 in the contracted mode)."""
    say("config2 B=256 contiguous output, strict", strict)
    cfg = datagen.config2(256, seed=0)
    dframes = to_dev(cfg["frames"])
    out = torch.full((256, 3, 128, 64), float("nan"), dtype=torch.float32, device="cuda:0")
    with Plan(cfg["chain"], 256, strict=strict) as p:
        p.run(dframes, cfg["items"], outs=[out[b] for b in range(256)])
        g = host([out])[0]
    assert not np.isnan(g).any()
    refs = oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"], shadow=False)
    for b, r in enumerate(refs):
        if strict:
            assert_bitexact(g[b], r["out"], f"item {b}")
        else:
            assert_close(g[b], r, s_floor=1.0, what=f"item {b}")


def test_batched_equals_single_item_runs():
    say("HF batch == single runs")
    cfg = datagen.config2(12, seed=4)
    dframes = to_dev(cfg["frames"])
    with Plan(cfg["chain"], 12) as p:
        batched = host(p.run(dframes, cfg["items"]))
        single = [host(p.run(dframes, [it]))[0] for it in cfg["items"]]
    for b in range(12):
        assert_bitexact(batched[b], single[b], f"item {b}")


def test_every_launch_config_gives_the_same_bits():
    say("all 20 launch configs")
    cfg = datagen.config2(9, seed=5)
    dframes = to_dev(cfg["frames"])
    base = None
    with Plan(cfg["chain"], 9) as p:
        for c in fk.fk_autotune_space():
            p.set_config(c.block_threads, c.coarsen)
            outs = host(p.run(dframes, cfg["items"]))
            if base is None:
                base = outs
            else:
                for b in range(9):
                    assert_bitexact(outs[b], base[b], f"config {c} item {b}")


def test_graph_replays_match_eager_runs():
    say("hipGraph replays")
    g = datagen.rng(21)
    fr = datagen.frame(g, 720, 1280, 3)
    dframes = to_dev([fr])
    chain = datagen.normalize_chain(64, 128)
    with Plan(chain, 32, use_graph=True) as pg, Plan(chain, 32) as pe:
        for rep, n in enumerate([32, 5, 17, 32, 1, 9]):
            items = datagen.random_crops(g, n, 1280, 720)
            a = host(pg.run(dframes, items))
            torch.cuda.synchronize()
            b = host(pe.run(dframes, items))
            for i in range(n):
                assert_bitexact(a[i], b[i], f"replay {rep} item {i}")


def test_device_table_runs_of_changing_size():
    """Batches above the kernel-argument forms go through the device table,
    of which a run uploads only its own n items and n + 1 tile offsets: runs
    of changing n on one plan (outputs in reverse address order, so no
    constant stride) match the oracle bit for bit, whatever the earlier runs
    left in the table ring."""
    say("device table, changing batch sizes")
    g = datagen.rng(23)
    fr = datagen.frame(g, 720, 1280, 3)
    dframes = to_dev([fr])
    chain = datagen.normalize_chain(64, 128)
    with Plan(chain, 200, strict=True) as p:
        for rep, n in enumerate([200, 45, 120, 33, 200, 57]):
            items = datagen.random_crops(g, n, 1280, 720)
            outs = list(reversed(alloc_outs(chain, items)))
            got = host(p.run(dframes, items, outs=outs))
            refs = oracle.run_chain(chain, [fr], items)
            for i in range(n):
                assert_bitexact(got[i], refs[i]["out"], f"run {rep} (n={n}) item {i}")


# --------------------------------------------- general chains and edges --

CASES = [
    # read kind, dtype, C, out dtype, layout, frame hw, roi (x, y, w, h), out (w, h)
    ("crop_resize", "u8", 3, "f32", "packed", (90, 130), (3, 5, 101, 77), (61, 33)),
    ("crop_resize", "u8", 4, "f16", "planar", (90, 130), (1, 2, 64, 50), (128, 96)),
    ("crop_resize", "f16", 1, "f32", "planar", (40, 300), (17, 3, 250, 30), (37, 11)),
    ("crop_resize", "f32", 3, "f16", "packed", (64, 64), (0, 0, 64, 64), (64, 64)),
    ("plain", "u8", 3, "f32", "planar", (33, 47), (5, 2, 39, 29), None),
    ("plain", "u8", 1, "f16", "packed", (31, 67), (0, 0, 67, 31), None),
    ("plain", "f16", 4, "f32", "packed", (20, 24), (3, 1, 17, 13), None),
    ("plain", "f32", 3, "f32", "packed", (25, 40), (0, 0, 40, 25), None),
    ("plain", "u8", 4, "f32", "packed", (16, 64), (0, 0, 64, 16), None),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}x{c[2]}-{c[3]}-{c[4]}" for c in CASES])
@pytest.mark.parametrize("seed", [0, 1])
def test_general_chains_ragged_and_unaligned(case, seed):
    rk, dt, C, odt, layout, hw, roi, out = case
    say("general", case, "seed", seed)
    g = datagen.rng(1000 + seed)
    fr = datagen.frame(g, hw[0], hw[1], C, dtype=dt)
    ops = []
    for kind in ["mul", "swap", "sub", "cvt", "mul", "add", "div", "swap", "add", "mul", "sub"]:
        if kind in ("swap", "cvt"):
            ops.append({"kind": kind, "k": []})
        else:
            n_k = C if g.uniform() < 0.5 else 1
            lo, hi = (0.5, 1.5) if kind in ("mul", "div") else (-1.0, 1.0)
            ops.append({"kind": kind, "k": [datagen.f32(g.uniform(lo, hi)) for _ in range(n_k)]})
    chain = {"read": {"kind": rk, "dtype": dt, "channels": C,
                      "out_w": out[0] if out else 0, "out_h": out[1] if out else 0},
             "ops": ops, "write": {"dtype": odt, "layout": layout}}
    x, y, w, h = roi
    it = {"frame": 0, "x": x, "y": y, "w": w, "h": h,
          "out_w": out[0] if out else w, "out_h": out[1] if out else h}
    refs = oracle.run_chain(chain, [fr], [it])
    for coarsen in (1, 4):
        dframes = to_dev([fr])
        for strict in (True, False):
            with Plan(chain, 1, strict=strict, config_source=fk.FK_CONFIG_MANUAL,
                      manual=(64, coarsen)) as p:
                o = host(p.run(dframes, [it]))[0]
            if strict:
                assert_bitexact(o, refs[0]["out"], f"k={coarsen}")
            else:
                assert_close(o, refs[0], what=f"k={coarsen}")


def test_frame_with_row_padding():
    say("frame with padded pitch")
    g = datagen.rng(7)
    big = datagen.frame(g, 50, 80, 3)
    view_np = big[:, :70]  # rows of 80 px, image of 70 px
    chain = datagen.normalize_chain(40, 24)
    it = {"frame": 0, "x": 2, "y": 3, "w": 60, "h": 40, "out_w": 40, "out_h": 24}
    ref = oracle.run_chain(chain, [np.ascontiguousarray(view_np)], [it])[0]
    dbig = to_dev([big])[0]
    dview = dbig[:, :70]
    with Plan(chain, 1, strict=True) as p:
        o = host(p.run([dview], [it]))[0]
    assert_bitexact(o, ref["out"], "padded pitch")


def test_frame_rows_of_16_mib_take_64_bit_offsets():
    """A pitch of 2^24 bytes puts the frame outside the 32-bit row-offset
    form (IF_SMALL_FRAME): the crop+resize reads through 64-bit offsets and
    still matches the oracle bit for bit."""
    say("frame with a 16 MiB pitch")
    g = datagen.rng(17)
    H, W = 5, 64
    img = datagen.frame(g, H, W, 3)
    dbig = torch.zeros((H, 1 << 24), dtype=torch.uint8, device="cuda:0")
    dbig[:, :W * 3] = torch.from_numpy(img.reshape(H, W * 3)).to("cuda:0")
    dview = dbig[:, :W * 3].unflatten(1, (W, 3))
    assert dview.stride(0) == 1 << 24
    chain = datagen.normalize_chain(24, 9)
    items = [{"frame": 0, "x": 3, "y": 1, "w": 50, "h": 4, "out_w": 24, "out_h": 9},
             {"frame": 0, "x": 0, "y": 0, "w": 64, "h": 5, "out_w": 7, "out_h": 3}]
    refs = oracle.run_chain(chain, [img], items)
    for strict in (True, False):
        with Plan(chain, 2, strict=strict) as p:
            outs = host(p.run([dview], items))
        for b in range(2):
            if strict:
                assert_bitexact(outs[b], refs[b]["out"], f"item {b}")
            else:
                assert_close(outs[b], refs[b], s_floor=1.0, what=f"item {b}")
    del dbig


def test_single_pixel_and_extreme_scales():
    say("1x1 ROI, 1x1 output, extreme scales")
    g = datagen.rng(8)
    fr = datagen.frame(g, 600, 800, 3)
    chain = datagen.normalize_chain(1, 1)
    items = [
        {"frame": 0, "x": 5, "y": 6, "w": 1, "h": 1, "out_w": 1, "out_h": 1},
        {"frame": 0, "x": 0, "y": 0, "w": 800, "h": 600, "out_w": 1, "out_h": 1},
        {"frame": 0, "x": 799, "y": 599, "w": 1, "h": 1, "out_w": 300, "out_h": 2},
        {"frame": 0, "x": 0, "y": 0, "w": 800, "h": 2, "out_w": 3, "out_h": 257},
    ]
    refs = oracle.run_chain(chain, [fr], items)
    dframes = to_dev([fr])
    with Plan(chain, 4, strict=True) as p:
        outs = host(p.run(dframes, items))
    for b in range(4):
        assert_bitexact(outs[b], refs[b]["out"], f"item {b}")


def test_multiple_frames_in_one_batch():
    say("items over several frames")
    g = datagen.rng(9)
    frames = [datagen.frame(g, 200 + 37 * i, 300 + 11 * i, 3) for i in range(3)]
    chain = datagen.normalize_chain(64, 128)
    items = []
    for i in range(9):
        its = datagen.random_crops(g, 1, frames[i % 3].shape[1], frames[i % 3].shape[0], 20, 190,
                                   frame_index=i % 3)
        items += its
    refs = oracle.run_chain(chain, frames, items)
    check_both_modes(chain, frames, items, refs, s_floor=1.0, what="multi-frame")


# --------------------------------------------------------------- unfused --

@pytest.mark.parametrize("which", ["config0", "config1", "general"])
def test_unfused_baseline_matches_oracle_bitwise(which):
    say("unfused", which)
    if which == "config0":
        cfg = datagen.config0(seed=2, frame_hw=(400, 600), crop=(13, 17, 300, 222), out=(64, 128))
    elif which == "config1":
        cfg = datagen.config1(16, seed=2, frame_hw=(50, 70))
    else:
        g = datagen.rng(3)
        fr = datagen.frame(g, 40, 60, 4, dtype="f16")
        chain = {"read": {"kind": "crop_resize", "dtype": "f16", "channels": 4, "out_w": 30, "out_h": 50},
                 "ops": [{"kind": "swap", "k": []}, {"kind": "mul", "k": [0.5, 0.25, 2.0, 1.5]},
                         {"kind": "sub", "k": [0.1]}, {"kind": "div", "k": [0.7, 0.9, 1.1, 1.3]}],
                 "write": {"dtype": "f16", "layout": "planar"}}
        cfg = {"frames": [fr], "chain": chain,
               "items": [{"frame": 0, "x": 3, "y": 4, "w": 51, "h": 33, "out_w": 30, "out_h": 50}]}
    refs = oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"])
    dframes = to_dev(cfg["frames"])
    with Plan(cfg["chain"], len(cfg["items"]), strict=True) as p:
        u = host(p.run_unfused(dframes, cfg["items"]))
        f = host(p.run(dframes, cfg["items"]))
    for b, r in enumerate(refs):
        assert_bitexact(u[b], r["out"], "unfused vs oracle")
        assert_bitexact(f[b], u[b], "fused vs unfused")


# --------------------------------------------------------------- errors --

def test_invalid_runs_return_status_and_launch_nothing():
    say("error paths")
    cfg = datagen.config0(seed=0, frame_hw=(100, 120), crop=(0, 0, 50, 50), out=(16, 16))
    dframes = to_dev(cfg["frames"])
    with Plan(cfg["chain"], 2) as p:
        outs = alloc_outs(cfg["chain"], cfg["items"])
        bad = dict(cfg["items"][0], x=100)
        arr = fk.make_items(cfg["chain"], dframes, [bad], outs)
        with pytest.raises(fk.FKError) as e:
            fk.fk_run(p.h, arr, 1, fk.stream_handle())
        assert e.value.status == fk.FK_ERR_INVALID_ARG
        arr = fk.make_items(cfg["chain"], dframes, cfg["items"] * 3, outs * 3)
        with pytest.raises(fk.FKError):
            fk.fk_run(p.h, arr, 3, fk.stream_handle())  # over max_batch
        with pytest.raises(fk.FKError):
            fk.fk_run(p.h, arr, 0, fk.stream_handle())
        torch.cuda.synchronize()
        assert torch.isnan(outs[0]).all()
        with pytest.raises(fk.FKError):
            fk.fk_plan_set_config(p.h, fk.fk_launch_config(100, 1))


# ------------------------------------------- random chains (cost-model set) --

@pytest.mark.parametrize("seed", range(4))
def test_random_chains_match_oracle(seed):
    """Chains drawn like the cost model's dataset (any read kind, dtype,
    channel count, op mix, layout and output dtype), at reduced sizes."""
    say("random chains, seed", seed)
    g = datagen.rng(500 + seed)
    for k in range(10):
        spec = datagen.random_chain_spec(g, max_ops=64, side=(16, 300), max_batch=4)
        ch = spec["chain"]
        fh, fw = spec["frame_hw"]
        frames = [datagen.frame(g, fh, fw, ch["read"]["channels"], dtype=ch["read"]["dtype"])
                  for _ in range(spec["batch"])]
        items = spec["items"]
        refs = oracle.run_chain(ch, frames, items)
        dframes = to_dev(frames)
        for strict in (True, False):
            with Plan(ch, len(items), strict=strict) as p:
                outs = host(p.run(dframes, items))
            for b, (o, r) in enumerate(zip(outs, refs)):
                what = f"chain {k} item {b} ({ch['read']['kind']} {ch['read']['dtype']}x{ch['read']['channels']} " \
                       f"{len(ch['ops'])} ops -> {ch['write']['dtype']} {ch['write']['layout']})"
                if strict:
                    assert_bitexact(o, r["out"], what)
                else:
                    assert_close(o, r, what=what)


# ------------------------------------------ compact kernel-argument batches --

def test_compact_argument_batches_match_table_path_and_oracle():
    """Batches of one frame, one output size and a constant output stride
    travel in the kernel arguments (up to 312 items); the table path (graph
    replay) and the oracle agree with them bit for bit."""
    say("compact batches")
    cfg = datagen.config2(50, seed=8)
    dframes = to_dev(cfg["frames"])
    out_c = torch.full((50, 3, 128, 64), float("nan"), dtype=torch.float32, device="cuda:0")
    out_t = torch.full((50, 3, 128, 64), float("nan"), dtype=torch.float32, device="cuda:0")
    with Plan(cfg["chain"], 50, strict=True) as pc, Plan(cfg["chain"], 50, strict=True, use_graph=True) as pt:
        pc.run(dframes, cfg["items"], outs=[out_c[b] for b in range(50)])
        pt.run(dframes, cfg["items"], outs=[out_t[b] for b in range(50)])
        a, b = host([out_c, out_t])
    assert_bitexact(a, b, "compact vs table")
    refs = oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"][::7])
    for k, r in zip(range(0, 50, 7), refs):
        assert_bitexact(a[k], r["out"], f"item {k}")
    # plain reads: equal-size ROIs at odd offsets (unaligned source rows)
    g = datagen.rng(9)
    fr = datagen.frame(g, 200, 301, 3)
    chain = {"read": {"kind": "plain", "dtype": "u8", "channels": 3, "out_w": 0, "out_h": 0},
             "ops": [{"kind": "swap", "k": []}, {"kind": "mul", "k": [0.5]}, {"kind": "add", "k": [1.0, 2.0, 3.0]}],
             "write": {"dtype": "f32", "layout": "packed"}}
    items = [{"frame": 0, "x": int(g.integers(0, 301 - 37)), "y": int(g.integers(0, 200 - 21)), "w": 37, "h": 21,
              "out_w": 37, "out_h": 21} for _ in range(40)]
    out = torch.full((40, 21, 37, 3), float("nan"), dtype=torch.float32, device="cuda:0")
    with Plan(chain, 40, strict=True) as p:
        p.run(to_dev([fr]), items, outs=[out[b] for b in range(40)])
        o = host([out])[0]
    refs = oracle.run_chain(chain, [fr], items)
    for k in range(40):
        assert_bitexact(o[k], refs[k]["out"], f"plain item {k}")


# ------------------------------------------------------- timed launches --

@pytest.mark.parametrize("graph", [False, True])
def test_timed_run_matches_run_and_records_its_kernel(graph):
    """fk_run_timed gives fk_run's bits and a positive kernel duration from
    the events its launch records (a graph plan records them around the
    graph launch)."""
    say("timed run, graph =", graph)
    cfg = datagen.config1(256, seed=2, frame_hw=(270, 480))
    dframes = to_dev(cfg["frames"])
    with Plan(cfg["chain"], 1, use_graph=graph) as p:
        ref = host(p.run(dframes, cfg["items"]))[0]
        outs = alloc_outs(cfg["chain"], cfg["items"])
        arr = fk.make_items(cfg["chain"], dframes, cfg["items"], outs)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        e1.record()
        torch.cuda.synchronize()
        fk.fk_run_timed(p.h, arr, 1, fk.stream_handle(), e0.cuda_event, e1.cuda_event)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        got = host(outs)[0]
    assert_bitexact(got, ref, "timed vs plain run")
    assert 0.0 < ms < 50.0
