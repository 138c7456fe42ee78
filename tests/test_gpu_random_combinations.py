"""Random combinations against the oracle: every read kind (plain,
bilinear and nearest crop+resize, NV12 1:1 and NV12 resize), input dtype,
channel count, op mix, output dtype and layout, drawn together with a
launch configuration from the 20, the tier (automatic or run-time op
list), eager or graph launches, the gather option, and where the frame
sits in memory (dense, rows padded by 1, 4 or 64 elements, or u8 frames
1-3 bytes past a dword boundary).  Strict plans give the oracle's bits,
fused and unfused; contracted plans stay within the tolerance.  The same
draws cover stats writes (order-free min/max exact, sums within the fp64
reordering bound) and fp64 chains.  FK_RANDOM_BLOCKS=n runs n blocks of
8 cases per test instead of the default."""
import os

import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_2508_07071_amd as fk
from fkhelpers import Plan, assert_bitexact, assert_close, host

pytestmark = pytest.mark.gpu

KINDS = ["plain", "crop_resize", "crop_nearest", "nv12", "nv12_resize"]


def blocks(default):
    return range(int(os.environ.get("FK_RANDOM_BLOCKS", default)))


def say(*a):
    print("[case]", *a, flush=True)


def place(fr, g):
    """The frame on the device: dense, as a view with padded rows, or (u8)
    at a base 1-3 bytes past a dword boundary."""
    mode = int(g.integers(0, 3))
    t = torch.from_numpy(fr)
    if mode == 1:
        pad = int(g.choice([1, 4, 64]))
        shp = list(fr.shape)
        shp[1] += pad
        big = torch.zeros(shp, dtype=t.dtype)
        big[:, :fr.shape[1]] = t
        return big.to("cuda:0")[:, :fr.shape[1]], f"rows+{pad}"
    if mode == 2 and fr.dtype == np.uint8:
        off = int(g.integers(1, 4))
        buf = torch.zeros(fr.size + 16, dtype=torch.uint8, device="cuda:0")
        buf[off:off + fr.size] = t.reshape(-1).to("cuda:0")
        return buf[off:off + fr.size].view(fr.shape), f"base+{off}"
    return t.to("cuda:0"), "dense"


def draw(g):
    kind = KINDS[int(g.integers(0, len(KINDS)))]
    spec = datagen.random_chain_spec(g, max_ops=40, side=(16, 400), max_batch=6)
    ch = spec["chain"]
    fh, fw = spec["frame_hw"]
    if kind.startswith("nv12"):
        fh, fw = max(2, fh & ~1), max(2, fw & ~1)
        ch["read"].update(kind=kind, dtype="u8", channels=3)
        for op in ch["ops"]:
            if len(op["k"]) > 1:
                op["k"] = (op["k"] * 3)[:3]
        nf = 1 + int(g.integers(0, 2))
        frames = [datagen.nv12_frame(g, fh, fw) for _ in range(nf)]
        items = []
        for b in range(1 + int(g.integers(0, 6))):
            w, h = int(g.integers(1, fw + 1)), int(g.integers(1, fh + 1))
            x, y = int(g.integers(0, fw - w + 1)), int(g.integers(0, fh - h + 1))
            ow, oh = (w, h) if kind == "nv12" else (int(g.integers(1, 200)), int(g.integers(1, 200)))
            items.append({"frame": b % nf, "x": x, "y": y, "w": w, "h": h, "out_w": ow, "out_h": oh})
    else:
        if kind == "crop_nearest":
            ch["read"]["kind"] = "crop_nearest"
        nf = max(it["frame"] for it in spec["items"]) + 1
        frames = [datagen.frame(g, fh, fw, ch["read"]["channels"], dtype=ch["read"]["dtype"])
                  for _ in range(nf)]
        items = spec["items"]
    return ch, frames, items, (fh, fw)


@pytest.mark.parametrize("block", blocks(16))
def test_random_combinations_match_oracle(block):
    space = fk.fk_autotune_space()
    for i in range(block * 8, block * 8 + 8):
        g = datagen.rng(90000 + i)
        ch, frames, items, (fh, fw) = draw(g)
        refs = oracle.run_chain(ch, frames, items)
        placed = [place(f, g) for f in frames]
        dframes = [p[0] for p in placed]
        cfg = space[int(g.integers(0, len(space)))]
        tier = [fk.FK_TIER_AUTO, fk.FK_TIER_RUNTIME][int(g.integers(0, 2))]
        graph = bool(g.integers(0, 4) == 0)
        gather = [fk.FK_GATHER_DIRECT, fk.FK_GATHER_LDS][int(g.integers(0, 2))]
        what = (f"case {i}: {ch['read']['kind']} {ch['read']['dtype']}x{ch['read']['channels']} "
                f"{len(ch['ops'])} ops -> {ch['write']['dtype']} {ch['write']['layout']}, B={len(items)}, "
                f"{fh}x{fw} {[p[1] for p in placed]}, {cfg.block_threads}x{cfg.coarsen}, tier {tier}, "
                f"graph {graph}, gather {gather}")
        say(what)
        for strict in (True, False):
            with Plan(ch, len(items), strict=strict, tier=tier, use_graph=graph, gather=gather) as p:
                p.set_config(cfg.block_threads, cfg.coarsen)
                outs = host(p.run(dframes, items))
                uouts = host(p.run_unfused(dframes, items)) if strict else None
            for b, (o, r) in enumerate(zip(outs, refs)):
                if strict:
                    assert_bitexact(o, r["out"], f"{what}: strict item {b}")
                    assert_bitexact(uouts[b], r["out"], f"{what}: unfused item {b}")
                else:
                    assert_close(o, r, what=f"{what}: contracted item {b}")


@pytest.mark.parametrize("block", blocks(4))
def test_random_stats_combinations_match_oracle(block):
    from test_gpu_stats import check, image_of, stats_of
    space = fk.fk_autotune_space()
    for i in range(block * 8, block * 8 + 8):
        g = datagen.rng(77000 + i)
        ch, frames, items, (fh, fw) = draw(g)
        st = [r["out"] for r in oracle.run_chain(stats_of(ch), frames, items)]
        ims = oracle.run_chain(image_of(ch), frames, items)
        placed = [place(f, g) for f in frames]
        dframes = [p[0] for p in placed]
        cfg = space[int(g.integers(0, len(space)))]
        tier = [fk.FK_TIER_AUTO, fk.FK_TIER_RUNTIME][int(g.integers(0, 2))]
        graph = bool(g.integers(0, 4) == 0)
        what = (f"stats case {i}: {ch['read']['kind']} {ch['read']['dtype']}x{ch['read']['channels']} "
                f"{len(ch['ops'])} ops, B={len(items)}, {fh}x{fw} {[p[1] for p in placed]}, "
                f"{cfg.block_threads}x{cfg.coarsen}, tier {tier}, graph {graph}")
        say(what)
        for strict in (True, False):
            with Plan(stats_of(ch), len(items), strict=strict, tier=tier, use_graph=graph) as p:
                p.set_config(cfg.block_threads, cfg.coarsen)
                first = host(p.run(dframes, items))
                again = host(p.run(dframes, items))  # partials and counters start clean
            for b in range(len(items)):
                check(first[b], st[b], ims[b], strict, f"{what} item {b} strict={strict}")
                check(again[b], st[b], ims[b], strict, f"{what} rerun item {b} strict={strict}")


@pytest.mark.parametrize("block", blocks(4))
def test_random_f64_combinations_match_oracle(block):
    from test_gpu_f64 import REL64
    space = fk.fk_autotune_space()
    for i in range(block * 8, block * 8 + 8):
        g = datagen.rng(66000 + i)
        spec = datagen.random_chain_spec(g, max_ops=48, side=(16, 300), max_batch=5)
        ch = spec["chain"]
        ch["read"].update(kind="plain", dtype=["u8", "f16", "f32", "f64"][int(g.integers(0, 4))], out_w=0, out_h=0)
        ch["write"]["dtype"] = "f64"
        fh, fw = spec["frame_hw"]
        nf = 1 + int(g.integers(0, 3))
        frames = [datagen.frame(g, fh, fw, ch["read"]["channels"], dtype=ch["read"]["dtype"]) for _ in range(nf)]
        items = []
        for b in range(1 + int(g.integers(0, 5))):
            w, h = int(g.integers(1, fw + 1)), int(g.integers(1, fh + 1))
            items.append({"frame": b % nf, "x": int(g.integers(0, fw - w + 1)),
                          "y": int(g.integers(0, fh - h + 1)), "w": w, "h": h})
        refs = oracle.run_chain(ch, frames, items)
        placed = [place(f, g) for f in frames]
        dframes = [p[0] for p in placed]
        cfg = space[int(g.integers(0, len(space)))]
        graph = bool(g.integers(0, 4) == 0)
        what = (f"fp64 case {i}: {ch['read']['dtype']}x{ch['read']['channels']} {len(ch['ops'])} ops -> f64 "
                f"{ch['write']['layout']}, B={len(items)}, {fh}x{fw} {[p[1] for p in placed]}, "
                f"{cfg.block_threads}x{cfg.coarsen}, graph {graph}")
        say(what)
        for strict in (True, False):
            with Plan(ch, len(items), strict=strict, use_graph=graph) as p:
                p.set_config(cfg.block_threads, cfg.coarsen)
                outs = host(p.run(dframes, items))
                uouts = host(p.run_unfused(dframes, items)) if strict else None
            for b, (o, r) in enumerate(zip(outs, refs)):
                if strict:
                    assert_bitexact(o, r["out"], f"{what}: item {b}")
                    assert_bitexact(uouts[b], r["out"], f"{what}: unfused item {b}")
                else:
                    assert_close(o, r, rel=REL64, what=f"{what}: item {b}")
