"""The LDS-staged gather of the normalise chain (plan option
FK_GATHER_LDS): a block copies the tap rows of a band of output rows into
LDS with 16-byte loads over the ROI's width and reads the taps from there.
It must give the oracle's bits in the strict mode and the direct gather's
bits in the contracted mode, for every launch configuration, for items that
take the staged path and for those that fall back to direct gathers
(frame base or pitch not a multiple of 16, a last 16-byte chunk past the
end of the frame, rows too wide for the block's LDS)."""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_2508_07071_amd as fk
from fkhelpers import Plan, alloc_outs, assert_bitexact, host, to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def run(chain, dframes, items, strict, gather, cfg=None, outs=None):
    with Plan(chain, len(items), strict=strict, gather=gather) as p:
        if cfg:
            p.set_config(*cfg)
        return host(p.run(dframes, items, outs=outs))


@pytest.mark.parametrize("cfg", [(64, 1), (256, 1), (256, 4), (1024, 8), (128, 2)])
def test_config2_batch50_matches_oracle_and_direct(cfg):
    say("LDS gather, config2 B=50, config", cfg)
    c = datagen.config2(50, seed=11)
    dframes = to_dev(c["frames"])
    refs = oracle.run_chain(c["chain"], c["frames"], c["items"])
    got = run(c["chain"], dframes, c["items"], True, fk.FK_GATHER_LDS, cfg)
    for b, (g, r) in enumerate(zip(got, refs)):
        assert_bitexact(g, r["out"], f"strict item {b}")
    lds = run(c["chain"], dframes, c["items"], False, fk.FK_GATHER_LDS, cfg)
    direct = run(c["chain"], dframes, c["items"], False, fk.FK_GATHER_DIRECT, cfg)
    for b, (x, y) in enumerate(zip(lds, direct)):
        assert_bitexact(x, y, f"contracted item {b}")


def test_config2_batch256_one_tensor():
    """The benchmark's form: 256 crops into one [B][3][128][64] tensor (one
    compact kernel-argument launch)."""
    say("LDS gather, config2 B=256 one tensor")
    c = datagen.config2(256, seed=0)
    dframes = to_dev(c["frames"])
    out = torch.full((256, 3, 128, 64), float("nan"), dtype=torch.float32, device="cuda:0")
    run(c["chain"], dframes, c["items"], True, fk.FK_GATHER_LDS, outs=[out[b] for b in range(256)])
    g = host([out])[0]
    assert not np.isnan(g).any()
    sample = list(range(0, 256, 7))
    refs = oracle.run_chain(c["chain"], c["frames"], [c["items"][b] for b in sample])
    for b, r in zip(sample, refs):
        assert_bitexact(g[b], r["out"], f"item {b}")


def edge_items():
    # (x, y, w, h, out_w, out_h) in a 40 x 250 frame (750-byte rows)
    return [
        (0, 0, 250, 40, 64, 128),    # whole frame: ends on the last row and the last byte
        (3, 0, 100, 39, 64, 128),    # stops above the last row
        (240, 30, 10, 10, 64, 128),  # upscale at the right edge, touching the last row
        (5, 5, 1, 1, 3, 2),          # one pixel
        (7, 2, 20, 10, 1, 1),        # one output pixel
        (1, 1, 247, 3, 200, 7),      # wide, three rows
    ]


@pytest.mark.parametrize("layout", ["packed", "pitch768", "offset3"])
def test_staged_and_fallback_items_match_oracle(layout):
    """A 250-pixel-wide frame: packed rows (750 bytes: not a multiple of 16,
    every item reads directly), rows padded to 768 bytes (staged, except
    items whose last chunk would pass the end of the last row), and a frame
    whose base is 3 bytes past a 16-byte boundary (direct)."""
    say("LDS gather, edge items, frame", layout)
    g = datagen.rng(12)
    H, W = 40, 250
    img = datagen.frame(g, H, W, 3)
    if layout == "packed":
        dfr = to_dev([img])[0]
    elif layout == "pitch768":
        big = torch.zeros((H, 768), dtype=torch.uint8, device="cuda:0")
        big[:, :W * 3] = torch.from_numpy(img.reshape(H, W * 3)).to("cuda:0")
        dfr = big[:, :W * 3].unflatten(1, (W, 3))
        assert dfr.stride(0) == 768
    else:
        buf = torch.zeros(H * W * 3 + 64, dtype=torch.uint8, device="cuda:0")
        buf[3:3 + H * W * 3] = torch.from_numpy(img.reshape(-1)).to("cuda:0")
        dfr = buf[3:3 + H * W * 3].view(H, W, 3)
        assert dfr.data_ptr() % 16 == 3
    for ow, oh in [(64, 128), (3, 2), (1, 1), (200, 7)]:
        chain = datagen.normalize_chain(ow, oh)
        items = [{"frame": 0, "x": x, "y": y, "w": w, "h": h, "out_w": a, "out_h": b}
                 for x, y, w, h, a, b in edge_items() if (a, b) == (ow, oh)]
        refs = oracle.run_chain(chain, [img], items)
        for cfg in [(64, 1), (256, 2), (1024, 1)]:
            got = run(chain, [dfr], items, True, fk.FK_GATHER_LDS, cfg)
            for b, (gg, r) in enumerate(zip(got, refs)):
                assert_bitexact(gg, r["out"], f"{layout} {cfg} item {items[b]}")


def test_rows_wider_than_the_lds_fall_back():
    """A 4000-pixel-wide ROI (12,000-byte rows) fits one band in the LDS of
    a 256-thread block (32 KiB) but not in that of a 64-thread block (8 KiB),
    which reads directly; both give the oracle's bits."""
    say("LDS gather, 4000-pixel rows")
    g = datagen.rng(13)
    fr = datagen.frame(g, 64, 4096, 3)
    chain = datagen.normalize_chain(512, 16)
    items = [{"frame": 0, "x": 16, "y": 3, "w": 4000, "h": 50, "out_w": 512, "out_h": 16},
             {"frame": 0, "x": 1, "y": 0, "w": 4095, "h": 64, "out_w": 512, "out_h": 16}]
    refs = oracle.run_chain(chain, [fr], items)
    dframes = to_dev([fr])
    for cfg in [(64, 1), (256, 1), (512, 4)]:
        got = run(chain, dframes, items, True, fk.FK_GATHER_LDS, cfg)
        for b, (gg, r) in enumerate(zip(got, refs)):
            assert_bitexact(gg, r["out"], f"{cfg} item {b}")


def test_table_path_and_graph_replay():
    """Items over several frames (the device run table) and graph replays
    take the staged kernel too."""
    say("LDS gather, run table and graph")
    g = datagen.rng(14)
    # 512-pixel rows: 1536-byte pitch, a multiple of 16
    frames = [datagen.frame(g, 300, 512, 3) for _ in range(3)]
    items = []
    for f in range(3):
        items += datagen.random_crops(g, 20, 512, 300, frame_index=f)
    chain = datagen.normalize_chain(64, 128)
    refs = oracle.run_chain(chain, frames, items)
    dframes = to_dev(frames)
    for graph in (False, True):
        with Plan(chain, len(items), strict=True, gather=fk.FK_GATHER_LDS, use_graph=graph) as p:
            for _ in range(3):
                outs = alloc_outs(chain, items)
                got = host(p.run(dframes, items, outs=outs))
                for b, (gg, r) in enumerate(zip(got, refs)):
                    assert_bitexact(gg, r["out"], f"graph={graph} item {b}")


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_random_rois_and_output_sizes(seed):
    """Random geometry through the staged gather: frames 16-1024 px wide in
    multiples of 16 px (16-byte-aligned rows, so items may stage), ROIs of
    1 px up to the whole frame, outputs of 1-300 px per side (down- and
    upsampling, per item), in one run over several frames (the run table);
    strict bits against the oracle, contracted bits against the direct
    gather."""
    say("LDS gather, random ROIs, seed", seed)
    g = datagen.rng(1400 + seed)
    frames = []
    for _ in range(3):
        w = 16 * int(g.integers(1, 65))
        h = int(g.integers(2, 400))
        frames.append(datagen.frame(g, h, w, 3))
    items = []
    for _ in range(24):
        f = int(g.integers(0, 3))
        fh, fw = frames[f].shape[:2]
        w = datagen.log_uniform_int(g, 1, fw)
        h = datagen.log_uniform_int(g, 1, fh)
        items.append({"frame": f, "x": int(g.integers(0, fw - w + 1)), "y": int(g.integers(0, fh - h + 1)),
                      "w": w, "h": h, "out_w": datagen.log_uniform_int(g, 1, 300),
                      "out_h": datagen.log_uniform_int(g, 1, 300)})
    chain = datagen.normalize_chain(0, 0)
    refs = oracle.run_chain(chain, frames, items)
    dframes = to_dev(frames)
    cfg = [(64, 1), (256, 2), (1024, 1), (128, 4)][seed]
    got = run(chain, dframes, items, True, fk.FK_GATHER_LDS, cfg)
    for b, (gg, r) in enumerate(zip(got, refs)):
        assert_bitexact(gg, r["out"], f"{cfg} item {items[b]}")
    lds = run(chain, dframes, items, False, fk.FK_GATHER_LDS, cfg)
    direct = run(chain, dframes, items, False, fk.FK_GATHER_DIRECT, cfg)
    for b, (x, y) in enumerate(zip(lds, direct)):
        assert_bitexact(x, y, f"contracted {cfg} item {items[b]}")


def test_unknown_gather_mode_is_refused():
    chain = datagen.normalize_chain(64, 128)
    with pytest.raises(fk.FKError) as e:
        fk.fk_plan_create(fk.chain_desc(chain), 1, fk.plan_opts(gather=2))
    assert e.value.status == fk.FK_ERR_INVALID_ARG
