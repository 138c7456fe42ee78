"""The stats write (per channel min, max, sum, mean of the chain's fp32
values from one read; the reduction pattern of Section IV-C) on the GPU,
through the C ABI, against the oracle.

Min and max are order-free, so strict plans match the oracle exactly.  The
sum is an fp64 accumulation whose order depends on the launch; two orders
of the same n values differ by at most 2 (n - 1) 2^-53 sum|x|, the bound
used here (mean: the same over n, plus one rounding).  Default plans
contract Mul+Add into FMA, so their values, and hence the statistics,
move within the chain's elementwise tolerance on top."""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_2508_07071_amd as fk
from fkhelpers import Plan, host, to_dev

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def say(*a):
    print("[case]", *a, flush=True)


def stats_of(chain):
    return dict(chain, write={"dtype": "f64", "layout": "stats"})


def image_of(chain):
    return dict(chain, write={"dtype": "f32", "layout": "packed"})


def oracle_refs(chain, frames, items):
    st = [r["out"] for r in oracle.run_chain(stats_of(chain), frames, items)]
    ims = oracle.run_chain(image_of(chain), frames, items)
    return st, ims


def check(g, st, im, strict, what):
    C = st.shape[0]
    vals = im["out"].reshape(-1, C).astype(np.float64)
    n = vals.shape[0]
    for c in range(C):
        absum = np.abs(vals[:, c]).sum()
        if strict:
            assert g[c, 0] == st[c, 0] and g[c, 1] == st[c, 1], (what, c, g[c], st[c])
            slack = 0.0
        else:
            tol = 1e-5 * np.maximum(np.abs(vals[:, c]), im["smax"].reshape(-1, C)[:, c])
            assert abs(g[c, 0] - st[c, 0]) <= tol.max() and abs(g[c, 1] - st[c, 1]) <= tol.max(), (what, c)
            slack = tol.sum()
        bound = 2 * (n - 1) * U * absum + slack
        assert abs(g[c, 2] - st[c, 2]) <= bound, (what, c, g[c, 2], st[c, 2], bound)
        assert abs(g[c, 3] - st[c, 3]) <= bound / n + U * abs(st[c, 3]), (what, c)


def run_stats(chain, dframes, items, **kw):
    with Plan(stats_of(chain), len(items), **kw) as p:
        return host(p.run(dframes, items))


def test_normalise_chain_stats_config0():
    say("stats: config0 crop 512^2 -> 224^2, normalise")
    cfg = datagen.config0(seed=0)
    st, ims = oracle_refs(cfg["chain"], cfg["frames"], cfg["items"])
    dframes = to_dev(cfg["frames"])
    for strict in (True, False):
        g = run_stats(cfg["chain"], dframes, cfg["items"], strict=strict)[0]
        check(g, st[0], ims[0], strict, f"config0 strict={strict}")


@pytest.mark.parametrize("seed", range(3))
def test_random_chains_stats_match_oracle(seed):
    say("stats: random chains, seed", seed)
    g = datagen.rng(700 + seed)
    for k in range(8):
        spec = datagen.random_chain_spec(g, max_ops=32, side=(16, 300), max_batch=4)
        ch = spec["chain"]
        fh, fw = spec["frame_hw"]
        frames = [datagen.frame(g, fh, fw, ch["read"]["channels"], dtype=ch["read"]["dtype"])
                  for _ in range(spec["batch"])]
        items = spec["items"]
        st, ims = oracle_refs(ch, frames, items)
        dframes = to_dev(frames)
        for strict in (True, False):
            outs = run_stats(ch, dframes, items, strict=strict)
            for b, o in enumerate(outs):
                check(o, st[b], ims[b], strict, f"chain {k} item {b} strict={strict}")


def test_full_4k_frame_integer_sums_are_exact():
    """A 3840x2160x3 u8 frame, cvt only: every partial sum is an integer
    below 2^53, so the sum is exact in any order; min/max/mean against
    numpy over the frame (512 blocks per item, every launch config)."""
    say("stats: 4K u8 frame")
    g = datagen.rng(3)
    fr = datagen.frame(g, 2160, 3840, 3)
    ch = {"read": {"kind": "plain", "dtype": "u8", "channels": 3, "out_w": 0, "out_h": 0},
          "ops": [{"kind": "cvt", "k": []}], "write": {"dtype": "f32", "layout": "packed"}}
    items = [datagen.whole_frame_item(fr)]
    want = np.stack([fr.reshape(-1, 3).min(0), fr.reshape(-1, 3).max(0),
                     fr.reshape(-1, 3).astype(np.float64).sum(0)], 1).astype(np.float64)
    dframes = to_dev([fr])
    with Plan(stats_of(ch), 1) as p:
        for t in (64, 256, 1024):
            for k in (1, 8):
                p.set_config(t, k)
                o = host(p.run(dframes, items))[0]
                np.testing.assert_array_equal(o[:, :3], want, err_msg=f"T={t} K={k}")
                np.testing.assert_array_equal(o[:, 3], want[:, 2] / (2160 * 3840))


def test_many_items_compact_and_table_paths():
    """300 crops of one frame into one output tensor (kernel-argument
    form), and the same crops as separate outputs (device table)."""
    say("stats: 300 crops")
    cfg = datagen.config2(300, seed=4)
    ch = cfg["chain"]
    st, ims = oracle_refs(ch, cfg["frames"], cfg["items"])
    dframes = to_dev(cfg["frames"])
    B = len(cfg["items"])
    one = torch.full((B, 3, 4), float("nan"), dtype=torch.float64, device="cuda:0")
    with Plan(stats_of(ch), B, strict=True) as p:
        compact = host(p.run(dframes, cfg["items"], outs=[one[b] for b in range(B)]))
        table = host(p.run(dframes, cfg["items"]))
    for b in range(B):
        check(compact[b], st[b], ims[b], True, f"compact item {b}")
        np.testing.assert_array_equal(compact[b], table[b])


def test_repeat_runs_and_graph_replays_are_identical():
    """Repeated eager runs and graph replays (partials and combine captured
    together) give the same bits as the first run."""
    say("stats: repeats and graph replays")
    cfg = datagen.config2(40, seed=5)
    ch = cfg["chain"]
    dframes = to_dev(cfg["frames"])
    with Plan(stats_of(ch), 40) as p:
        first = host(p.run(dframes, cfg["items"]))
        for _ in range(3):
            again = host(p.run(dframes, cfg["items"]))
            for a, b in zip(first, again):
                np.testing.assert_array_equal(a, b)
    with Plan(stats_of(ch), 40, use_graph=True) as p:
        for _ in range(4):
            rep = host(p.run(dframes, cfg["items"]))
            for a, b in zip(first, rep):
                np.testing.assert_array_equal(a, b)


def test_unfused_stats_match_oracle():
    say("stats: unfused baseline")
    cfg = datagen.config2(6, seed=6)
    ch = cfg["chain"]
    st, ims = oracle_refs(ch, cfg["frames"], cfg["items"])
    dframes = to_dev(cfg["frames"])
    with Plan(stats_of(ch), 6, strict=True) as p:
        outs = host(p.run_unfused(dframes, cfg["items"]))
    for b, o in enumerate(outs):
        check(o, st[b], ims[b], True, f"unfused item {b}")


def test_timed_stats_run_brackets_both_kernels():
    """fk_run_timed on a stats plan: the same results as fk_run, and an
    elapsed time from the first kernel's start to the combine's end."""
    say("stats: timed run")
    cfg = datagen.config2(12, seed=8)
    ch = stats_of(cfg["chain"])
    dframes = to_dev(cfg["frames"])
    with Plan(ch, 12) as p:
        ref = host(p.run(dframes, cfg["items"]))
        outs = [torch.full((3, 4), float("nan"), dtype=torch.float64, device="cuda:0") for _ in range(12)]
        arr = fk.make_items(ch, dframes, cfg["items"], outs)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        e1.record()
        torch.cuda.synchronize()
        fk.fk_run_timed(p.h, arr, 12, fk.stream_handle(), e0.cuda_event, e1.cuda_event)
        torch.cuda.synchronize()
        assert 0.0 < e0.elapsed_time(e1) < 50.0
        got = host(outs)
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("C", [1, 3, 4])
def test_u8_cast_only_stats_match_oracle_and_float_path(C):
    """u8 chains with no arithmetic after the cast (integer accumulation)
    against the oracle, exactly: whole frames, dword-aligned and unaligned
    crops, widths that are not a multiple of 4, with and without the
    channel swap.  The same chain with a Mul by 1 (float accumulation, the
    same values) gives the same bits."""
    g = datagen.rng(40 + C)
    H, W = 45, 203
    frames = [datagen.frame(g, H, W, C) for _ in range(2)]
    # W * C bytes per row: 203, 609, 812 -> rows dword-aligned only for C = 4
    items = [datagen.whole_frame_item(frames[0]),
             {"frame": 1, "x": 4, "y": 3, "w": 96, "h": 40, "out_w": 96, "out_h": 40},
             {"frame": 0, "x": 1, "y": 0, "w": 64, "h": 17, "out_w": 64, "out_h": 17},
             {"frame": 1, "x": 8, "y": 5, "w": 13, "h": 9, "out_w": 13, "out_h": 9}]
    aligned = np.ascontiguousarray(frames[0][:, :200])  # 200 * C bytes per row
    dframes = to_dev(frames + [aligned])
    items.append({"frame": 2, "x": 0, "y": 0, "w": 200, "h": H, "out_w": 200, "out_h": H})
    frames_all = frames + [aligned]
    for swap in ([False, True] if C >= 3 else [False]):
        say("stats: u8 cast only, C", C, "swap", swap)
        ops = ([{"kind": "swap", "k": []}] if swap else []) + [{"kind": "cvt", "k": []}]
        ch = {"read": {"kind": "plain", "dtype": "u8", "channels": C, "out_w": 0, "out_h": 0},
              "ops": ops, "write": {"dtype": "f32", "layout": "packed"}}
        ch_f = dict(ch, ops=ops + [{"kind": "mul", "k": [1.0]}])
        st = [r["out"] for r in oracle.run_chain(stats_of(ch), frames_all, items)]
        for t, k in ((256, 8), (64, 1), (1024, 2)):
            with Plan(stats_of(ch), len(items), config_source=fk.FK_CONFIG_MANUAL,
                      manual=(t, k)) as p:
                got = host(p.run(dframes, items))
            with Plan(stats_of(ch_f), len(items), config_source=fk.FK_CONFIG_MANUAL,
                      manual=(t, k)) as p:
                got_f = host(p.run(dframes, items))
            for b in range(len(items)):
                np.testing.assert_array_equal(got[b], st[b], err_msg=f"item {b} T={t} K={k} swap={swap}")
                np.testing.assert_array_equal(got[b], got_f[b], err_msg=f"float path, item {b}")
