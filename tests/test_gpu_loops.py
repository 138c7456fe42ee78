"""The loop (repeat) op on the GPU, through the C ABI, against the oracle:
the compile-time loop chain (one Mul and one Add run P times, the trip
count a kernel argument) on the batch-50 60x120 workload, and loops inside
run-time op lists.  Strict plans are bit-exact; default plans (contracted
to FMA) are within |g - r| <= 1e-5 * max(|r|, s), s = the oracle's largest
intermediate magnitude."""
import numpy as np
import pytest

import datagen
import oracle
import paper_2508_07071_amd as fk
from fkhelpers import Plan, assert_bitexact, assert_close, host, to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def run_modes(chain, frames, items, refs, what, tier=None, static=None, config=None):
    dframes = to_dev(frames)
    kw = {} if tier is None else {"tier": tier}
    for strict in (True, False):
        with Plan(chain, len(items), strict=strict, **kw) as p:
            if static is not None:
                assert fk.fk_plan_get_tier(p.h) == int(static)
            if config is not None:
                p.set_config(*config)
            outs = host(p.run(dframes, items))
        for b, (g, r) in zip(range(len(items)), zip(outs, refs)):
            if r is None:
                continue
            if strict:
                assert_bitexact(g, r["out"], f"{what} strict item {b}")
            else:
                assert_close(g, r, what=f"{what} item {b}")


@pytest.mark.parametrize("channels", [1, 3])
@pytest.mark.parametrize("pairs", [1, 7, 100])
def test_loop_batch_matches_oracle(pairs, channels):
    say("loop batch 50 x 60x120, pairs", pairs, "channels", channels)
    cfg = datagen.loop_batch(pairs, seed=pairs, channels=channels)
    refs = oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"])
    run_modes(cfg["chain"], cfg["frames"], cfg["items"], refs, f"static P={pairs}", static=True)
    run_modes(cfg["chain"], cfg["frames"], cfg["items"], refs, f"runtime P={pairs}",
              tier=fk.FK_TIER_RUNTIME, static=False)


def test_loop_batch_10000_pairs_sampled_items():
    """The longest chain of the sweep (10^4 Mul+Add pairs) in the launch
    shape the benchmark times; the oracle checks three items, and every
    item is held to the affine closed form m^P x + a (1 - m^P) / (1 - m)."""
    pairs = 10000
    say("loop batch 50 x 60x120, pairs", pairs)
    cfg = datagen.loop_batch(pairs, seed=11)
    sample = (0, 26, 49)
    items = cfg["items"]
    refs = [None] * len(items)
    for b, r in zip(sample, oracle.run_chain(cfg["chain"], cfg["frames"], [items[b] for b in sample])):
        refs[b] = r
    run_modes(cfg["chain"], cfg["frames"], items, refs, f"P={pairs}", static=True)
    m, a = cfg["chain"]["ops"][1]["k"][0], cfg["chain"]["ops"][2]["k"][0]
    with Plan(cfg["chain"], len(items)) as p:
        outs = host(p.run(to_dev(cfg["frames"]), items))
    fr = cfg["frames"][0].astype(np.float64)
    mp = m ** pairs
    for b, o in enumerate(outs):
        it = items[b]
        x = fr[it["y"]:it["y"] + it["h"], it["x"]:it["x"] + it["w"]]
        exact = mp * x + a * (1 - mp) / (1 - m)
        assert np.all(np.abs(o - exact) <= 1e-5 * max(255.0, 1.0 / (1 - m)))


def test_loop_chain_every_launch_config_same_bits():
    say("loop chain, 20 launch configs")
    cfg = datagen.loop_batch(100, seed=5, batch=9, hw=(37, 61))
    dframes = to_dev(cfg["frames"])
    ref = None
    with Plan(cfg["chain"], len(cfg["items"]), strict=True) as p:
        for t in (64, 128, 256, 512, 1024):
            for k in (1, 2, 4, 8):
                p.set_config(t, k)
                outs = host(p.run(dframes, cfg["items"]))
                if ref is None:
                    ref = outs
                for g, r in zip(outs, ref):
                    assert_bitexact(g, r, f"T={t} K={k}")


def add_loops(g, ops):
    out, run = [], 0
    for o in ops:
        out.append(o)
        run = run + 1 if o["kind"] in ("mul", "add", "sub", "div") else 0
        if run and g.uniform() < 0.3:
            out.append({"kind": "loop", "span": int(g.integers(1, run + 1)), "count": int(g.integers(1, 6))})
            run = 0
    return out


@pytest.mark.parametrize("seed", range(3))
def test_random_chains_with_loops_match_oracle(seed):
    say("random chains with loops, seed", seed)
    g = datagen.rng(900 + seed)
    for k in range(8):
        spec = datagen.random_chain_spec(g, max_ops=24, side=(16, 200), max_batch=3)
        ch = spec["chain"]
        ch["ops"] = add_loops(g, ch["ops"])
        fh, fw = spec["frame_hw"]
        frames = [datagen.frame(g, fh, fw, ch["read"]["channels"], dtype=ch["read"]["dtype"])
                  for _ in range(spec["batch"])]
        refs = oracle.run_chain(ch, frames, spec["items"])
        run_modes(ch, frames, spec["items"], refs, f"chain {k} ({len(ch['ops'])} ops)")


def test_unfused_loop_chain_matches_fused_bitwise():
    say("unfused loop chain")
    cfg = datagen.loop_batch(7, seed=2, batch=5)
    dframes = to_dev(cfg["frames"])
    refs = oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"])
    with Plan(cfg["chain"], len(cfg["items"]), strict=True) as p:
        fused = host(p.run(dframes, cfg["items"]))
        unfused = host(p.run_unfused(dframes, cfg["items"]))
    for b, (f, u, r) in enumerate(zip(fused, unfused, refs)):
        assert_bitexact(u, r["out"], f"unfused item {b}")
        assert_bitexact(f, u, f"fused vs unfused item {b}")
