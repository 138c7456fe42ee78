"""The launch-configuration autotuner on the GPU: it times all 20
configurations, picks the fastest with the documented tie-break, installs
it in the plan, and the tuned plan still matches the oracle bit for bit in
the strict mode.  The cost model's choice is then re-timed on the box
running the test against the autotuner's best."""
import math
import os

import numpy as np
import pytest

import datagen
import oracle
import paper_2508_07071_amd as fk
from fkhelpers import Plan, alloc_outs, assert_bitexact, host, to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def tune_and_check(cfg, reps=5):
    chain, items = cfg["chain"], cfg["items"]
    dframes = to_dev(cfg["frames"])
    space = [(c.block_threads, c.coarsen) for c in fk.fk_autotune_space()]
    with Plan(chain, len(items), strict=True) as p:
        outs = alloc_outs(chain, items)
        arr = fk.make_items(chain, dframes, items, outs)
        best, times = fk.fk_autotune(p.h, arr, len(items), reps)
        t = np.asarray(times, np.float64)
        assert t.shape == (20,)
        assert np.all(np.isfinite(t)) and np.all(t > 0), times
        # the first minimum in the space's order: fewer threads, then less
        # coarsening, win ties
        i = int(np.flatnonzero(t == t.min())[0])
        assert (best.block_threads, best.coarsen) == space[i], (best, times)
        cur = fk.fk_plan_get_config(p.h)
        assert (cur.block_threads, cur.coarsen) == space[i]
        got = host(p.run(dframes, items, outs=alloc_outs(chain, items)))
    refs = oracle.run_chain(chain, cfg["frames"], items)
    for b, (g, r) in enumerate(zip(got, refs)):
        assert_bitexact(g, r["out"], f"tuned {space[i]} item {b}")
    return space[i], t


def test_autotune_config2_batch50():
    say("autotune config2 B=50")
    cfg = datagen.config2(50, seed=2)
    tune_and_check(cfg)


def test_autotune_config1_small_frame():
    say("autotune config1 N=16, 270x480")
    cfg = datagen.config1(16, seed=4, frame_hw=(270, 480))
    tune_and_check(cfg)


def test_autotune_runtime_tier_chain():
    say("autotune run-time chain")
    g = datagen.rng(31)
    fr = datagen.frame(g, 200, 300, 4, dtype="f16")
    chain = {"read": {"kind": "crop_resize", "dtype": "f16", "channels": 4, "out_w": 40, "out_h": 24},
             "ops": [{"kind": "swap", "k": []}, {"kind": "div", "k": [1.5, 0.75, 1.25, 1.0]},
                     {"kind": "sub", "k": [0.25]}],
             "write": {"dtype": "f16", "layout": "planar"}}
    items = [{"frame": 0, "x": int(x), "y": int(y), "w": 97, "h": 61, "out_w": 40, "out_h": 24}
             for x, y in [(0, 0), (11, 7), (200, 139), (50, 50)]]
    tune_and_check({"chain": chain, "frames": [fr], "items": items})


def test_autotune_rejects_bad_arguments():
    say("autotune argument checks")
    cfg = datagen.config2(4, seed=3)
    dframes = to_dev(cfg["frames"])
    with Plan(cfg["chain"], 4) as p:
        arr = fk.make_items(cfg["chain"], dframes, cfg["items"], alloc_outs(cfg["chain"], cfg["items"]))
        for n, reps in [(0, 3), (5, 3), (4, 0), (4, 20000)]:
            with pytest.raises(fk.FKError) as e:
                fk.fk_autotune(p.h, arr, n, reps)
            assert e.value.status == fk.FK_ERR_INVALID_ARG
        before = fk.fk_plan_get_config(p.h)
        assert (before.block_threads, before.coarsen) == (256, 1)


DATASET = os.path.join(os.path.dirname(fk.__file__), "data", "costmodel_dataset.npz")


@pytest.mark.skipif(not os.path.exists(DATASET), reason="labelled dataset not present")
def test_model_choice_against_live_autotune():
    """Train on the committed labels, then for 20 chains the dataset never
    saw (another seed, inputs up to 256 MiB) let the model pick a plan's
    configuration and compare its time with the autotuner's best, both
    timed here by the same sweep: geometric mean of t_best / t_pick >= 0.9."""
    say("cost model vs live autotune, 20 unseen chains")
    from paper_2508_07071_amd import costmodel as cm
    data = cm.load_shards([DATASET])
    model, rep = cm.fit(data, epochs=100)
    try:
        live = cm.live_quality(model, n=20, seed=20260, reps=10, max_input_bytes=1 << 28)
    finally:
        fk.fk_model_destroy(model)
    q = np.asarray(live["quality"])
    geo = math.exp(np.mean(np.log(q)))
    print(f"[live] model geomean {geo:.3f}, default {live['default']['geomean']:.3f}, "
          f"within 10%: {np.mean(q >= 0.9):.2f}", flush=True)
    assert geo >= 0.90, live
