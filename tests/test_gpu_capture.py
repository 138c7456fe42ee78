"""fk_run under the caller's stream capture: runs whose items travel in the
kernel arguments are captured as their launches, so a graph of several
runs replays them; every replay (with eager work between replays) gives the
bits of the same runs done eagerly.  Runs that need the run table, plans
that replay their own graph, and timed runs are refused under capture."""
import numpy as np
import pytest
import torch

import datagen
import paper_2508_07071_amd as fk
from fkhelpers import alloc_outs, assert_bitexact, to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("batch,one_tensor", [(8, False), (256, True)])
def test_graph_of_several_runs_replays_the_eager_bits(batch, one_tensor):
    say("capture 4 runs, batch", batch)
    c = datagen.config2(batch, seed=21)
    g = datagen.rng(22)
    frames = [torch.from_numpy(datagen.frame(g, 2160, 3840, 3)).to("cuda:0") for _ in range(4)]
    chain = c["chain"]
    outs, arrs = [], []
    for r in range(4):
        if one_tensor:
            o = torch.full((batch, 3, 128, 64), float("nan"), device="cuda:0")
            ol = [o[b] for b in range(batch)]
        else:
            ol = alloc_outs(chain, c["items"])
            o = ol
        outs.append(o)
        arrs.append(fk.make_items(chain, [frames[r]], c["items"], ol))
    plan = fk.fk_plan_create(fk.chain_desc(chain), batch, fk.plan_opts())
    try:
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            for r in range(4):
                fk.fk_run(plan, arrs[r], batch, fk.stream_handle(s))
        torch.cuda.synchronize()
        eager = [np.stack([t.cpu().numpy() for t in o]) if not one_tensor else o.cpu().numpy()
                 for o in outs]
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            for r in range(4):
                fk.fk_run(plan, arrs[r], batch, fk.stream_handle(s))
        for rep in range(3):
            for o in outs:  # eager work between replays
                for t in (o if not one_tensor else [o]):
                    t.fill_(float("nan"))
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            for r in range(4):
                got = np.stack([t.cpu().numpy() for t in outs[r]]) if not one_tensor else outs[r].cpu().numpy()
                assert_bitexact(got, eager[r], f"replay {rep} run {r}")
    finally:
        fk.fk_plan_destroy(plan)


def test_table_batches_graph_plans_and_timed_runs_are_refused_under_capture():
    say("capture refusals")
    g = datagen.rng(23)
    frames = to_dev([datagen.frame(g, 300, 512, 3) for _ in range(3)])
    items = []
    for f in range(3):
        items += datagen.random_crops(g, 20, 512, 300, frame_index=f)
    chain = datagen.normalize_chain(64, 128)
    arr = fk.make_items(chain, frames, items, alloc_outs(chain, items))
    small = fk.make_items(chain, frames, items[:4], alloc_outs(chain, items[:4]))
    plan = fk.fk_plan_create(fk.chain_desc(chain), len(items), fk.plan_opts())
    gplan = fk.fk_plan_create(fk.chain_desc(chain), len(items), fk.plan_opts(use_graph=True))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    ev1.record()
    torch.cuda.synchronize()
    try:
        s = torch.cuda.Stream()
        for what, call in [
            ("table batch", lambda: fk.fk_run(plan, arr, len(items), fk.stream_handle(s))),
            ("graph plan", lambda: fk.fk_run(gplan, small, 4, fk.stream_handle(s))),
            ("timed run", lambda: fk.fk_run_timed(plan, small, 4, fk.stream_handle(s),
                                                  ev0.cuda_event, ev1.cuda_event)),
        ]:
            graph = torch.cuda.CUDAGraph()
            with pytest.raises(fk.FKError) as e:
                with torch.cuda.graph(graph, stream=s):
                    call()
            assert e.value.status == fk.FK_ERR_UNSUPPORTED, what
            torch.cuda.synchronize()
        # the same runs are fine outside capture
        fk.fk_run(plan, arr, len(items), fk.stream_handle(s))
        fk.fk_run(gplan, small, 4, fk.stream_handle(s))
        torch.cuda.synchronize()
    finally:
        fk.fk_plan_destroy(plan)
        fk.fk_plan_destroy(gplan)
