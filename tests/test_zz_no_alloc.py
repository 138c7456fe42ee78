"""The no-allocation unfused entry (fk_run_unfused_noalloc): the unfused
baseline with its workspace in the library's own device array gives the
same bits as fk_run_unfused with a caller-allocated workspace, on two calls
in a row (the second with a smaller input, over the first call's leftover
workspace contents), allocates no device memory, and refuses items whose
workspace exceeds the array before launching anything."""
import numpy as np
import pytest
import torch

import datagen
import paper_2508_07071_amd as fk
from fkhelpers import Plan, alloc_outs, assert_bitexact, host, to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def both_entries(p, chain, dframes, items):
    """Outputs of the workspace entry and of the no-allocation entry."""
    ref = alloc_outs(chain, items)
    arr = fk.make_items(chain, dframes, items, ref)
    need = fk.fk_unfused_scratch_bytes(p.h, arr, len(items))
    assert 0 < need <= fk.FK_NOALLOC_SCRATCH_BYTES, need
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    fk.fk_run_unfused(p.h, arr, len(items), ws.data_ptr(), need, fk.stream_handle())
    got = alloc_outs(chain, items)
    arr2 = fk.make_items(chain, dframes, items, got)
    fk.fk_run_unfused_noalloc(p.h, arr2, len(items), fk.stream_handle())
    return host(ref), host(got)


def test_noalloc_matches_workspace_entry_then_smaller_input():
    cfg = datagen.config2(8, seed=5)
    chain = cfg["chain"]
    dframes = to_dev(cfg["frames"])
    g = datagen.rng(6)
    small = []
    for _ in range(3):
        w, h = int(g.integers(60, 121)), int(g.integers(60, 121))
        small.append({"frame": 0, "x": int(g.integers(0, 3840 - w + 1)),
                      "y": int(g.integers(0, 2160 - h + 1)), "w": w, "h": h,
                      "out_w": 64, "out_h": 128})
    with Plan(chain, 8, strict=True) as p:
        say("no-alloc unfused, config2 B=8 then B=3 smaller crops")
        r1, g1 = both_entries(p, chain, dframes, cfg["items"])
        f0 = free_bytes()
        r2, g2 = both_entries(p, chain, dframes, small)
        # the workspace entry's own buffer came from torch's cache, not the driver
        assert free_bytes() == f0
    for b, (x, y) in enumerate(zip(g1, r1)):
        assert not np.isnan(x).any(), f"call 1 item {b} not written"
        assert_bitexact(x, y, f"call 1 item {b}")
    for b, (x, y) in enumerate(zip(g2, r2)):
        assert not np.isnan(x).any(), f"call 2 item {b} not written"
        assert_bitexact(x, y, f"call 2 item {b}")


def test_noalloc_stats_write_matches_workspace_entry():
    """A stats write keeps its reduction partials in the workspace too."""
    say("no-alloc unfused, stats write")
    g = datagen.rng(7)
    fr = datagen.frame(g, 300, 500, 3)
    dframes = to_dev([fr])
    chain = {"read": {"kind": "crop_resize", "dtype": "u8", "channels": 3, "out_w": 96, "out_h": 80},
             "ops": [{"kind": "cvt", "k": []}, {"kind": "mul", "k": [0.5]}],
             "write": {"dtype": "f64", "layout": "stats"}}
    items = [{"frame": 0, "x": 10, "y": 20, "w": 300, "h": 200, "out_w": 96, "out_h": 80},
             {"frame": 0, "x": 0, "y": 0, "w": 50, "h": 40, "out_w": 96, "out_h": 80}]
    with Plan(chain, 2) as p:
        r, got = both_entries(p, chain, dframes, items)
    for b, (x, y) in enumerate(zip(got, r)):
        assert np.array_equal(x.view(np.uint64), y.view(np.uint64)), (b, x, y)


def test_noalloc_refuses_items_beyond_its_workspace():
    say("no-alloc unfused, oversized item refused")
    cfg = datagen.config2(1, seed=8)
    chain = cfg["chain"]
    dframes = to_dev(cfg["frames"])
    big = [{"frame": 0, "x": 0, "y": 0, "w": 2000, "h": 1500, "out_w": 64, "out_h": 128}]
    with Plan(chain, 1) as p:
        outs = alloc_outs(chain, big)
        arr = fk.make_items(chain, dframes, big, outs)
        assert fk.fk_unfused_scratch_bytes(p.h, arr, 1) > fk.FK_NOALLOC_SCRATCH_BYTES
        with pytest.raises(fk.FKError) as e:
            fk.fk_run_unfused_noalloc(p.h, arr, 1, fk.stream_handle())
        assert e.value.status == fk.FK_ERR_UNSUPPORTED
        with pytest.raises(fk.FKError) as e:
            fk.fk_run_unfused_noalloc(p.h, arr, 2, fk.stream_handle())
        assert e.value.status == fk.FK_ERR_INVALID_ARG
    assert np.isnan(host(outs)[0]).all()
