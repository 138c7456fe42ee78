"""Device memory saved by vertical fusion (the memory comparison of the
paper's evaluation, Section VI-L): the fused chain keeps every intermediate
in registers, so after a plan's first run further fused runs take no
device memory at all, while the unfused pipeline needs scratch for its
materialised intermediates -- the u8 crop and two ping-pong fp32 images
(each op reads one and writes the other)."""
import pytest
import torch

import datagen
import paper_2508_07071_amd as fk
from fkhelpers import Plan, alloc_outs, to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def a256(v):
    return (v + 255) // 256 * 256


def free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("batch", [10, 50, 300])
def test_fused_runs_take_no_device_memory(batch):
    """Batches of 60x120 items as in the paper's memory comparison: after
    the first run (which may create the plan's run-table ring for a batch
    too large for the kernel arguments) the device's free memory does not
    move over 20 more runs."""
    say("fused memory, batch", batch)
    g = datagen.rng(batch)
    # one frame per item: no constant-stride form, so batches above 32
    # items take the device run table
    frames = [datagen.frame(g, 64, 128, 3) for _ in range(batch)]
    dframes = to_dev(frames)
    chain = datagen.normalize_chain(60, 120)
    items = [{"frame": b, "x": 2, "y": 1, "w": 100, "h": 50, "out_w": 60, "out_h": 120}
             for b in range(batch)]
    outs = alloc_outs(chain, items)
    with Plan(chain, batch) as p:
        arr = fk.make_items(chain, dframes, items, outs)
        fk.fk_run(p.h, arr, batch, fk.stream_handle())
        f0 = free_bytes()
        for _ in range(20):
            fk.fk_run(p.h, arr, batch, fk.stream_handle())
        assert free_bytes() == f0


def test_unfused_scratch_is_the_materialised_intermediates():
    """The unfused baseline's scratch for one item is exactly its
    intermediates: the cropped u8 ROI plus two fp32 images of the larger of
    the ROI and the output (256-byte aligned each); the fused plan needs
    none of it.  For the paper's 60x120 float3 items one fp32 intermediate
    is 86,400 B (three of them, the paper's count for its pipeline, are
    259.2 KB)."""
    say("unfused scratch = intermediates")
    g = datagen.rng(3)
    fr = datagen.frame(g, 300, 400, 3)
    dframes = to_dev([fr])
    chain = datagen.normalize_chain(120, 60)
    cases = [(10, 20, 100, 50), (0, 0, 400, 300), (5, 5, 33, 17)]
    with Plan(chain, 1) as p:
        for x, y, w, h in cases:
            it = {"frame": 0, "x": x, "y": y, "w": w, "h": h, "out_w": 120, "out_h": 60}
            arr = fk.make_items(chain, dframes, [it], alloc_outs(chain, [it]))
            got = fk.fk_unfused_scratch_bytes(p.h, arr, 1)
            want = a256(w * h * 3) + 2 * a256(max(w * h, 120 * 60) * 3 * 4)
            assert got == want, (x, y, w, h, got, want)
    assert 120 * 60 * 3 * 4 == 86400


def test_unfused_run_with_exact_scratch_matches_fused():
    """The unfused pipeline runs in exactly the scratch it reports (a
    smaller buffer is refused) and gives the fused strict result."""
    say("unfused in its exact scratch")
    import numpy as np
    g = datagen.rng(4)
    fr = datagen.frame(g, 200, 256, 3)
    dframes = to_dev([fr])
    chain = datagen.normalize_chain(60, 120)
    items = [{"frame": 0, "x": 3, "y": 4, "w": 90, "h": 70, "out_w": 60, "out_h": 120}]
    with Plan(chain, 1, strict=True) as p:
        fused = p.run(dframes, items)
        outs = alloc_outs(chain, items)
        arr = fk.make_items(chain, dframes, items, outs)
        need = fk.fk_unfused_scratch_bytes(p.h, arr, 1)
        scratch = torch.empty(need, dtype=torch.uint8, device="cuda:0")
        with pytest.raises(fk.FKError):
            fk.fk_run_unfused(p.h, arr, 1, scratch.data_ptr(), need - 1, fk.stream_handle())
        fk.fk_run_unfused(p.h, arr, 1, scratch.data_ptr(), need, fk.stream_handle())
        torch.cuda.synchronize()
    assert np.array_equal(outs[0].cpu().numpy().view(np.uint32), fused[0].cpu().numpy().view(np.uint32))
