"""The serving loop: continuous batching gives every request the same result
alone and in a mix; the baseline modes agree; admission respects the
budget; results match the oracle."""
import time

import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_2508_07071_amd as fk
from fkhelpers import assert_bitexact, assert_close

pytestmark = pytest.mark.gpu

CHAIN = datagen.normalize_chain(224, 224)


def say(*a):
    print("[case]", *a, flush=True)


def requests(seed, n, max_crops=12, hw=((480, 640), (1080, 1920)), min_crops=1, big=False):
    g = datagen.rng(seed)
    reqs = []
    for _ in range(n):
        H = int(g.integers(hw[0][0], hw[1][0] + 1))
        W = int(g.integers(hw[0][1], hw[1][1] + 1))
        frame = torch.from_numpy(datagen.frame(g, H, W, 3)).pin_memory()
        k = int(g.integers(min_crops, max_crops + 1))
        crops = []
        for _ in range(k):
            w = int(g.integers(60, min(600, W) + 1))
            h = int(g.integers(60, min(600, H) + 1))
            out = (224, 224) if (big or g.uniform() < 0.5) else (64, 128)
            crops.append({"x": int(g.integers(0, W - w + 1)), "y": int(g.integers(0, H - h + 1)),
                          "w": w, "h": h, "out_w": out[0], "out_h": out[1]})
        reqs.append((frame, crops))
    return reqs


def collect(srv, arena, tickets, crops_by_ticket, timeout=30.0):
    """Wait for every ticket; copy each crop's output to the host; release."""
    got = {}
    t_end = time.time() + timeout
    while len(got) < len(tickets) and time.time() < t_end:
        for c in fk.fk_server_poll(srv, 64):
            crops = crops_by_ticket[c.ticket]
            assert c.status == 0
            offs = fk.output_offsets(CHAIN, crops)
            outs = []
            for off, cr in zip(offs, crops):
                n = 3 * cr["out_h"] * cr["out_w"]
                base = c.outputs - arena.data_ptr() + off
                view = arena[base:base + 4 * n].view(torch.float32)
                outs.append(view.cpu().numpy().reshape(3, cr["out_h"], cr["out_w"]))
            got[c.ticket] = outs
            fk.fk_server_release(srv, c.ticket)
        time.sleep(1e-3)
    assert len(got) == len(tickets), f"{len(got)}/{len(tickets)} completed"
    return got


def serve(reqs, mode=fk.FK_SERVER_BATCHED, budget=0, strict=True, arena_mb=512, stagger=0.0,
          max_inflight=3):
    desc = fk.chain_desc(CHAIN)
    arena = torch.empty(arena_mb << 20, dtype=torch.uint8, device="cuda:0")
    srv = fk.fk_server_create(fk.server_opts(desc, arena, budget_bytes=budget, mode=mode,
                                             strict=strict, max_batch_items=256,
                                             max_inflight=max_inflight))
    try:
        crops_by_ticket, order = {}, []
        for frame, crops in reqs:
            t = fk.fk_server_submit(srv, fk.make_request(frame, crops))
            crops_by_ticket[t] = crops
            order.append(t)
            if stagger:
                time.sleep(stagger)
        got = collect(srv, arena, order, crops_by_ticket)
        t_end = time.time() + 5
        st = fk.fk_server_stats_get(srv)
        while st.bytes_in_use and time.time() < t_end:  # releases apply asynchronously
            time.sleep(1e-3)
            st = fk.fk_server_stats_get(srv)
    finally:
        fk.fk_server_destroy(srv)
        torch.cuda.synchronize()
    return [got[t] for t in order], st


def test_alone_and_in_the_mix_give_the_same_bits():
    say("alone vs mix")
    # 640x480 frames with 48-64 crops of 224x224 each.  Frames already on
    # the device, submitted in a burst with one launch in flight: the
    # requests that arrive while it runs are merged into the next launches.
    reqs = requests(1, 24, min_crops=48, max_crops=64, hw=((480, 640), (480, 640)), big=True)
    dev = [(f.to("cuda:0"), c) for f, c in reqs]
    torch.cuda.synchronize()
    target = reqs[7]
    alone, _ = serve([target], max_inflight=1)
    mixed, st = serve(dev, max_inflight=1)
    assert st.launches < len(reqs), st.launches  # launches shared between requests
    for a, b in zip(alone[0], mixed[7]):
        assert_bitexact(b, a, "request 7 in the mix")
    # host frames: each copy (~40 us) outlasts a launch, so requests mostly
    # launch alone; still the same bits, staggered or not
    for kw in ({"max_inflight": 1}, {"max_inflight": 3, "stagger": 0.0005}):
        mixed_h, _ = serve(reqs, **kw)
        for a, b in zip(alone[0], mixed_h[7]):
            assert_bitexact(b, a, f"request 7 among host frames {kw}")


def test_server_outputs_match_oracle():
    say("server vs oracle")
    reqs = requests(2, 3, max_crops=5)
    got, _ = serve(reqs, strict=True)
    for (frame, crops), outs in zip(reqs, got):
        f = frame.numpy()
        items = [dict(c, frame=0) for c in crops]
        refs = oracle.run_chain(CHAIN, [f], items)
        for o, r in zip(outs, refs):
            assert_bitexact(o, r["out"], "strict server")
    got2, _ = serve(reqs, strict=False)
    for (frame, crops), outs in zip(reqs, got2):
        refs = oracle.run_chain(CHAIN, [frame.numpy()], [dict(c, frame=0) for c in crops])
        for o, r in zip(outs, refs):
            assert_close(o, r, s_floor=1.0, what="default server")


def test_baseline_modes_agree_bitwise():
    say("modes agree")
    reqs = requests(3, 6, max_crops=6)
    base, st_b = serve(reqs, mode=fk.FK_SERVER_BATCHED)
    per, st_p = serve(reqs, mode=fk.FK_SERVER_PER_REQUEST)
    unf, _ = serve(reqs, mode=fk.FK_SERVER_UNFUSED)
    for i in range(len(reqs)):
        for a, b, c in zip(base[i], per[i], unf[i]):
            assert_bitexact(b, a, "per-request")
            assert_bitexact(c, a, "unfused")
    assert st_p.launches >= len(reqs)


def test_budget_defers_admission_and_rejects_oversize():
    say("budget")
    reqs = requests(4, 10, max_crops=4, hw=((480, 640), (720, 1280)))
    # room for about two requests at a time
    budget = 2 * (1280 * 720 * 3 + 4 * 224 * 224 * 12 + 4096)
    got, st = serve(reqs, budget=budget)
    assert len(got) == 10 and st.peak_bytes <= budget and st.completed == 10
    desc = fk.chain_desc(CHAIN)
    arena = torch.empty(64 << 20, dtype=torch.uint8, device="cuda:0")
    srv = fk.fk_server_create(fk.server_opts(desc, arena, budget_bytes=1 << 20))
    try:
        frame, crops = reqs[0]
        with pytest.raises(fk.FKError) as e:
            fk.fk_server_submit(srv, fk.make_request(frame, crops))
        assert e.value.status == fk.FK_ERR_BUDGET
        bad = [dict(crops[0], x=frame.shape[1])]
        with pytest.raises(fk.FKError) as e:
            fk.fk_server_submit(srv, fk.make_request(frame, bad))
        assert e.value.status == fk.FK_ERR_INVALID_ARG
    finally:
        fk.fk_server_destroy(srv)


def test_release_returns_all_memory():
    say("release")
    reqs = requests(5, 5, max_crops=3)
    _, st = serve(reqs)
    assert st.completed == 5 and st.bytes_in_use == 0 and st.peak_bytes > 0


def test_release_only_after_completion():
    """A ticket's memory returns to the budget only once a poll has handed
    out its completion: releasing an unknown ticket, a ticket not yet
    returned by a poll (queued, running or finished unseen), or a ticket
    twice is refused and changes nothing."""
    say("release before completion")
    reqs = requests(41, 3, max_crops=4)
    desc = fk.chain_desc(CHAIN)
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda:0")
    srv = fk.fk_server_create(fk.server_opts(desc, arena, max_batch_items=64))
    try:
        with pytest.raises(fk.FKError) as e:
            fk.fk_server_release(srv, 12345)
        assert e.value.status == fk.FK_ERR_BAD_STATE
        tickets = [fk.fk_server_submit(srv, fk.make_request(fr, cr)) for fr, cr in reqs]
        done = set()
        t_end = time.time() + 30
        while len(done) < len(tickets) and time.time() < t_end:
            for c in fk.fk_server_poll(srv, 16):
                assert c.status == 0
                done.add(c.ticket)
            for t in tickets:
                if t not in done:
                    with pytest.raises(fk.FKError) as e:
                        fk.fk_server_release(srv, t)
                    assert e.value.status == fk.FK_ERR_BAD_STATE
            time.sleep(1e-3)
        assert done == set(tickets)
        for t in tickets:
            fk.fk_server_release(srv, t)
            with pytest.raises(fk.FKError) as e:
                fk.fk_server_release(srv, t)
            assert e.value.status == fk.FK_ERR_BAD_STATE
        t_end = time.time() + 5
        while fk.fk_server_stats_get(srv).bytes_in_use and time.time() < t_end:
            time.sleep(1e-3)
        assert fk.fk_server_stats_get(srv).bytes_in_use == 0
    finally:
        fk.fk_server_destroy(srv)


def test_device_frames_match_host_frames_and_merge_into_launches():
    """Requests whose frames are already on the device (no copy) give the
    bits of the same frames sent from the host and of the oracle; their
    budget blocks hold only outputs, and a burst of them submitted while
    the GPU is busy is merged into launches carrying several requests."""
    say("device-resident frames")
    reqs = requests(5, 16, min_crops=8, max_crops=24, hw=((480, 640), (720, 1280)))
    host_out, st_host = serve(reqs)
    dev_reqs = [(f.to("cuda:0"), c) for f, c in reqs]
    torch.cuda.synchronize()
    dev_out, st_dev = serve(dev_reqs, max_inflight=1)
    for i in range(len(reqs)):
        for j, (a, b) in enumerate(zip(host_out[i], dev_out[i])):
            assert_bitexact(b, a, f"request {i} crop {j}")
    assert st_dev.peak_bytes < st_host.peak_bytes
    assert st_dev.launches < len(reqs), (st_dev.launches, len(reqs))
    # a mix of host and device frames
    mix = [r if i % 2 else dev_reqs[i] for i, r in enumerate(reqs)]
    mix_out, _ = serve(mix)
    for i in range(len(reqs)):
        for j, (a, b) in enumerate(zip(host_out[i], mix_out[i])):
            assert_bitexact(b, a, f"mixed request {i} crop {j}")
    # the oracle, for two requests
    for i in (0, 9):
        frame, crops = reqs[i]
        refs = oracle.run_chain(CHAIN, [frame.numpy()], [dict(c, frame=0) for c in crops])
        for j, r in enumerate(refs):
            assert_bitexact(dev_out[i][j], r["out"], f"oracle request {i} crop {j}")


def test_device_flag_on_a_host_frame_is_refused():
    """A request that says its frame is on the device must point at device
    memory: a pinned host frame with the flag set is refused at submit."""
    say("device flag on a host frame")
    frame, crops = requests(6, 1)[0]
    desc = fk.chain_desc(CHAIN)
    arena = torch.empty(64 << 20, dtype=torch.uint8, device="cuda:0")
    srv = fk.fk_server_create(fk.server_opts(desc, arena))
    try:
        req = fk.make_request(frame, crops)
        assert req.frame_on_device == 0
        req.frame_on_device = 1
        with pytest.raises(fk.FKError) as e:
            fk.fk_server_submit(srv, req)
        assert e.value.status == fk.FK_ERR_INVALID_ARG
        assert fk.fk_server_stats_get(srv).submitted == 0
    finally:
        fk.fk_server_destroy(srv)
