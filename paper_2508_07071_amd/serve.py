"""Open-loop serving workload on the library's server (fk_server_*).

Poisson arrivals at a fixed rate; each request is one uint8 BGR frame
(sides uniform in 640x480 .. 3840x2160) with 1..64 crops, each resized to
224x224 or 64x128 (width x height) and normalised to planar fp32.  Frames
come from a pool of pinned host buffers: a request's W x H frame is a dense
image over the first W*H*3 bytes of a pool frame.  Latency = completion time -
scheduled arrival time on the server's monotonic clock.  With a device pool
the frames are already on the device (as a GPU decoder would leave them) and
the server reads them in place.
"""
from __future__ import annotations

import gc
import time

import numpy as np


def make_pool(n_frames=8, seed=0, max_hw=(2160, 3840), device=False):
    """Frames of random bytes: pinned host tensors, or device tensors."""
    import torch
    g = np.random.default_rng(seed)
    pool = []
    for _ in range(n_frames):
        f = torch.from_numpy(g.integers(0, 256, size=(max_hw[0], max_hw[1], 3), dtype=np.uint8))
        pool.append(f.to("cuda:0") if device else f.pin_memory())
    return pool


def run(rate_hz, n_requests, mode, pool, arena, seed=0, warmup_frac=0.1, max_batch_items=2048,
        max_inflight=3, budget_bytes=0, deadline_s=60.0, config=(0, 0), request_kw=None):
    """Serve n_requests arrivals at rate_hz; returns a stats dict.  Frames
    come from `pool` (host frames are copied, device frames read in place);
    `request_kw` goes to datagen.poisson_requests (frame sizes, crop counts,
    output size)."""
    import datagen
    import paper_2508_07071_amd as fk

    g = datagen.rng(seed)
    reqs = datagen.poisson_requests(g, rate_hz, n_requests, **(request_kw or {}))
    on_device = pool[0].is_cuda
    chain = datagen.normalize_chain(224, 224)
    desc = fk.chain_desc(chain)
    srv = fk.fk_server_create(fk.server_opts(desc, arena, budget_bytes=budget_bytes,
                                             max_batch_items=max_batch_items,
                                             max_inflight=max_inflight, mode=mode, config=config))
    done = {}
    in_bytes = out_bytes = crops = 0
    try:
        built = []
        for i, r in enumerate(reqs):
            fh, fw = r["frame_hw"]
            # a dense fh x fw x 3 image over the pool frame's (random) bytes
            frame = pool[i % len(pool)].view(-1)[:fh * fw * 3].view(fh, fw, 3)
            built.append(fk.make_request(frame, r["crops"], 0.0))
            in_bytes += 0 if on_device else fh * fw * 3
            crops += len(r["crops"])
            out_bytes += sum(c["out_w"] * c["out_h"] * 12 for c in r["crops"])
        # the load generator must not pause: a collection over tens of
        # thousands of request objects would hold back later arrivals (and
        # count as their latency, which starts at the scheduled arrival)
        gc.collect()
        gc.freeze()
        gc.disable()
        t0 = fk.fk_server_clock() + 0.05
        tickets = {}

        def drain():
            for c in fk.fk_server_poll(srv, 512):
                done[c.ticket] = (c.status, c.t_arrival, c.t_admit, c.t_launch, c.t_done, c.n_crops)
                fk.fk_server_release(srv, c.ticket)

        for i, r in enumerate(reqs):
            t_arr = t0 + r["t_arrival"]
            while True:
                now = fk.fk_server_clock()
                if now >= t_arr:
                    break
                drain()
                if t_arr - now > 2e-4:
                    time.sleep(min(t_arr - now - 1e-4, 1e-3))
            built[i].t_arrival = t_arr
            tickets[fk.fk_server_submit(srv, built[i])] = i
        t_end = fk.fk_server_clock() + deadline_s
        while len(done) < len(reqs) and fk.fk_server_clock() < t_end:
            drain()
            time.sleep(2e-4)
        st = fk.fk_server_stats_get(srv)
    finally:
        gc.enable()
        gc.unfreeze()
        fk.fk_server_destroy(srv)
    if len(done) < len(reqs):
        return {"rate_hz": rate_hz, "mode": mode, "error": f"only {len(done)}/{len(reqs)} completed"}
    rows = np.array([done[t][1:5] for t in sorted(done)])
    bad = sum(1 for v in done.values() if v[0] != 0)
    skip = int(len(rows) * warmup_frac)
    lat = (rows[skip:, 3] - rows[skip:, 0]) * 1e3
    span = rows[:, 3].max() - rows[:, 0].min()
    return {
        "rate_hz": rate_hz, "mode": ["batched", "per_request", "unfused"][mode],
        "frames": "device" if on_device else "host",
        "requests": len(reqs), "failed": bad, "crops": crops,
        "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "mean_ms": round(float(lat.mean()), 3),
        "queue_ms_p50": round(float(np.percentile((rows[skip:, 1] - rows[skip:, 0]) * 1e3, 50)), 3),
        "throughput_req_s": round(len(reqs) / span, 1), "crops_per_s": round(crops / span, 1),
        "h2d_gb_s": round(in_bytes / span / 1e9, 2), "out_gb_s": round(out_bytes / span / 1e9, 2),
        "launches": int(st.launches), "crops_per_launch": round(st.crops_launched / max(1, st.launches), 1),
        "peak_mb": round(st.peak_bytes / 1e6, 1),
    }
