#!/usr/bin/env python3
"""Benchmark of the fused memory-bound chain on one MI355X.

Default workload (vertical-fusion depth sweep): one 3840x2160x3 uint8 frame
(seeded uniform bytes); chain = convert to fp32, then N alternating
multiply/add ops with seeded constants, written packed HWC fp32, for
N in {1, 4, 16, 64, 256}.  One step runs the fused chain once at every
depth (five launches).  Buffers rotate over 24 (frame, output) sets (600 MB
of frames, 3 GB in all), so a frame has left the 256 MB Infinity Cache
before it is read again and every launch reads its frame from HBM.  (With
four sets the frames stayed in that cache, since the nontemporal output
stores do not displace them, and the HBM-bound launches read 18.9 us
instead of 22.3 us.)

Printed JSON line:
  value        algorithmic bytes of the step (5 x 124,416,000 B) / step time
  roofline     the dominant kernel (the 256-op launch, the longest of a
               step) against its bound; its average duration comes from the
               HIP event pair each of its launches records inside the timed
               region as its kernel starts and ends (fk_run_timed; the only
               events recorded there)
  per_depth    every depth's average kernel time, GB/s, fraction of HBM peak,
               and the unfused one-kernel-per-op baseline with the speedup
  cpu_baseline the CPU oracle (single thread) on a band of rows of the same
               frame through the whole sweep, scaled to GB/s

Other workloads (--workload), for the design notes, not the headline line:
"hf" (batched uneven crops), "loop" (long Mul+Add chains through the loop
op on a batch of small images), "stats" (the reduction write), "sweeps"
(the paper's data-size, plain-read batch and data-type sweeps), "reads"
(nearest-neighbour and NV12 reads), "serve" (the serving loop), "costmodel"
(training and evaluating the launch-configuration model) and "copy" (a
plain device copy, the bandwidth reference).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# MI355X's published fp32 vector peak (packed fp32: two FMAs per lane and cycle)
FP32_PEAK_TFLOPS = 157.3
# The library's fp32 ceiling: its kernels are compiled without packed fp32
# instructions, so one FMA per lane and cycle: 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz x 2 flops
FP32_ISSUE_CEILING_TFLOPS = 78.6
# smallest HBM read request: a gather that touches one byte of a 32-byte
# sector moves the whole sector
SECTOR_BYTES = 32
DEPTHS = [1, 4, 16, 64, 256]
FRAME_HW = (2160, 3840)


def alu_roof(tflops):
    """Roofline record of an fp32-ALU-bound kernel: the fraction of the
    published peak, and of the library's non-packed issue ceiling beside it."""
    return {"bound": "alu", "achieved": round(tflops, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tflops / FP32_PEAK_TFLOPS, 4),
            "issue_ceiling": FP32_ISSUE_CEILING_TFLOPS,
            "frac_of_issue_ceiling": round(tflops / FP32_ISSUE_CEILING_TFLOPS, 4),
            "peak_note": "peak = published packed-fp32 rate; the kernels are built without packed fp32 "
                         "instructions, so issue_ceiling (one FMA per lane per cycle) is the rate they can reach"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def timeit(fn, reps=50, warm_s=0.0):
    """Mean ms per call over `reps` back-to-back calls of fn, bracketed by
    events on the current stream, after one call and a synchronisation.
    warm_s > 0 first runs that many seconds of back-to-back calls: right
    after an autotuning pass (short bursts, each followed by a
    synchronisation) a 50-call point reads up to twice its steady time,
    and 2 ms of calls settle it."""
    import torch
    t_end = time.perf_counter() + warm_s
    fn()
    while time.perf_counter() < t_end:
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


ROTATE_BYTES = 600 << 20  # frames a rotating measurement cycles through


def rotation_sets(frame_bytes):
    """How many copies of a frame a rotating measurement cycles through so
    that a frame has left the 256 MB Infinity Cache before it is read
    again."""
    return max(2, -(-ROTATE_BYTES // frame_bytes))


def rotating_ms(run, sets, reps=50, warm_s=0.0):
    """Mean ms per call of run(set) over `reps` back-to-back calls that cycle
    through `sets` (timeit's bracketing)."""
    turn = [0]

    def one():
        run(sets[turn[0] % len(sets)])
        turn[0] += 1
    return timeit(one, reps, warm_s)


def vf_sweep(args):
    import numpy as np
    import torch

    import datagen
    import paper_2508_07071_amd as fk

    dev = torch.device("cuda:0")
    H, W = FRAME_HW
    in_bytes = H * W * 3
    out_bytes = H * W * 3 * 4
    alg_bytes = in_bytes + out_bytes  # 124,416,000 B per launch, any depth
    R = args.rotate

    cfgs = {n: datagen.config1(n, seed=args.seed, frame_hw=FRAME_HW) for n in DEPTHS}
    frame_np = cfgs[DEPTHS[0]]["frames"][0]
    frames = [torch.from_numpy(frame_np).to(dev) for _ in range(R)]
    outs = [torch.empty((H, W, 3), dtype=torch.float32, device=dev) for _ in range(R)]
    item = datagen.whole_frame_item(frame_np)
    stream = fk.stream_handle()

    plans, items_by_set, tuned = {}, {}, {}
    for n in DEPTHS:
        ch = cfgs[n]["chain"]
        desc = fk.chain_desc(ch)
        opts = fk.plan_opts(strict=args.strict)
        h = fk.fk_plan_create(desc, R, opts)
        plans[n] = (h, desc)
        items_by_set[n] = [fk.make_items(ch, [frames[r]], [item], [outs[r]]) for r in range(R)]
        if args.autotune:
            # tuned as the step runs it: one frame per launch, frames read
            # from HBM (rotating sets).  fk_autotune would time all sets in
            # one batched launch, whose best configuration differs: 256 x 8
            # at N = 256 there, 111.7 us as a single launch against 97-100.
            times = []
            for c in fk.fk_autotune_space():
                fk.fk_plan_set_config(h, c)
                times.append(rotating_ms(lambda it: fk.fk_run(h, it, 1, stream), items_by_set[n], 40, 0.002))
            best = fk.fk_autotune_space()[min(range(len(times)), key=times.__getitem__)]
            fk.fk_plan_set_config(h, best)
            log(f"N={n} autotune (single launches, rotating sets) ms:",
                {f"{c.block_threads}x{c.coarsen}": round(t, 4) for c, t in zip(fk.fk_autotune_space(), times)})
        else:
            best = fk.fk_plan_get_config(h)
        tuned[n] = (best.block_threads, best.coarsen, fk.fk_plan_get_tier(h))
        log(f"N={n}: config {best.block_threads}x{best.coarsen} static={tuned[n][2]}")

    counter = [0]
    dom = DEPTHS[-1]  # the longest launch of a step (ALU-bound at 256 ops)

    def step(events=None, i=0, only=None):
        for n in DEPTHS:
            if only is not None and n != only:
                continue
            r = counter[0] % R
            counter[0] += 1
            timed = events is not None and (only is not None or n == dom)
            if timed:
                # the launch itself records the pair as its kernel starts and
                # ends (no separate event markers in the stream)
                fk.fk_run_timed(plans[n][0], items_by_set[n][r], 1, stream,
                                events[i][0].cuda_event, events[i][1].cuda_event)
            else:
                fk.fk_run(plans[n][0], items_by_set[n][r], 1, stream)

    def make_events(k):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]
        for a, b in ev:  # materialise the HIP events (outside any timed region)
            a.record()
            b.record()
        torch.cuda.synchronize()
        return ev

    # The baselines and the other depths' launch times are measured first,
    # outside the timed region.  Run before the warm-up, they also take the
    # GPU out of its first milliseconds of load, during which the ALU-bound
    # depth runs up to 12% slower while the clocks settle (measured: the
    # N = 256 launches of the first 50 steps average 106 us, of the next 50
    # 98 us, and 94.5-95 us from then on).
    # unfused baseline: one kernel per op
    unfused_ms = {}
    if not args.no_unfused:
        for n in DEPTHS:
            h = plans[n][0]
            it = items_by_set[n][0]
            nbytes = fk.fk_unfused_scratch_bytes(h, it, 1)
            scratch = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            reps = 3 if n <= 64 else 2
            fk.fk_run_unfused(h, items_by_set[n][1 % R], 1, scratch.data_ptr(), nbytes, stream)
            torch.cuda.synchronize()
            ts = []
            for i in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                fk.fk_run_unfused(h, items_by_set[n][i % R], 1, scratch.data_ptr(), nbytes, stream)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            unfused_ms[n] = float(np.median(ts))
            del scratch
        log("unfused ms", {n: round(v, 3) for n, v in unfused_ms.items()})

    kern_ms = {}
    # every other depth's launch time (its own launches back to back)
    for n in DEPTHS[:-1]:
        ev = make_events(args.steps)
        for i in range(args.steps):
            step(ev, i, only=n)
        torch.cuda.synchronize()
        kern_ms[n] = float(np.mean([a.elapsed_time(b) for a, b in ev]))

    for _ in range(args.warmup):
        step()
    # timing events are created up front: none is created inside the timed
    # loop, and only the dominant kernel's launches carry them
    dom_events = make_events(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(dom_events, i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    kern_ms[dom] = float(np.mean([a.elapsed_time(b) for a, b in dom_events]))
    log("kernel ms", {n: round(kern_ms[n], 4) for n in DEPTHS}, "step ms", round(ms_per_step, 4))

    per_depth = []
    for n in DEPTHS:
        gbps = alg_bytes / (kern_ms[n] * 1e-3) / 1e9
        flops = 2.0 * (n // 2) * in_bytes + (n % 2) * in_bytes  # n element-ops per element
        d = {"n_ops": n, "kernel_ms": round(kern_ms[n], 5), "gbps": round(gbps, 1),
             "hbm_frac": round(gbps / HBM_PEAK_GBPS, 4),
             "alu_frac": round(flops / (kern_ms[n] * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4),
             "alu_frac_of_issue_ceiling": round(flops / (kern_ms[n] * 1e-3) / 1e12 /
                                                FP32_ISSUE_CEILING_TFLOPS, 4),
             "launch_config": list(tuned[n][:2]), "compile_time_chain": bool(tuned[n][2])}
        if n in unfused_ms:
            ubytes = in_bytes + out_bytes + n * 2 * out_bytes  # every op reads+writes fp32
            ubytes -= out_bytes  # the first op reads u8 instead of fp32
            d["unfused_ms"] = round(unfused_ms[n], 4)
            d["unfused_gbps_alg"] = round(alg_bytes / (unfused_ms[n] * 1e-3) / 1e9, 1)
            d["unfused_moved_gb"] = round(ubytes / 1e9, 3)
            d["speedup_vs_unfused"] = round(unfused_ms[n] / kern_ms[n], 2)
        per_depth.append(d)

    n = dom
    flops = 2.0 * (n // 2) * in_bytes + (n % 2) * in_bytes
    alu_s = flops / (FP32_PEAK_TFLOPS * 1e12)
    hbm_s = alg_bytes / (HBM_PEAK_GBPS * 1e9)
    if alu_s > hbm_s:
        roof = alu_roof(flops / (kern_ms[n] * 1e-3) / 1e12)
    else:
        achieved = alg_bytes / (kern_ms[n] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4)}
    roof["kernel"] = f"fused cvt+{n} mul/add ops, 3840x2160x3 u8 -> packed fp32"
    roof["kernel_ms"] = round(kern_ms[n], 5)
    roof["traffic"] = measured_traffic(n)

    value = len(DEPTHS) * alg_bytes / (ms_per_step * 1e-3) / 1e9
    res = {
        "metric": "fused-chain GB/s (fraction of HBM peak) vs unfused per-op",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "hbm_frac": round(value / HBM_PEAK_GBPS, 4),
        "config": {"workload": "vf_depth_sweep: 3840x2160x3 u8 frame, cvt + N alternating mul/add, "
                               "N in {1,4,16,64,256}, packed HWC fp32 out",
                   "frame": "3840x2160x3 u8", "depths": DEPTHS, "bytes_per_launch": alg_bytes,
                   "rotation_sets": R, "fp_mode": "strict" if args.strict else "contracted",
                   "seed": args.seed},
        "roofline": roof,
        "hbm_bound_depths": {
            "n_ops": [d["n_ops"] for d in per_depth if d["n_ops"] <= 16],
            "gbps": [d["gbps"] for d in per_depth if d["n_ops"] <= 16],
            "hbm_frac": [d["hbm_frac"] for d in per_depth if d["n_ops"] <= 16]},
        "per_depth": per_depth,
    }
    if unfused_ms:
        tot_f = sum(kern_ms.values())
        tot_u = sum(unfused_ms.values())
        res["unfused"] = {"ms_per_step": round(tot_u, 4),
                          "value": round(len(DEPTHS) * alg_bytes / (tot_u * 1e-3) / 1e9, 1),
                          "unit": "GB/s", "speedup": round(tot_u / tot_f, 2)}
    for n in DEPTHS:
        fk.fk_plan_destroy(plans[n][0])
    return res, cfgs


def tap_bytes(item, channels=3, pitch=None, sector=SECTOR_BYTES):
    """Bytes the bilinear crop+resize read of one item must fetch, as
    (distinct tapped pixels x C, the 32-byte sectors holding those bytes x
    32), for a u8 frame with a 32-byte aligned base and the given row pitch.
    The taps follow the read's half-pixel rule: source coordinate
    (o + 0.5) * (w / ow) - 0.5, clamped at 0; taps at its floor and the next
    pixel, clamped to the ROI."""
    import numpy as np

    def taps(n_out, n_in):
        scale = np.float32(np.float32(n_in) / np.float32(n_out))
        # (o + 0.5) * scale is exact in fp64, so one rounding to fp32 gives
        # the fused multiply-add of the read
        s = ((np.arange(n_out) + 0.5) * np.float64(scale) - 0.5).astype(np.float32)
        lo = np.minimum(np.floor(np.maximum(s, 0)).astype(np.int64), n_in - 1)
        return np.unique(np.concatenate([lo, np.minimum(lo + 1, n_in - 1)]))

    X = taps(item["out_w"], item["w"])
    Y = taps(item["out_h"], item["h"])
    pitch = pitch or 3840 * channels
    offs = ((item["x"] + X)[:, None] * channels + np.arange(channels)[None, :]).ravel()
    secs = np.unique(((item["y"] + Y)[:, None] * pitch + offs[None, :]) // sector)
    return len(X) * len(Y) * channels, len(secs) * sector


def hot_chain_rows(args):
    """The hot chain (crop + bilinear resize -> BGR->RGB -> fp32 -> *1/255 ->
    -mean -> /std -> planar split) at the sizes of config 0 (one 512x512 crop
    of a 1920x1080 frame -> 224x224) and config 2 (B uneven crops of a
    3840x2160 frame -> 64x128 into one [B][3][128][64] tensor, B in
    {1, 8, 50, 256}), plus a point beyond the configs: 4096 crops over 24
    distinct 3840x2160 frames (597 MB of frames).

    Per row: the autotuned launch config; the kernel's device time from the
    events its own launch records (mean over reps), cold (each launch
    preceded by a 512 MB read of another buffer, which evicts the frame from
    the 256 MB Infinity Cache) and warm (back to back on one frame); the
    time per fk_run call back to back (host launch included), the same with
    graph replay, one fused launch per crop, and the unfused baseline;
    algorithmic bytes (distinct tapped bytes + outputs), the 32-byte sectors
    those taps fall in + outputs (what HBM must move), and GB/s and HBM
    fractions of both over the cold kernel time."""
    import numpy as np
    import torch

    import datagen
    import paper_2508_07071_amd as fk

    dev = torch.device("cuda:0")
    stream = fk.stream_handle()
    gather = fk.FK_GATHER_LDS if args.gather == "lds" else fk.FK_GATHER_DIRECT
    flush_buf = torch.ones(512 << 20, dtype=torch.uint8, device=dev)

    def flush():
        flush_buf.max()  # reads 512 MB, writes one byte

    def events(k):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]
        for a, b in ev:
            a.record()
            b.record()
        torch.cuda.synchronize()
        return ev

    def kernel_us(plan, arrs, n, reps, flushed=False):
        """Mean device time of `reps` launches that record their own start
        and end events; launch i takes argument set i % len(arrs)."""
        ev = events(reps)
        fk.fk_run(plan, arrs[-1], n, stream)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(ev):
            if flushed:
                flush()
            fk.fk_run_timed(plan, arrs[i % len(arrs)], n, stream, a.cuda_event, b.cuda_event)
        torch.cuda.synchronize()
        return 1e3 * float(np.mean([a.elapsed_time(b) for a, b in ev]))

    def row(name, chain, frames_np, items, out_shape, reps, baselines=True, beyond=False):
        B = len(items)
        # copies of the frame set (and outputs), at least 600 MB of frames in
        # all, so that launches rotating over them read HBM, not the cache
        set_bytes = sum(f.nbytes for f in frames_np)
        R = max(1, min(128, -(-600_000_000 // set_bytes)))
        arrs, keep = [], []
        for _ in range(R):
            frames = [torch.from_numpy(f).to(dev) for f in frames_np]
            out = torch.empty(out_shape, dtype=torch.float32, device=dev)
            outs = [out[b] for b in range(B)] if len(out_shape) == 4 else [out]
            arrs.append(fk.make_items(chain, frames, items, outs))
            keep.append((frames, out))
        frames, out = keep[0]
        outs = [out[b] for b in range(B)] if len(out_shape) == 4 else [out]
        arr = arrs[0]
        desc = fk.chain_desc(chain)
        C = chain["read"]["channels"]
        tb = np.array([tap_bytes(it, C, frames_np[it["frame"]].shape[1] * C) for it in items]).sum(0)
        out_b = sum(it["out_w"] * it["out_h"] * C * 4 for it in items)
        r = {"case": name, "batch": B, "gather": args.gather, "alg_bytes": int(tb[0]) + out_b,
             "sector_bytes": int(tb[1]) + out_b, "rotation_sets": R,
             "rotation_mb": round(R * set_bytes / 1e6, 1)}
        if beyond:
            r["beyond_configs"] = True
        h = fk.fk_plan_create(desc, B, fk.plan_opts(gather=gather))
        if name in fixed:
            best = fk.fk_launch_config(*fixed[name])
            fk.fk_plan_set_config(h, best)
        else:
            best, _ = fk.fk_autotune(h, arr, B, 10)
        r["autotuned"] = [best.block_threads, best.coarsen]
        r["kernel_us"] = round(kernel_us(h, arrs, B, reps), 2)
        for key, b in (("gbps", r["alg_bytes"]), ("gbps_sector", r["sector_bytes"])):
            r[key] = round(b / (r["kernel_us"] * 1e-6) / 1e9, 1)
        r["hbm_frac"] = round(r["gbps"] / HBM_PEAK_GBPS, 4)
        r["hbm_frac_sector"] = round(r["gbps_sector"] / HBM_PEAK_GBPS, 4)
        if args.hot_profile:
            fk.fk_plan_destroy(h)
            log(r)
            return r
        r["kernel_us_flushed"] = round(kernel_us(h, arrs[:1], B, reps, flushed=True), 2)
        r["kernel_us_warm"] = round(kernel_us(h, arrs[:1], B, reps), 2)
        r["call_us"] = round(1e3 * timeit(lambda: fk.fk_run(h, arr, B, stream), reps, warm_s=2e-3), 2)
        if baselines:
            singles = [fk.make_items(chain, frames, [it], [outs[b]]) for b, it in enumerate(items)]
            r["per_crop_us"] = round(1e3 * timeit(lambda: [fk.fk_run(h, s1, 1, stream) for s1 in singles],
                                                  max(2, reps // 20)), 2)
            nbytes = fk.fk_unfused_scratch_bytes(h, arr, B)
            scratch = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            r["unfused_us"] = round(1e3 * timeit(
                lambda: fk.fk_run_unfused(h, arr, B, scratch.data_ptr(), nbytes, stream),
                max(2, reps // 40)), 2)
            del scratch
            r["speedup_vs_unfused"] = round(r["unfused_us"] / r["call_us"], 2)
            r["speedup_vs_per_crop"] = round(r["per_crop_us"] / r["call_us"], 2)
        fk.fk_plan_destroy(h)
        if baselines:
            hg = fk.fk_plan_create(desc, B, fk.plan_opts(use_graph=True, gather=gather))
            fk.fk_plan_set_config(hg, best)
            r["graph_call_us"] = round(1e3 * timeit(lambda: fk.fk_run(hg, arr, B, stream), reps,
                                                    warm_s=2e-3), 2)
            fk.fk_plan_destroy(hg)
            # the caller's own capture of 10 runs (kernel-argument batches
            # are captured as their launches): per-run time of the replays
            hc = fk.fk_plan_create(desc, B, fk.plan_opts(gather=gather))
            fk.fk_plan_set_config(hc, best)
            cs = torch.cuda.Stream()
            graph = torch.cuda.CUDAGraph()
            try:
                with torch.cuda.graph(graph, stream=cs):
                    for _ in range(10):
                        fk.fk_run(hc, arr, B, fk.stream_handle(cs))
                r["graph_10_runs_us_per_run"] = round(
                    1e3 * timeit(graph.replay, max(2, reps // 10), warm_s=2e-3) / 10, 2)
            except fk.FKError:
                r["graph_10_runs_us_per_run"] = None  # a table batch: not capturable
            del graph
            fk.fk_plan_destroy(hc)
        log(r)
        return r

    # launch configs from an earlier run's JSON line (profiler runs), by case
    fixed = {}
    if args.hot_configs:
        with open(args.hot_configs) as f:
            prev = json.loads([ln for ln in f if ln.strip().startswith("{")][-1])
        fixed = {r["case"]: tuple(r["autotuned"]) for r in prev.get("per_config", [])}

    rows = []
    c0 = datagen.config0(seed=args.seed)
    reps = args.hot_reps
    rows.append(row("config0: 512x512 crop of 1920x1080 -> 224x224", c0["chain"], c0["frames"],
                    c0["items"], (3, 224, 224), reps))
    for B in (1, 8, 50, 256):
        c2 = datagen.config2(B, seed=args.seed)
        rows.append(row(f"config2: B={B} crops of 3840x2160 -> 64x128", c2["chain"], c2["frames"],
                        c2["items"], (B, 3, 128, 64), reps))
    g = datagen.rng(args.seed + 77)
    n_frames = 24
    frames = [datagen.frame(g, 2160, 3840, 3) for _ in range(n_frames)]
    items = []
    for f in range(n_frames):
        items += datagen.random_crops(g, 4096 // n_frames + (f < 4096 % n_frames), 3840, 2160, frame_index=f)
    rows.append(row("4096 crops over 24 distinct 3840x2160 frames -> 64x128", datagen.normalize_chain(64, 128),
                    frames, items, (len(items), 3, 128, 64), max(5, reps // 4), baselines=False,
                    beyond=True))
    return rows


def serving_row(args, rate=1000.0, n=2000, device_rate=20000.0):
    """One serving point of config 4 (Poisson arrivals at `rate` req/s, n
    requests, host frames copied per request) and one beyond it (frames
    already on the device, at `device_rate`), each with continuous batching
    and with per-request fused launches; 64 GB arena and budget."""
    import torch

    import paper_2508_07071_amd as fk
    from paper_2508_07071_amd import serve

    arena = torch.empty(64 << 30, dtype=torch.uint8, device=torch.device("cuda:0"))
    out = {}
    for frames, r_hz in (("host", rate), ("device", device_rate)):
        pool = serve.make_pool(8, seed=args.seed, device=frames == "device")
        for mode, name in ((fk.FK_SERVER_BATCHED, "batched"), (fk.FK_SERVER_PER_REQUEST, "per_request")):
            r = serve.run(r_hz, n, mode, pool, arena, seed=args.seed, budget_bytes=64 << 30)
            log(r)
            out[name if frames == "host" else f"device_frames_{name}"] = r
        del pool
    del arena
    return out


def measured_traffic(n_ops):
    """HBM bytes per launch of the depth-n kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary (copy-kernel scaled), or None
    when the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "vf_depth_sweep_4k_traffic.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for f in ("fk_device.hpp", "fk_internal.hpp", "fk_static.hip"):
            h.update(open(os.path.join(ROOT, "paper_2508_07071_amd", "csrc", f), "rb").read())
        if h.hexdigest()[:16] != rec["source_digest"]:
            return None
        return rec["traffic_bytes_per_launch"].get(str(n_ops))
    except (OSError, ValueError, KeyError):
        return None


def _oracle_band(job):
    """Worker of the all-core CPU baseline: the oracle on one band of rows
    through every depth (a separate process, no GPU)."""
    import numpy as np

    import datagen
    import oracle

    band, chains = job
    band = np.ascontiguousarray(band)
    item = datagen.whole_frame_item(band)
    t0 = time.perf_counter()
    for chain in chains:
        oracle.run_chain(chain, [band], [item], shadow=False)
    return time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_vf(args, cfgs):
    """The oracle as it stands (per-op fp32 passes over the whole image, no
    fp64 shadow) on the host: one thread on a band of rows, and every core
    of this process's affinity set (at most 16 worker processes) on the
    whole frame split into bands; the oracle's time for config 0 and for
    config 2 at B = 256, single-threaded."""
    import multiprocessing as mp

    import numpy as np

    import datagen
    import oracle

    frame = cfgs[DEPTHS[0]]["frames"][0]
    H = frame.shape[0]
    rows = min(args.cpu_rows, H)
    band = np.ascontiguousarray(frame[:rows])
    item = datagen.whole_frame_item(band)
    t0 = time.perf_counter()
    for n in DEPTHS:
        oracle.run_chain(cfgs[n]["chain"], [band], [item], shadow=False)
    dt1 = time.perf_counter() - t0
    single = {"value": round(len(DEPTHS) * band.size * 5 / dt1 / 1e9, 4), "unit": "GB/s", "cores": 1,
              "sample": f"rows 0..{rows - 1} of the 3840x2160 frame through all five depths, {dt1:.1f} s"}

    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    chains = [cfgs[n]["chain"] for n in DEPTHS]
    cuts = np.linspace(0, H, workers + 1).astype(int)
    bands = [(frame[a:b], chains) for a, b in zip(cuts[:-1], cuts[1:])]
    with mp.get_context("spawn").Pool(workers) as pool:
        pool.map(_oracle_band, [(frame[:8], chains)] * workers)  # start and import in every worker
        t0 = time.perf_counter()
        per = pool.map(_oracle_band, bands)
        dtn = time.perf_counter() - t0
    res = {"value": round(len(DEPTHS) * frame.size * 5 / dtn / 1e9, 4), "unit": "GB/s", "cores": workers,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"the whole 3840x2160 frame in {workers} row bands, one worker process each, "
                     f"through all five depths: {dtn:.1f} s wall ({sum(per):.1f} s of worker time); "
                     f"unfused per-op fp32 passes, no fp64 shadow",
           "single_thread": single}

    c0 = datagen.config0(seed=args.seed)
    t0 = time.perf_counter()
    oracle.run_chain(c0["chain"], c0["frames"], c0["items"], shadow=False)
    res["config0_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    c2 = datagen.config2(256, seed=args.seed)
    t0 = time.perf_counter()
    oracle.run_chain(c2["chain"], c2["frames"], c2["items"], shadow=False)
    res["config2_b256_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    return res


def hf_workload(args):
    """Batched uneven crops (config 2 sizes): fused single launch vs per-crop
    launches vs unfused per-op per-crop, eager and hipGraph.  Runs are back
    to back on one frame, which stays in the Infinity Cache; the default
    run's per_config rows time the same batches with the frames read from
    HBM."""
    import numpy as np
    import torch

    import datagen
    import paper_2508_07071_amd as fk

    dev = torch.device("cuda:0")
    stream = fk.stream_handle()
    rows = []
    for B in (1, 8, 50, 256):
        cfg = datagen.config2(B, seed=args.seed)
        ch = cfg["chain"]
        frame = torch.from_numpy(cfg["frames"][0]).to(dev)
        out = torch.empty((B, 3, 128, 64), dtype=torch.float32, device=dev)
        arr = fk.make_items(ch, [frame], cfg["items"], [out[b] for b in range(B)])
        desc = fk.chain_desc(ch)
        # bytes the read must move: the distinct tapped pixels (taps), or the
        # tapped rows' full ROI span (rows: what line-granular reads fetch
        # when taps are closer than a cache line, as in downscales)
        taps = sum(min(it["w"], 2 * 64) * min(it["h"], 2 * 128) * 3 for it in cfg["items"])
        rows_b = sum(it["w"] * min(it["h"], 2 * 128) * 3 for it in cfg["items"])
        alg = taps + B * 3 * 128 * 64 * 4
        alg_rows = rows_b + B * 3 * 128 * 64 * 4


        res = {"batch": B, "alg_bytes": alg, "alg_bytes_rows": alg_rows}
        for graph in (False, True):
            h = fk.fk_plan_create(desc, B, fk.plan_opts(use_graph=graph))
            if not graph:
                best, _ = fk.fk_autotune(h, arr, B, 10)
                res["autotuned"] = [best.block_threads, best.coarsen]
                cfg_best = best
            else:
                fk.fk_plan_set_config(h, cfg_best)
            ms = timeit(lambda: fk.fk_run(h, arr, B, stream), warm_s=2e-3)
            res["graph_ms" if graph else "fused_ms"] = round(ms, 4)
            if not graph:
                singles = [fk.make_items(ch, [frame], [it], [out[b]]) for b, it in enumerate(cfg["items"])]
                res["per_crop_ms"] = round(timeit(lambda: [fk.fk_run(h, s, 1, stream) for s in singles], 10), 4)
                nbytes = fk.fk_unfused_scratch_bytes(h, arr, B)
                scratch = torch.empty(nbytes, dtype=torch.uint8, device=dev)
                res["unfused_ms"] = round(timeit(lambda: fk.fk_run_unfused(h, arr, B, scratch.data_ptr(), nbytes, stream), 5), 4)
            fk.fk_plan_destroy(h)
        res["fused_gbps"] = round(alg / (res["fused_ms"] * 1e-3) / 1e9, 1)
        res["fused_gbps_rows"] = round(alg_rows / (res["fused_ms"] * 1e-3) / 1e9, 1)
        res["speedup_vs_per_crop"] = round(res["per_crop_ms"] / res["fused_ms"], 2)
        res["speedup_vs_unfused"] = round(res["unfused_ms"] / res["fused_ms"], 2)
        log(res)
        rows.append(res)
    rows.append(hf_large(args))
    out = {"workload": "hf_batch_sweep (config 2 sizes)", "rows": rows}
    if not args.no_cpu_baseline:
        import datagen
        import oracle
        cfg = datagen.config2(50, seed=args.seed)
        t0 = time.perf_counter()
        oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"], shadow=True)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(50 / dt, 1), "unit": "crops/s", "cores": 1, "kind": "oracle",
                               "sample": f"the B=50 batch (64x128 outputs), {dt:.2f} s single-threaded"}
    return out


def hf_large(args, n_frames=8, per_frame=512):
    """Beyond the configs: 4096 crops spread over 8 distinct 3840x2160 frames
    (200 MB of frames, 400 MB of outputs), so the resize gather reads HBM,
    not the Infinity Cache.  Algorithmic bytes = distinct tapped rows x
    distinct tapped columns x 3 + outputs."""
    import numpy as np
    import torch

    import datagen
    import paper_2508_07071_amd as fk

    dev = torch.device("cuda:0")
    stream = fk.stream_handle()
    g = datagen.rng(args.seed + 77)
    frames = [torch.from_numpy(datagen.frame(g, 2160, 3840, 3)).to(dev) for _ in range(n_frames)]
    items = []
    for f in range(n_frames):
        items += datagen.random_crops(g, per_frame, 3840, 2160, frame_index=f)
    B = len(items)
    chain = datagen.normalize_chain(64, 128)
    out = torch.empty((B, 3, 128, 64), dtype=torch.float32, device=dev)
    arr = fk.make_items(chain, frames, items, [out[b] for b in range(B)])
    taps = sum(min(it["w"], 128) * min(it["h"], 256) * 3 for it in items)
    alg = taps + B * 3 * 128 * 64 * 4
    alg_rows = sum(it["w"] * min(it["h"], 256) * 3 for it in items) + B * 3 * 128 * 64 * 4
    h = fk.fk_plan_create(fk.chain_desc(chain), B, fk.plan_opts())
    best, times = fk.fk_autotune(h, arr, B, 5)
    ms = min(times)
    fk.fk_plan_destroy(h)
    res = {"batch": B, "frames": n_frames, "beyond_configs": True, "alg_bytes": alg,
           "alg_bytes_rows": alg_rows, "fused_gbps_rows": round(alg_rows / (ms * 1e-3) / 1e9, 1),
           "autotuned": [best.block_threads, best.coarsen], "fused_ms": round(ms, 4),
           "fused_gbps": round(alg / (ms * 1e-3) / 1e9, 1),
           "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
    log(res)
    return res


LOOP_PAIRS = [1, 10, 100, 1000, 5000, 10000]


def loop_workload(args):
    """Vertical plus horizontal fusion with long chains (Section VI-D): a
    batch of 50 uint8 images of 60x120 held in one tensor; convert to fp32,
    then P Mul+Add pairs through the loop op, packed fp32 out, for P in
    LOOP_PAIRS.  For each P: the fused batched launch (the compile-time loop
    chain), the same fused chain launched once per image (vertical fusion
    only), and the unfused baseline (one kernel per op per image).
    Algorithmic work per launch: 2 P flops per element (a multiply and an
    add), 50 x 7200 elements; bytes 7200 x (1 + 4) per image."""
    import numpy as np
    import torch

    import datagen
    import paper_2508_07071_amd as fk

    dev = torch.device("cuda:0")
    stream = fk.stream_handle()
    B, (h, w) = 50, (120, 60)
    elems = B * h * w
    alg_bytes = elems * (1 + 4)


    rows = []
    for P in LOOP_PAIRS:
        cfg = datagen.loop_batch(P, seed=args.seed)
        ch = cfg["chain"]
        frame = torch.from_numpy(cfg["frames"][0]).to(dev)
        out = torch.empty((B, h, w, 1), dtype=torch.float32, device=dev)
        arr = fk.make_items(ch, [frame], cfg["items"], [out[b] for b in range(B)])
        plan = fk.fk_plan_create(fk.chain_desc(ch), B, fk.plan_opts(strict=args.strict))
        c = fk.fk_plan_get_config(plan)
        flops = 2.0 * P * elems
        r = {"pairs": P, "compile_time_chain": bool(fk.fk_plan_get_tier(plan)),
             "launch_config": [c.block_threads, c.coarsen]}
        r["fused_ms"] = round(timeit(lambda: fk.fk_run(plan, arr, B, stream), 100), 5)
        singles = [fk.make_items(ch, [frame], [it], [out[b]]) for b, it in enumerate(cfg["items"])]
        r["per_image_ms"] = round(timeit(lambda: [fk.fk_run(plan, s1, 1, stream) for s1 in singles],
                                         20 if P <= 1000 else 3), 5)
        if not args.no_unfused:
            nbytes = fk.fk_unfused_scratch_bytes(plan, arr, B)
            scratch = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
            reps = 3 if P <= 100 else 1
            r["unfused_ms"] = round(timeit(lambda: fk.fk_run_unfused(plan, arr, B, scratch.data_ptr(), nbytes,
                                                                   stream), reps), 4)
            r["unfused_launches"] = B * (1 + 2 * P)
            r["speedup_vs_unfused"] = round(r["unfused_ms"] / r["fused_ms"], 1)
            del scratch
        r["tflops"] = round(flops / (r["fused_ms"] * 1e-3) / 1e12, 3)
        r["alu_frac"] = round(r["tflops"] / FP32_PEAK_TFLOPS, 4)
        r["alu_frac_of_issue_ceiling"] = round(r["tflops"] / FP32_ISSUE_CEILING_TFLOPS, 4)
        r["gbps"] = round(alg_bytes / (r["fused_ms"] * 1e-3) / 1e9, 1)
        r["speedup_hf_vs_per_image"] = round(r["per_image_ms"] / r["fused_ms"], 2)
        fk.fk_plan_destroy(plan)
        log(r)
        rows.append(r)
    # beyond the paper's batch: 1000 images, so that the 1.8 M work units
    # fill every SIMD many times over (at 50 images, 1,406 waves on 1,024
    # SIMDs leave the last wave round 37% full)
    big_b, big_p = 1000, 1000
    cfg = datagen.loop_batch(big_p, seed=args.seed, batch=big_b)
    frame = torch.from_numpy(cfg["frames"][0]).to(dev)
    out = torch.empty((big_b, h, w, 1), dtype=torch.float32, device=dev)
    arr = fk.make_items(cfg["chain"], [frame], cfg["items"], [out[b] for b in range(big_b)])
    plan = fk.fk_plan_create(fk.chain_desc(cfg["chain"]), big_b, fk.plan_opts(strict=args.strict))
    ms = timeit(lambda: fk.fk_run(plan, arr, big_b, stream), 20)
    fk.fk_plan_destroy(plan)
    tf = 2.0 * big_p * big_b * h * w / (ms * 1e-3) / 1e12
    big = {"pairs": big_p, "batch": big_b, "beyond_configs": True, "fused_ms": round(ms, 5),
           "tflops": round(tf, 3), "alu_frac": round(tf / FP32_PEAK_TFLOPS, 4),
           "alu_frac_of_issue_ceiling": round(tf / FP32_ISSUE_CEILING_TFLOPS, 4)}
    log(big)
    top = rows[-1]
    tot_flops = sum(2.0 * r["pairs"] * elems for r in rows)
    tot_ms = sum(r["fused_ms"] for r in rows)
    res = {"metric": "loop-chain fused TFLOP/s (2 flops per Mul+Add pair and element)",
           "value": round(tot_flops / (tot_ms * 1e-3) / 1e12, 3), "unit": "TFLOP/s", "n_gpus": 1,
           "higher_is_better": True, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "vf_hf_loop: 50 x 60x120 u8 images, cvt + P (mul, add) pairs via the loop op, "
                                  "packed fp32", "pairs": LOOP_PAIRS, "batch": B,
                      "fp_mode": "strict" if args.strict else "contracted", "seed": args.seed},
           "roofline": {**alu_roof(top["tflops"]), "traffic": None,
                        "kernel": f"fused loop chain, {top['pairs']} pairs, 50 x 60x120 u8 -> packed fp32",
                        "kernel_ms": top["fused_ms"]},
           "rows": rows, "large_batch": big}
    if not args.no_cpu_baseline:
        import oracle
        P, nimg = 10000, 4
        cfg = datagen.loop_batch(P, seed=args.seed)
        t0 = time.perf_counter()
        oracle.run_chain(cfg["chain"], cfg["frames"], cfg["items"][:nimg], shadow=True)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(2.0 * P * nimg * h * w / dt / 1e12, 6), "unit": "TFLOP/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"{nimg} of the 50 images at {P} pairs, {dt:.2f} s single-threaded"}
    return res


def stats_workload(args):
    """The stats write (Section IV-C's reduction pattern: min, max, sum and
    mean per channel from one read).  Workload: 16 distinct 3840x2160x3 u8
    frames (398 MB), cvt then the stats write, one item per frame; runs
    alternate between two such sets (796 MB), so the frames come from HBM,
    not the 256 MB Infinity Cache.  Compared with: the fused transform writing the fp32
    image followed by four torch reductions (amin, amax, sum, mean) over it,
    and the unfused baseline (one kernel per op, then one reduction pass per
    statistic).  Algorithmic bytes = the frames read once (the 16 x 3 x 4
    doubles written are negligible)."""
    import numpy as np
    import torch

    import datagen
    import paper_2508_07071_amd as fk

    dev = torch.device("cuda:0")
    stream = fk.stream_handle()
    F, (H, W) = 16, FRAME_HW
    g = datagen.rng(args.seed)
    frames = [torch.from_numpy(datagen.frame(g, H, W, 3)).to(dev) for _ in range(F)]
    chain = {"read": {"kind": "plain", "dtype": "u8", "channels": 3, "out_w": 0, "out_h": 0},
             "ops": [{"kind": "cvt", "k": []}], "write": {"dtype": "f64", "layout": "stats"}}
    items = [{"frame": f, "x": 0, "y": 0, "w": W, "h": H, "out_w": W, "out_h": H} for f in range(F)]
    stats = torch.empty((F, 3, 4), dtype=torch.float64, device=dev)
    arr = fk.make_items(chain, frames, items, [stats[f] for f in range(F)])
    # a second set of frames (copies) for the timed runs to alternate with
    frames2 = [f.clone() for f in frames]
    arr2 = fk.make_items(chain, frames2, items, [stats[f] for f in range(F)])
    sets = [arr, arr2]
    turn = [0]

    def next_set():
        turn[0] += 1
        return sets[turn[0] % 2]
    alg = F * H * W * 3


    plan = fk.fk_plan_create(fk.chain_desc(chain), F, fk.plan_opts())
    res = {"frames": F, "alg_bytes": alg}
    if args.autotune:
        best, _ = fk.fk_autotune(plan, arr, F, 5)
        res["autotuned"] = [best.block_threads, best.coarsen]
    c = fk.fk_plan_get_config(plan)
    res["launch_config"] = [c.block_threads, c.coarsen]
    res["fused_ms"] = round(timeit(lambda: fk.fk_run(plan, next_set(), F, stream), 50, warm_s=2e-3), 5)
    res["fused_gbps"] = round(alg / (res["fused_ms"] * 1e-3) / 1e9, 1)
    res["hbm_frac"] = round(res["fused_gbps"] / HBM_PEAK_GBPS, 4)
    # fused transform to fp32, then four library reductions over the image
    img_chain = dict(chain, write={"dtype": "f32", "layout": "packed"})
    img = torch.empty((F, H, W, 3), dtype=torch.float32, device=dev)
    iplan = fk.fk_plan_create(fk.chain_desc(img_chain), F, fk.plan_opts())
    iarr = fk.make_items(img_chain, frames, items, [img[f] for f in range(F)])

    def transform_then_reduce():
        fk.fk_run(iplan, iarr, F, stream)
        v = img.view(F, -1, 3)
        return torch.amin(v, 1), torch.amax(v, 1), torch.sum(v, 1, dtype=torch.float64), torch.mean(v, 1)
    res["transform_then_torch_ms"] = round(timeit(transform_then_reduce, 10), 4)
    fk.fk_plan_destroy(iplan)
    del img
    if not args.no_unfused:
        nbytes = fk.fk_unfused_scratch_bytes(plan, arr, F)
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        res["unfused_ms"] = round(timeit(lambda: fk.fk_run_unfused(plan, arr, F, scratch.data_ptr(), nbytes,
                                                                 stream), 3), 4)
        res["speedup_vs_unfused"] = round(res["unfused_ms"] / res["fused_ms"], 1)
        del scratch
    res["speedup_vs_transform_then_torch"] = round(res["transform_then_torch_ms"] / res["fused_ms"], 1)
    fk.fk_plan_destroy(plan)
    log(res)
    out = {"metric": "stats-write GB/s (min, max, sum, mean per channel from one read)",
           "value": res["fused_gbps"], "unit": "GB/s", "n_gpus": 1, "higher_is_better": True,
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "stats: 16 x 3840x2160x3 u8 frames, cvt, per-channel min/max/sum/mean",
                      "seed": args.seed},
           "roofline": {"bound": "hbm", "achieved": res["fused_gbps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                        "frac": res["hbm_frac"], "traffic": None,
                        "kernel": "k_stats plain u8x3, 16 frames per launch", "kernel_ms": res["fused_ms"]},
           "result": res}
    if not args.no_cpu_baseline:
        import oracle
        fr = datagen.frame(datagen.rng(args.seed), H // 8, W, 3)
        t0 = time.perf_counter()
        oracle.run_chain(chain, [fr], [datagen.whole_frame_item(fr)])
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(fr.nbytes / dt / 1e9, 3), "unit": "GB/s", "cores": 1,
                               "kind": "oracle", "sample": f"one 3840x270x3 band, {dt:.2f} s single-threaded"}
    return out


DATA_SIZES = [100, 1000, 10000, 100000, 282370, 1000000, 4000000, 9032740, 16654030]
HF_PLAIN_BATCHES = [1, 10, 50, 100, 300, 600, 1191]
IPO_SIZES = [1, 5, 10, 25, 50, 100, 250, 500]
DTYPE_PAIRS = [("u8", "f32"), ("u8", "f16"), ("f16", "f32"), ("f16", "f16"), ("f32", "f32"), ("f32", "f16"),
               ("f32", "f64"), ("f64", "f64")]
# fp32 vs fp64 arithmetic on a whole frame: one 3840x2160 single-channel fp32
# frame, cvt then N alternating mul/add through the run-time op list
PRECISION_DEPTHS = [4, 64, 256]


def sweeps_workload(args):
    """The paper's parameter sweeps on this library (Sections VI-C, VI-E,
    VI-G, VI-I), fused vs the unfused one-kernel-per-op baseline:
      data_size: 1-D fp32 arrays of N values (rows of 4096 above 4096), 100
                 Mul+Add pairs through the loop op, no batch;
      hf_plain:  B single-channel 60x120 u8 images, Read -> Cast -> Mul ->
                 Sub -> Div -> Write, one batched launch vs one launch per
                 image vs unfused (default configuration), the batch
                 through the device run table (one output tensor per item),
                 and the autotuner's own time for its choice and for the
                 default;
      dtypes:    the same chain at B = 50 for eight input -> output types,
                 two of them (f32 -> f64, f64 -> f64) computing in fp64;
      precision: cvt + N mul/add (N in 4, 64, 256) over one 3840x2160 fp32
                 frame, computed in fp32 and in fp64 (timed over rotating
                 copies of the frame, read from HBM);
      instructions_per_op: 500 multiplications as ops of M instructions
                 over 66,355,200 fp32 values, fused vs one kernel per op."""
    import numpy as np
    import torch

    import datagen
    import paper_2508_07071_amd as fk

    dev = torch.device("cuda:0")
    stream = fk.stream_handle()


    def setup(cfg):
        # one output tensor for the batch (equal item sizes), one view per
        # item: a constant output stride, as a batched consumer would use
        ch = cfg["chain"]
        frame = torch.from_numpy(cfg["frames"][0]).to(dev)
        shape = fk.out_shape(ch, cfg["items"][0])
        assert all(fk.out_shape(ch, it) == shape for it in cfg["items"])
        batch_out = torch.empty((len(cfg["items"]),) + tuple(shape), dtype=fk.TORCH_DTYPE[ch["write"]["dtype"]],
                                device=dev)
        outs = [batch_out[b] for b in range(len(cfg["items"]))]
        arr = fk.make_items(ch, [frame], cfg["items"], outs)
        plan = fk.fk_plan_create(fk.chain_desc(ch), len(cfg["items"]), fk.plan_opts())
        return ch, frame, outs, arr, plan

    def unfused_ms(plan, arr, n, reps):
        nbytes = fk.fk_unfused_scratch_bytes(plan, arr, n)
        scratch = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        return timeit(lambda: fk.fk_run_unfused(plan, arr, n, scratch.data_ptr(), nbytes, stream), reps)

    data_size = []
    for n in DATA_SIZES:
        cfg = datagen.data_size_case(n, seed=args.seed)
        ch, frame, outs, arr, plan = setup(cfg)
        r = {"n": int(cfg["frames"][0].size), "compile_time_chain": bool(fk.fk_plan_get_tier(plan))}
        r["fused_ms"] = round(timeit(lambda: fk.fk_run(plan, arr, 1, stream), 50), 5)
        if not args.no_unfused:
            r["unfused_ms"] = round(unfused_ms(plan, arr, 1, 3), 4)
            r["speedup"] = round(r["unfused_ms"] / r["fused_ms"], 1)
        fk.fk_plan_destroy(plan)
        log("data_size", r)
        data_size.append(r)

    hf_plain = []
    for B in HF_PLAIN_BATCHES:
        cfg = datagen.cast_chain_batch(B, seed=args.seed)
        ch, frame, outs, arr, plan = setup(cfg)
        r = {"batch": B, "fused_ms": round(timeit(lambda: fk.fk_run(plan, arr, B, stream), 50), 5)}
        singles = [fk.make_items(ch, [frame], [it], [outs[b]]) for b, it in enumerate(cfg["items"])]
        r["per_image_ms"] = round(timeit(lambda: [fk.fk_run(plan, s1, 1, stream) for s1 in singles], 5), 4)
        r["speedup_vs_per_image"] = round(r["per_image_ms"] / r["fused_ms"], 1)
        if not args.no_unfused:
            r["unfused_ms"] = round(unfused_ms(plan, arr, B, 3), 4)
            r["speedup_vs_unfused"] = round(r["unfused_ms"] / r["fused_ms"], 1)
        # the same batch with one output tensor per item, in reverse address
        # order (no constant stride): its parameters go through the device
        # run table and its upload kernel
        # (up to 32 items travel in the kernel arguments either way)
        if B > 32:
            sep = [torch.empty_like(o) for o in outs][::-1]
            arr_t = fk.make_items(ch, [frame], cfg["items"], sep)
            r["table_ms"] = round(timeit(lambda: fk.fk_run(plan, arr_t, B, stream), 50), 5)
        # the autotuner's choice and its own time for it (median of 3
        # samples of 10 back-to-back launches), next to its time for the
        # default configuration
        best, times = fk.fk_autotune(plan, arr, B, 10)
        space = [(c.block_threads, c.coarsen) for c in fk.fk_autotune_space()]
        r["autotuned"] = [best.block_threads, best.coarsen]
        r["autotuned_ms"] = round(min(times), 5)
        r["tuner_default_ms"] = round(times[space.index((256, 1))], 5)
        fk.fk_plan_destroy(plan)
        log("hf_plain", r)
        hf_plain.append(r)

    dtypes = []
    for din, dout in DTYPE_PAIRS:
        cfg = datagen.cast_chain_batch(50, din, dout, seed=args.seed)
        ch, frame, outs, arr, plan = setup(cfg)
        r = {"in": din, "out": dout, "fused_ms": round(timeit(lambda: fk.fk_run(plan, arr, 50, stream), 50), 5)}
        if not args.no_unfused:
            r["unfused_ms"] = round(unfused_ms(plan, arr, 50, 3), 4)
            r["speedup"] = round(r["unfused_ms"] / r["fused_ms"], 1)
        fk.fk_plan_destroy(plan)
        log("dtypes", r)
        dtypes.append(r)
    # Section VI-I's remark that double precision turns the kernel compute-
    # bound, checked at a size where arithmetic can show: the same op list in
    # fp32 (fp32 write) and in fp64 (fp64 write) over one 3840x2160 fp32 frame
    # (autotuned on one frame, then timed over rotating frame copies, so the
    # frames come from HBM)
    precision = []
    g = datagen.rng(args.seed + 5)
    pframe = torch.from_numpy(datagen.frame(g, 2160, 3840, 1, dtype="f32")).to(dev)
    pframes = [pframe] + [pframe.clone() for _ in range(rotation_sets(pframe.numel() * 4) - 1)]
    it = {"frame": 0, "x": 0, "y": 0, "w": 3840, "h": 2160}
    for n_ops in PRECISION_DEPTHS:
        base = datagen.muladd_chain(n_ops, datagen.rng(args.seed + n_ops), channels=1)
        for dout in ("f32", "f64"):
            ch = dict(base, read=dict(base["read"], dtype="f32"), write={"dtype": dout, "layout": "packed"})
            outs = [torch.empty((2160, 3840, 1), dtype=fk.TORCH_DTYPE[dout], device=dev) for _ in pframes]
            arrs = [fk.make_items(ch, [f], [it], [o]) for f, o in zip(pframes, outs)]
            plan = fk.fk_plan_create(fk.chain_desc(ch), 1, fk.plan_opts(tier=fk.FK_TIER_RUNTIME))
            best, times = fk.fk_autotune(plan, arrs[0], 1, 5)
            ms = rotating_ms(lambda a: fk.fk_run(plan, a, 1, stream), arrs, 50, warm_s=2e-3)
            nbytes = 2160 * 3840 * (4 + outs[0].element_size())
            r = {"n_ops": n_ops, "out": dout, "autotuned": [best.block_threads, best.coarsen],
                 "rotation_sets": len(pframes), "fused_ms": round(ms, 5),
                 "gbps": round(nbytes / (ms * 1e-3) / 1e9, 1),
                 "gflops": round(n_ops * 2160 * 3840 / (ms * 1e-3) / 1e9, 1),
                 "autotune_one_frame_ms": round(min(times), 5)}
            fk.fk_plan_destroy(plan)
            del outs, arrs
            log("precision", r)
            precision.append(r)
    del pframes

    # Section VI-E: 500 fp32 multiplications split into ops of M instructions
    # over 66,355,200 values (the paper's 259,200 blocks of 256 threads):
    # one fused kernel vs the unfused baseline with one kernel per op, each
    # applying its multiplication M times
    per_op = []
    for M in IPO_SIZES:
        cfg = datagen.instructions_per_op_case(M, n_elems=66355200, seed=args.seed)
        ch = cfg["chain"]
        frame = torch.from_numpy(cfg["frames"][0]).to(dev)
        out = torch.empty(fk.out_shape(ch, cfg["items"][0]), dtype=torch.float32, device=dev)
        arr = fk.make_items(ch, [frame], cfg["items"], [out])
        plan = fk.fk_plan_create(fk.chain_desc(ch), 1, fk.plan_opts(unfused_loop_kernel=True))
        r = {"per_op": M, "ops": -(-500 // M), "fused_ms": round(timeit(lambda: fk.fk_run(plan, arr, 1, stream), 10), 4)}
        if not args.no_unfused:
            r["unfused_ms"] = round(unfused_ms(plan, arr, 1, 2), 4)
            r["speedup"] = round(r["unfused_ms"] / r["fused_ms"], 2)
        fk.fk_plan_destroy(plan)
        del frame, out
        log("instructions_per_op", r)
        per_op.append(r)
    top = data_size[-1]
    n = top["n"]
    flops = 2.0 * 100 * n
    tf = flops / (top["fused_ms"] * 1e-3) / 1e12
    return {"metric": "paper sweeps: fused vs unfused times", "value": round(tf, 3), "unit": "TFLOP/s",
            "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "sweeps: data size (VI-G), plain-read HF (VI-C), data types (VI-I)",
                       "seed": args.seed},
            "roofline": {**alu_roof(tf), "traffic": None,
                         "kernel": f"fused 100 mul+add pairs over {n} fp32 values", "kernel_ms": top["fused_ms"]},
            "data_size": data_size, "hf_plain": hf_plain, "dtypes": dtypes, "precision": precision,
            "instructions_per_op": per_op}


def reads_workload(args):
    """The other read ops (nearest-neighbour and NV12), fused vs the unfused
    baseline (fused times over rotating copies of the frame, read from HBM):
      nv12_full:   a 3840x2160 NV12 frame (12.4 MB) converted to planar fp32
                   B, G, R (99.5 MB written): HBM-bound, algorithmic bytes =
                   frame + output;
      nv12_crops:  256 uneven crops of the same frame, resized bilinearly to
                   64x128 and normalised (the hot chain on NV12 input);
      nearest_crops: the same 256 crops of a 3840x2160x3 u8 frame with a
                   nearest-neighbour resize."""
    import torch

    import datagen
    import paper_2508_07071_amd as fk

    dev = torch.device("cuda:0")
    stream = fk.stream_handle()
    H, W = FRAME_HW
    g = datagen.rng(args.seed)


    def measure(ch, frame, items, alg, name, reps=50):
        # autotuned on the frame, then timed over rotating (frame copy,
        # outputs) sets, so the frames come from HBM
        R = rotation_sets(frame.numel() * frame.element_size())
        frames = [frame] + [frame.clone() for _ in range(R - 1)]
        arrs = []
        for f in frames:
            outs = [torch.empty(fk.out_shape(ch, it), dtype=fk.TORCH_DTYPE[ch["write"]["dtype"]], device=dev)
                    for it in items]
            arrs.append((fk.make_items(ch, [f], items, outs), outs))
        arr = arrs[0][0]
        n = len(items)
        plan = fk.fk_plan_create(fk.chain_desc(ch), n, fk.plan_opts())
        best, _ = fk.fk_autotune(plan, arr, n, 5)
        r = {"case": name, "items": n, "alg_bytes": alg, "autotuned": [best.block_threads, best.coarsen],
             "rotation_sets": R}
        # the autotuner times one frame, which stays cached; every
        # configuration timed again over the rotating sets picks the one
        # that is fastest from HBM
        sweep = {}
        for c in fk.fk_autotune_space():
            fk.fk_plan_set_config(plan, c)
            sweep[(c.block_threads, c.coarsen)] = rotating_ms(lambda a: fk.fk_run(plan, a[0], n, stream), arrs, 20)
        hbm_best = min(sweep, key=sweep.get)
        fk.fk_plan_set_config(plan, fk.fk_launch_config(*hbm_best))
        r["best_from_hbm"] = list(hbm_best)
        r["fused_ms"] = round(rotating_ms(lambda a: fk.fk_run(plan, a[0], n, stream), arrs, reps,
                                          warm_s=2e-3), 5)
        r["gbps"] = round(alg / (r["fused_ms"] * 1e-3) / 1e9, 1)
        r["hbm_frac"] = round(r["gbps"] / HBM_PEAK_GBPS, 4)
        if not args.no_unfused:
            nbytes = fk.fk_unfused_scratch_bytes(plan, arr, n)
            scratch = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
            r["unfused_ms"] = round(timeit(lambda: fk.fk_run_unfused(plan, arr, n, scratch.data_ptr(), nbytes,
                                                                   stream), 3), 4)
            r["speedup_vs_unfused"] = round(r["unfused_ms"] / r["fused_ms"], 1)
        fk.fk_plan_destroy(plan)
        del frames, arrs
        log(r)
        return r

    nv12 = torch.from_numpy(datagen.nv12_frame(g, H, W)).to(dev)
    rows = []
    full = {"read": {"kind": "nv12", "dtype": "u8", "channels": 3, "out_w": 0, "out_h": 0},
            "ops": [], "write": {"dtype": "f32", "layout": "planar"}}
    rows.append(measure(full, nv12, [{"frame": 0, "x": 0, "y": 0, "w": W, "h": H}],
                        H * W * 3 // 2 + H * W * 3 * 4, "nv12_full"))
    crops = datagen.random_crops(g, 256, W, H)
    norm = datagen.normalize_chain(64, 128)
    taps = sum(min(it["w"], 128) * min(it["h"], 256) * 3 // 2 for it in crops)
    rows.append(measure(dict(norm, read=dict(norm["read"], kind="nv12_resize")), nv12, crops,
                        taps + 256 * 3 * 128 * 64 * 4, "nv12_crops"))
    bgr = torch.from_numpy(datagen.frame(g, H, W, 3)).to(dev)
    taps = sum(min(it["w"], 64) * min(it["h"], 128) * 3 for it in crops)
    rows.append(measure(dict(norm, read=dict(norm["read"], kind="crop_nearest")), bgr, crops,
                        taps + 256 * 3 * 128 * 64 * 4, "nearest_crops"))
    top = rows[0]
    return {"metric": "other read ops: fused GB/s vs unfused", "value": top["gbps"], "unit": "GB/s",
            "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "reads: NV12 4K frame to planar fp32; 256 NV12 / nearest crops -> 64x128",
                       "seed": args.seed},
            "roofline": {"bound": "hbm", "achieved": top["gbps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": top["hbm_frac"], "traffic": None,
                         "kernel": "NV12 3840x2160 -> planar fp32 BGR", "kernel_ms": top["fused_ms"]},
            "rows": rows}


def serve_workload(args):
    """Serving loop (config 4 sizes): open-loop Poisson arrivals, continuous
    batching vs per-request fused vs per-request unfused; p50/p99 latency."""
    import torch

    from paper_2508_07071_amd import serve

    import paper_2508_07071_amd as fk

    dev = torch.device("cuda:0")
    arena = torch.empty(args.arena_gb << 30, dtype=torch.uint8, device=dev)
    pool = serve.make_pool(8, seed=args.seed)
    rows = []
    modes = [fk.FK_SERVER_BATCHED, fk.FK_SERVER_PER_REQUEST, fk.FK_SERVER_UNFUSED]
    for rate in args.rates:
        for mode in modes:
            if mode == fk.FK_SERVER_UNFUSED and rate > 2000:
                continue  # saturated from about 1,200 req/s on
            n = max(args.serve_requests, int(rate * args.serve_seconds))
            if mode == fk.FK_SERVER_UNFUSED and rate > 1000:
                n = min(n, 1000)  # past its capacity the baseline's backlog only grows
            log(f"serve rate={rate} mode={mode} n={n}")
            r = serve.run(rate, n, mode, pool, arena, seed=args.seed, budget_bytes=args.budget_gb << 30)
            log(r)
            rows.append(r)
    # beyond config 4: the same requests on frames already on the device (no
    # PCIe copy), at rates where the fused launches, not the copies, load
    # the GPU
    dpool = serve.make_pool(8, seed=args.seed, device=True)
    # heavier requests: 640x480 frames, 48-64 crops each resized to 224x224
    heavy = {"w_range": (640, 640), "h_range": (480, 480), "min_crops": 48, "max_crops": 64,
             "out_size": (224, 224)}
    for kind, rates, kw in (("config-4 requests", args.device_rates, None),
                            ("640x480 frames, 48-64 crops of 224x224", args.heavy_rates, heavy)):
        for rate in rates:
            for mode in modes[:2]:
                n = max(args.serve_requests, int(rate * args.serve_seconds))
                log(f"serve device frames, {kind}, rate={rate} mode={mode} n={n}")
                r = serve.run(rate, n, mode, dpool, arena, seed=args.seed,
                              budget_bytes=args.budget_gb << 30, request_kw=kw)
                r["beyond_configs"] = True
                r["requests_kind"] = kind
                log(r)
                rows.append(r)
    del dpool
    out = {"workload": "serving: Poisson arrivals, 640x480..3840x2160 u8 frames, 1-64 crops -> "
                       "224x224 or 64x128 normalised planar fp32", "arena_gb": args.arena_gb,
           "budget_gb": args.budget_gb or args.arena_gb, "rows": rows}
    if not args.no_cpu_baseline:
        import datagen
        import oracle
        g = datagen.rng(args.seed)
        reqs = datagen.poisson_requests(g, 200.0, 10)
        chain = datagen.normalize_chain(224, 224)
        big = datagen.frame(datagen.rng(args.seed + 1), 2160, 3840, 3)
        t0 = time.perf_counter()
        for r in reqs:
            fh, fw = r["frame_hw"]
            frame = big.reshape(-1)[:fh * fw * 3].reshape(fh, fw, 3)
            oracle.run_chain(chain, [frame], [dict(c, frame=0) for c in r["crops"]], shadow=False)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(len(reqs) / dt, 2), "unit": "req/s", "cores": 1, "kind": "oracle",
                               "sample": f"10 requests of the same distribution, {dt:.2f} s single-threaded"}
    return out


def costmodel_workload(args):
    """Learned cost model (config 3): train on the GPU from labelled shards,
    evaluate on the held-out chains; the fp64 numpy oracle's epoch time is
    the CPU baseline."""
    import numpy as np

    import paper_2508_07071_amd as fk
    from paper_2508_07071_amd import costmodel as cm

    # the committed labelled dataset unless shards are named
    shards = args.data or [os.path.join(os.path.dirname(cm.__file__), "data", "costmodel_dataset.npz")]
    data = cm.load_shards(shards)
    model, rep = cm.fit(data, epochs=args.epochs)
    out = {"workload": "cost model: 20,000 training / 2,000 held-out random chains", "report": rep}
    # the model's choice re-timed on this GPU against a fresh exhaustive
    # autotune, on chains the dataset never saw (another seed)
    live = cm.live_quality(model, n=args.live_chains, seed=20260, reps=10, max_input_bytes=1 << 28)
    out["live"] = {"chains": args.live_chains, "model": live["model"], "default": live["default"]}
    log("live", out["live"])
    if not args.no_cpu_baseline:
        from oracle import mlp
        X = data["features"][:rep["n_train"]]
        Y = cm.targets_from_times(data["times_ms"][:rep["n_train"]])
        p = fk.fk_model_get_params(model).astype(np.float64)
        mean, std = fk.fk_model_get_normalization(model)
        Xs = ((X - mean) / std).astype(np.float64)
        dims = [fk.FK_MODEL_FEATURES, rep["hidden"], rep["hidden"], rep["hidden"], fk.FK_MODEL_OUTPUTS]
        t0 = time.perf_counter()
        for r0 in range(0, Xs.shape[0], rep["batch"]):
            mlp.loss_grad(p, dims, Xs[r0:r0 + rep["batch"]], Y[r0:r0 + rep["batch"]])
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(dt, 3), "unit": "s/epoch", "cores": 1, "kind": "oracle",
                               "sample": "one epoch of forward+backward on the training set, numpy fp64",
                               "gpu_s_per_epoch": rep["gpu_seconds_per_epoch"]}
    fk.fk_model_destroy(model)
    return out


def copy_workload(args):
    """Device-to-device copy of known size (torch's copy kernel): measured
    HBM bandwidth for context, and the reference for scaling rocprofv3's
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    dev = torch.device("cuda:0")
    nbytes = 256 << 20
    bufs = [torch.empty(nbytes, dtype=torch.uint8, device=dev) for _ in range(8)]
    for b in bufs:
        b.fill_(1)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for i in range(args.warmup):
        bufs[(2 * i + 1) % 8].copy_(bufs[(2 * i) % 8])
    torch.cuda.synchronize()
    e0.record()
    for i in range(args.steps):
        bufs[(2 * i + 1) % 8].copy_(bufs[(2 * i) % 8])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    return {"workload": "d2d copy 256 MiB (read + write), 4 rotating pairs", "bytes_per_copy": 2 * nbytes,
            "ms": round(ms, 5), "gbps": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


def trace_summary(path, what):
    """Markdown rows from a rocprofv3 CSV, one per (kernel, grid, block):
    kernel durations from a kernel trace (what = "trace"), or the average
    counter value per dispatch from a counter collection (what = "pmc")."""
    import csv
    from collections import defaultdict

    groups = defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            key = (r["Kernel_Name"], r.get("Grid_Size", r.get("Grid_Size_X", "")),
                   r.get("Workgroup_Size", r.get("Workgroup_Size_X", "")),
                   r.get("Stream_Id", r.get("Queue_Id", "")), r.get("Counter_Name", ""))
            if what == "trace":
                groups[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
            else:
                groups[key].append(float(r["Counter_Value"]))
    unit = "us" if what == "trace" else "per dispatch"
    print(f"| kernel | grid (threads) | block | stream/queue | counter | dispatches | avg {unit} | min | max |")
    print("|---|---|---|---|---|---|---|---|---|")
    for (k, g, b, q, c), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        print(f"| `{k}` | {g} | {b} | {q} | {c} | {len(v)} | {sum(v) / len(v):.2f} | {min(v):.2f} | "
              f"{max(v):.2f} |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="vf", choices=["vf", "hf", "loop", "stats", "sweeps", "reads", "copy", "serve", "costmodel"])
    ap.add_argument("--data", nargs="+", default=[],
                    help="cost-model label shards (default: the committed dataset)")
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--live-chains", type=int, default=100,
                    help="cost model: unseen chains re-timed against a fresh autotune on this GPU")
    ap.add_argument("--rates", type=float, nargs="+", default=[200, 500, 1000, 2000, 4000, 6000],
                    help="serving rates with host frames (config 4 is 200..2000; 4000 and 6000 "
                         "find where the frame copies saturate PCIe)")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--serve-requests", type=int, default=2000, help="at least this many requests per rate")
    ap.add_argument("--device-rates", type=float, nargs="+", default=[2000, 10000, 20000],
                    help="serving rates with frames already on the device")
    ap.add_argument("--heavy-rates", type=float, nargs="+", default=[5000, 10000, 20000],
                    help="device-frame rates for 640x480 frames with 48-64 crops of 224x224")
    ap.add_argument("--arena-gb", type=int, default=64)
    ap.add_argument("--budget-gb", type=int, default=0, help="0 = the whole arena")
    ap.add_argument("--rotate", type=int, default=24,
                    help="(frame, output) sets the depth sweep rotates over; 24 keeps every "
                         "frame read coming from HBM")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--strict", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="tune each depth's launch config first on single launches over rotating frames "
                         "(default: the library default)")
    ap.add_argument("--no-unfused", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=432)
    ap.add_argument("--no-hot-chain", action="store_true",
                    help="skip the config 0 / config 2 rows")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving row")
    ap.add_argument("--hot-profile", action="store_true",
                    help="config 0 / config 2 rows: autotune and the rotating timed launches only "
                         "(for profiler runs: one kernel-trace row per batch size)")
    ap.add_argument("--hot-configs", metavar="JSON",
                    help="take the config 0 / config 2 launch configs from this earlier bench output "
                         "instead of autotuning")
    ap.add_argument("--gather", choices=["direct", "lds"], default="direct",
                    help="config 0 / config 2 rows: the tap reads of the bilinear gather "
                         "(direct per-pixel loads, or rows staged in LDS)")
    ap.add_argument("--hot-reps", type=int, default=200,
                    help="timed launches per measurement in the config 0 / config 2 rows")
    ap.add_argument("--trace-summary", metavar="CSV",
                    help="print a rocprofv3 kernel-trace CSV as markdown rows per kernel, grid and block")
    ap.add_argument("--pmc-summary", metavar="CSV",
                    help="the same for a rocprofv3 counter-collection CSV")
    args = ap.parse_args()
    if args.trace_summary or args.pmc_summary:
        trace_summary(args.trace_summary or args.pmc_summary, "trace" if args.trace_summary else "pmc")
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(items and frames shard across GPUs with no exchange; see the design notes).",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "hf":
        print(json.dumps(hf_workload(args)))
        return
    if args.workload == "costmodel":
        print(json.dumps(costmodel_workload(args)))
        return
    if args.workload == "loop":
        print(json.dumps(loop_workload(args)))
        return
    if args.workload == "stats":
        print(json.dumps(stats_workload(args)))
        return
    if args.workload == "sweeps":
        print(json.dumps(sweeps_workload(args)))
        return
    if args.workload == "reads":
        print(json.dumps(reads_workload(args)))
        return
    if args.workload == "serve":
        print(json.dumps(serve_workload(args)))
        return
    if args.workload == "copy":
        print(json.dumps(copy_workload(args)))
        return
    res, cfgs = vf_sweep(args)
    if not args.no_hot_chain:
        log("hot chain rows ...")
        res["per_config"] = hot_chain_rows(args)
    if not args.no_serving:
        log("serving row ...")
        res["serving"] = serving_row(args)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        res["cpu_baseline"] = cpu_baseline_vf(args, cfgs)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
