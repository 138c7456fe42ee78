"""Launch-configuration cost model: dataset labelling, training, evaluation.

  label     random chains (datagen.random_chain_spec) -> features
            (fk_model_features) and the autotuner's 20 per-launch times
            (fk_autotune); frames and outputs live in two preallocated
            device arenas
  train     network trained on the GPU by the library (fk_model_train);
            target = log(t_config / t_best) per configuration
  evaluate  quality = t_best / t_chosen per held-out chain (1 = the
            autotuned best), for the model and for the library default

Usage (GPU):
  python -m paper_2508_07071_amd.costmodel label --n 22000 --out DATASET.npz
  python -m paper_2508_07071_amd.costmodel fit --data DATASET.npz --model OUT.bin
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

ARENA_IN = 1 << 30    # per-chain input cap (bytes)
ARENA_OUT = 1 << 30   # per-chain output cap (bytes)
N_TRAIN, N_TEST = 20000, 2000


def _esize(dt):
    return {"u8": 1, "f16": 2, "f32": 4}[dt]


def fit_spec(spec):
    """Shrink a spec's batch so that input and output each fit 1 GiB."""
    ch = spec["chain"]
    C = ch["read"]["channels"]
    fh, fw = spec["frame_hw"]
    in_b = fw * fh * C * _esize(ch["read"]["dtype"])
    items = spec["items"]
    out_px = [it["out_w"] * it["out_h"] for it in items]
    out_b = max(out_px) * C * _esize(ch["write"]["dtype"])
    keep = max(1, min(len(items), ARENA_IN // in_b, ARENA_OUT // out_b))
    spec = dict(spec)
    spec["items"] = items[:keep]
    spec["batch"] = keep
    return spec


def label(n, seed=0, reps=3, log_every=250, start=0):
    """Label chains start .. start+n-1 of the seeded sequence."""
    import torch

    import datagen
    import paper_2508_07071_amd as fk

    dev = torch.device("cuda:0")
    arena_in = torch.full((ARENA_IN + (1 << 20),), 1, dtype=torch.uint8, device=dev)
    arena_out = torch.empty((ARENA_OUT + (1 << 20),), dtype=torch.uint8, device=dev)
    space = fk.fk_autotune_space()
    g = datagen.rng(seed)
    for _ in range(start):  # skip to this shard's first chain (no GPU work)
        datagen.random_chain_spec(g)
    feats = np.zeros((n, fk.FK_MODEL_FEATURES), np.float32)
    times = np.zeros((n, len(space)), np.float32)
    default_idx = np.zeros(n, np.int32)
    meta = []
    t0 = time.time()
    for i in range(n):
        spec = fit_spec(datagen.random_chain_spec(g))
        ch = spec["chain"]
        C = ch["read"]["channels"]
        fh, fw = spec["frame_hw"]
        desc, arr, B = batch_in_arenas(spec, arena_in, arena_out)
        plan = fk.fk_plan_create(desc, B)
        try:
            c = fk.fk_plan_get_config(plan)
            default_idx[i] = [(s.block_threads, s.coarsen) for s in space].index((c.block_threads, c.coarsen))
            feats[i] = fk.fk_model_features(plan, arr, B)
            _, t = fk.fk_autotune(plan, arr, B, reps)
            times[i] = t
        finally:
            fk.fk_plan_destroy(plan)
        meta.append({"read": ch["read"]["kind"], "dtype": ch["read"]["dtype"], "C": C,
                     "ops": len(ch["ops"]), "batch": B, "frame": [fw, fh],
                     "out": ch["write"]["dtype"] + "/" + ch["write"]["layout"]})
        if (i + 1) % log_every == 0:
            print(f"[label] {i + 1}/{n} chains, {time.time() - t0:.0f} s", flush=True)
    return {"features": feats, "times_ms": times, "default_idx": default_idx,
            "meta": np.array([json.dumps(m) for m in meta])}


def batch_in_arenas(spec, arena_in, arena_out):
    """(chain descriptor, fk_item array, batch size) of a spec's batch:
    item b reads frame b at a 256-byte aligned offset of arena_in (whatever
    bytes it holds) and writes its output at the next 256-byte aligned
    offset of arena_out."""
    import paper_2508_07071_amd as fk

    ch = spec["chain"]
    C = ch["read"]["channels"]
    fh, fw = spec["frame_hw"]
    es = _esize(ch["read"]["dtype"])
    fstride = (fw * fh * C * es + 255) // 256 * 256
    esz_out = _esize(ch["write"]["dtype"])
    items = spec["items"]
    B = len(items)
    arr = (fk.fk_item * B)()
    ooff = 0
    for b, it in enumerate(items):
        a = arr[b]
        a.src.ptr = arena_in.data_ptr() + b * fstride
        a.src.width, a.src.height, a.src.pitch_bytes = fw, fh, fw * C * es
        a.x, a.y, a.w, a.h = it["x"], it["y"], it["w"], it["h"]
        a.dst = arena_out.data_ptr() + ooff
        if ch["read"]["kind"] == "crop_resize":
            a.out_w, a.out_h = it["out_w"], it["out_h"]
            ob = it["out_w"] * it["out_h"] * C * esz_out
        else:
            a.out_w, a.out_h = 0, 0
            ob = it["w"] * it["h"] * C * esz_out
        ooff += (ob + 255) // 256 * 256
    assert B * fstride <= arena_in.numel() and ooff <= arena_out.numel()
    return fk.chain_desc(ch), arr, B


def live_quality(model, n=20, seed=20260, reps=10, max_input_bytes=1 << 28):
    """The model's choice re-timed on this GPU: for n random chains drawn
    from `seed` (inputs capped at max_input_bytes), the configuration that
    fk_plan_use_model installs is compared with fk_autotune's best from one
    sweep of all 20 configurations on this device.  Returns per-chain
    quality t_best / t_pick and the same for the library default."""
    import torch

    import datagen
    import paper_2508_07071_amd as fk

    dev = torch.device("cuda:0")
    arena_in = torch.full((max_input_bytes + (1 << 20),), 1, dtype=torch.uint8, device=dev)
    arena_out = torch.empty((ARENA_OUT + (1 << 20),), dtype=torch.uint8, device=dev)
    space = [(s.block_threads, s.coarsen) for s in fk.fk_autotune_space()]
    g = datagen.rng(seed)
    qs, qd, picks = [], [], []
    for _ in range(n):
        spec = fit_spec(datagen.random_chain_spec(g, max_input_bytes=max_input_bytes))
        desc, arr, B = batch_in_arenas(spec, arena_in, arena_out)
        plan = fk.fk_plan_create(desc, B)
        try:
            d = fk.fk_plan_get_config(plan)
            di = space.index((d.block_threads, d.coarsen))
            fk.fk_plan_use_model(plan, model, arr, B)
            c = fk.fk_plan_get_config(plan)
            pi = space.index((c.block_threads, c.coarsen))
            _, t = fk.fk_autotune(plan, arr, B, reps)
        finally:
            fk.fk_plan_destroy(plan)
        t = np.asarray(t, np.float64)
        qs.append(float(t.min() / t[pi]))
        qd.append(float(t.min() / t[di]))
        picks.append(space[pi])
    del arena_in, arena_out
    return {"quality": qs, "picks": picks, "model": summarize(qs), "default": summarize(qd)}


def load_shards(paths):
    """Concatenate label shards (ordered by their start index)."""
    parts = sorted((dict(np.load(p, allow_pickle=False)) for p in paths), key=lambda d: int(d.get("start", 0)))
    out = {}
    for k in ("features", "times_ms", "default_idx", "meta"):
        out[k] = np.concatenate([d[k] for d in parts])
    return out


def targets_from_times(times):
    t = np.asarray(times, np.float64)
    return np.log(t / t.min(axis=1, keepdims=True)).astype(np.float32)


def quality(times, choice):
    """t_best / t_chosen per row (1.0 = chose the fastest measured)."""
    t = np.asarray(times, np.float64)
    return t.min(axis=1) / t[np.arange(t.shape[0]), choice]


def summarize(q):
    q = np.asarray(q, np.float64)
    return {"geomean": float(np.exp(np.mean(np.log(q)))), "mean": float(q.mean()),
            "frac_within_10pct": float(np.mean(q >= 0.9)), "p10": float(np.quantile(q, 0.1)),
            "min": float(q.min())}


def fit(data, hidden=128, epochs=300, batch=512, lr=2e-3, seed=0, n_train=N_TRAIN):
    """Train on the first n_train rows, evaluate on the rest; returns
    (model handle, report dict)."""
    import paper_2508_07071_amd as fk

    X = data["features"]
    Tm = data["times_ms"]
    Y = targets_from_times(Tm)
    n_train = min(n_train, X.shape[0] - 1)
    model = fk.fk_model_create(hidden, seed)
    t0 = time.time()
    curve = fk.fk_model_train(model, X[:n_train], Y[:n_train], epochs, batch, lr, seed)
    train_s = time.time() - t0
    rep = {"n_train": int(n_train), "n_test": int(X.shape[0] - n_train), "epochs": epochs,
           "batch": batch, "lr": lr, "hidden": hidden, "train_seconds": round(train_s, 3),
           "loss_first": float(curve[0]), "loss_last": float(curve[-1])}
    t0 = time.time()
    pred = fk.fk_model_predict_batch(model, X[n_train:])
    rep["predict_us_per_chain"] = round((time.time() - t0) / max(1, X.shape[0] - n_train) * 1e6, 2)
    test_t = Tm[n_train:]
    rep["model"] = summarize(quality(test_t, pred.argmin(axis=1)))
    rep["default"] = summarize(quality(test_t, data["default_idx"][n_train:]))
    # one fixed configuration for all chains, the best such on the training set
    tr_q = [np.mean(np.log(quality(Tm[:n_train], np.full(n_train, j)))) for j in range(Tm.shape[1])]
    jbest = int(np.argmax(tr_q))
    rep["best_fixed_config_index"] = jbest
    rep["best_fixed"] = summarize(quality(test_t, np.full(test_t.shape[0], jbest)))
    pred_tr = fk.fk_model_predict_batch(model, X[:n_train])
    rep["model_train_set"] = summarize(quality(Tm[:n_train], pred_tr.argmin(axis=1)))
    rep["gpu_seconds_per_epoch"] = round(train_s / max(epochs, 1), 5)
    return model, rep


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("label")
    a.add_argument("--n", type=int, default=N_TRAIN + N_TEST)
    a.add_argument("--seed", type=int, default=0)
    a.add_argument("--reps", type=int, default=3)
    a.add_argument("--start", type=int, default=0)
    a.add_argument("--out", required=True)
    m = sub.add_parser("merge", help="concatenate label shards into one dataset file")
    m.add_argument("--data", required=True, nargs="+")
    m.add_argument("--out", required=True)
    b = sub.add_parser("fit")
    b.add_argument("--data", required=True, nargs="+", help="one or more label shards, in order")
    b.add_argument("--model", default=None)
    b.add_argument("--epochs", type=int, default=300)
    b.add_argument("--lr", type=float, default=2e-3)
    b.add_argument("--hidden", type=int, default=128)
    b.add_argument("--n-train", type=int, default=N_TRAIN)
    args = ap.parse_args()
    if args.cmd == "label":
        d = label(args.n, args.seed, args.reps, start=args.start)
        d["start"] = np.array(args.start)
        np.savez_compressed(args.out, **d)
        print(f"[label] wrote {args.out}", flush=True)
    elif args.cmd == "merge":
        d = load_shards(args.data)
        d["start"] = np.array(0)
        np.savez_compressed(args.out, **d)
        print(f"[merge] {d['features'].shape[0]} chains -> {args.out}", flush=True)
    else:
        import paper_2508_07071_amd as fk
        data = load_shards(args.data)
        model, rep = fit(data, hidden=args.hidden, epochs=args.epochs, lr=args.lr, n_train=args.n_train)
        if args.model:
            fk.fk_model_save(model, args.model)
        print(json.dumps(rep), flush=True)
        fk.fk_model_destroy(model)


if __name__ == "__main__":
    main()
