"""Seeded synthetic inputs for the fused preprocessing chain.

This module is shared by the GPU path's tests and benchmark and by the CPU
oracle's tests.  It holds no arithmetic of the method: it only draws frames,
crop rectangles, op constants and arrival times from numpy's PCG64 generator
(``numpy.random.default_rng(seed)``) and describes chains as plain data.

Draw order inside one workload is fixed: frame bytes first, then crop
parameters, then op constants, so the same seed always yields the same
workload whatever the consumer.

A chain is a dict::

    {"read":  {"kind": "plain" | "crop_resize" | "crop_nearest" | "nv12" | "nv12_resize",
               "dtype": "u8"|"f16"|"f32",
               "channels": 1|3|4, "out_w": int, "out_h": int},
     "ops":   [{"kind": "swap"|"cvt"|"mul"|"add"|"sub"|"div", "k": [floats]}
               | {"kind": "loop", "span": s, "count": n}],
     "write": {"dtype": "f32"|"f16", "layout": "packed"|"planar"}}

``k`` holds 0 (swap/cvt), 1 (scalar) or ``channels`` fp32-representable
constants.  A loop op repeats the ``s`` ops just before it so that they run
``n`` times in all.  An item is a dict ``{"frame": index, "x", "y", "w", "h",
"out_w", "out_h"}`` naming a region of interest of one of the frames.

The workloads mirror the paper's synthetic benchmarks (Section VI): uint8
images, Batch(Crop -> Resize -> ColorConvert -> Multiply -> Subtract ->
Divide -> Split) with 64x128 outputs (Sections VI-F and VI-J), and long
Mul/Add chains on a single large frame (Section VI-B).
"""
from __future__ import annotations

import math

import numpy as np

DTYPES = {"u8": np.uint8, "f16": np.float16, "f32": np.float32, "f64": np.float64}

# ImageNet-style normalisation constants of the hot chain, RGB order.
NORM_SCALE = float(np.float32(1.0) / np.float32(255.0))
NORM_MEAN = [float(np.float32(v)) for v in (0.485, 0.456, 0.406)]
NORM_STD = [float(np.float32(v)) for v in (0.229, 0.224, 0.225)]


def f32(v) -> float:
    """Round a Python number to the nearest fp32 value (as a Python float)."""
    return float(np.float32(v))


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def frame(g: np.random.Generator, h: int, w: int, c: int = 3, dtype: str = "u8") -> np.ndarray:
    """Uniform random packed HWC frame.  u8: every byte uniform in 0..255;
    f16/f32/f64: uniform in [0, 255) rounded to the storage type."""
    if dtype == "u8":
        return g.integers(0, 256, size=(h, w, c), dtype=np.uint8)
    vals = g.uniform(0.0, 255.0, size=(h, w, c))
    return vals.astype(DTYPES[dtype])


def index_coded_frame(h: int, w: int, c: int = 3) -> np.ndarray:
    """u8 frame whose bytes name their own coordinates:
    channel 0 = x mod 256, channel 1 = y mod 256,
    channel 2 = (x >> 8) | ((y >> 8) << 3), channel 3 (if any) = 255 - channel 0.
    Channels beyond those present are dropped; for c == 1 only x mod 256."""
    ys, xs = np.mgrid[0:h, 0:w]
    planes = [xs & 255, ys & 255, (xs >> 8) | ((ys >> 8) << 3), 255 - (xs & 255)]
    return np.stack(planes[:c], axis=-1).astype(np.uint8)


def linear_index_frame(h: int, w: int, c: int = 3) -> np.ndarray:
    """fp32 frame holding each element's linear index (exact below 2**24)."""
    n = h * w * c
    assert n < (1 << 24)
    return np.arange(n, dtype=np.float32).reshape(h, w, c)


def normalize_chain(out_w: int, out_h: int, channels: int = 3) -> dict:
    """Crop+bilinear resize -> BGR->RGB -> fp32 -> *1/255 -> -mean -> /std ->
    planar fp32: the hot chain of Sections VI-F and VI-J."""
    return {
        "read": {"kind": "crop_resize", "dtype": "u8", "channels": channels,
                 "out_w": out_w, "out_h": out_h},
        "ops": [
            {"kind": "swap", "k": []},
            {"kind": "cvt", "k": []},
            {"kind": "mul", "k": [NORM_SCALE]},
            {"kind": "sub", "k": NORM_MEAN[:channels] if channels == 3 else [NORM_MEAN[0]]},
            {"kind": "div", "k": NORM_STD[:channels] if channels == 3 else [NORM_STD[0]]},
        ],
        "write": {"dtype": "f32", "layout": "planar"},
    }


def muladd_chain(n_ops: int, g: np.random.Generator, channels: int = 3,
                 layout: str = "packed") -> dict:
    """Plain read -> fp32 -> n_ops alternating ops: op k is a multiply when k
    is even (constant uniform in [0.5, 1.5)) and an add when k is odd
    (constant uniform in [-1, 1)); one scalar constant per op, drawn in op
    order (Section VI-B's Mul+Add chains, with distinct constants)."""
    ops = [{"kind": "cvt", "k": []}]
    for k in range(n_ops):
        if k % 2 == 0:
            ops.append({"kind": "mul", "k": [f32(g.uniform(0.5, 1.5))]})
        else:
            ops.append({"kind": "add", "k": [f32(g.uniform(-1.0, 1.0))]})
    return {
        "read": {"kind": "plain", "dtype": "u8", "channels": channels, "out_w": 0, "out_h": 0},
        "ops": ops,
        "write": {"dtype": "f32", "layout": layout},
    }


def loop_chain(pairs: int, g: np.random.Generator, channels: int = 1,
               layout: str = "packed") -> dict:
    """Plain read -> fp32 -> one Mul and one Add run `pairs` times through a
    loop op (Sections VI-B and VI-D: one instance of each op type repeated
    by a loop op).  Multiplier uniform in [0.5, 0.95), addend uniform in
    [-1, 1), drawn in that order: the map is a contraction, so values stay
    within max(255, 20) for any number of pairs."""
    m = f32(g.uniform(0.5, 0.95))
    a = f32(g.uniform(-1.0, 1.0))
    ops = [{"kind": "cvt", "k": []}, {"kind": "mul", "k": [m]}, {"kind": "add", "k": [a]},
           {"kind": "loop", "span": 2, "count": int(pairs)}]
    return {
        "read": {"kind": "plain", "dtype": "u8", "channels": channels, "out_w": 0, "out_h": 0},
        "ops": ops,
        "write": {"dtype": "f32", "layout": layout},
    }


def loop_batch(pairs: int, seed: int = 0, batch: int = 50, hw=(120, 60), channels: int = 1) -> dict:
    """`batch` u8 images of hw (height, width) in one frame: columns of up
    to 512 images stacked vertically (image b at column b // 512, rows
    [(b % 512) h, (b % 512 + 1) h)); one item per image; loop_chain(pairs)
    (Section VI-D: batch 50 of 60 x 120 uchar images, Mul+Add pairs)."""
    g = rng(seed)
    h, w = hw
    per_col = 512
    cols = (batch + per_col - 1) // per_col
    fr = frame(g, min(batch, per_col) * h, cols * w, channels)
    items = [{"frame": 0, "x": (b // per_col) * w, "y": (b % per_col) * h, "w": w, "h": h,
              "out_w": w, "out_h": h} for b in range(batch)]
    return {"frames": [fr], "items": items, "chain": loop_chain(pairs, g, channels), "seed": seed}


def data_size_case(n_elems: int, pairs: int = 100, seed: int = 0, row: int = 4096) -> dict:
    """Section VI-G: a 1-D fp32 array of about n_elems values (uniform in
    [0, 255)), no batch, then `pairs` Mul+Add pairs through a loop op.  The
    array is held as one row when n_elems <= row, else as n_elems // row rows
    of `row` values (n rounded down to whole rows)."""
    g = rng(seed)
    w = min(n_elems, row)
    h = max(1, n_elems // row) if n_elems > row else 1
    fr = frame(g, h, w, 1, dtype="f32")
    m = f32(g.uniform(0.5, 0.95))
    a = f32(g.uniform(-1.0, 1.0))
    chain = {"read": {"kind": "plain", "dtype": "f32", "channels": 1, "out_w": 0, "out_h": 0},
             "ops": [{"kind": "mul", "k": [m]}, {"kind": "add", "k": [a]},
                     {"kind": "loop", "span": 2, "count": int(pairs)}],
             "write": {"dtype": "f32", "layout": "packed"}}
    return {"frames": [fr], "items": [whole_frame_item(fr)], "chain": chain, "seed": seed}


def instructions_per_op_case(per_op: int, total: int = 500, n_elems: int = 1 << 16, seed: int = 0,
                             row: int = 4096) -> dict:
    """Section VI-E: `total` fp32 multiplications split into ops of
    `per_op` instructions each (the last op takes the remainder), as a
    chain of Mul ops each looped `per_op` times, over a 1-D fp32 array held
    as rows of `row` values.  Multiplier uniform in [0.999, 1.001) (drawn
    after the values), so 500 products stay within a factor of two."""
    g = rng(seed)
    h = max(1, n_elems // row)
    fr = frame(g, h, min(n_elems, row), 1, dtype="f32")
    m = f32(g.uniform(0.999, 1.001))
    ops, left = [], total
    while left > 0:
        k = min(per_op, left)
        ops.append({"kind": "mul", "k": [m]})
        if k > 1:
            ops.append({"kind": "loop", "span": 1, "count": int(k)})
        left -= k
    chain = {"read": {"kind": "plain", "dtype": "f32", "channels": 1, "out_w": 0, "out_h": 0},
             "ops": ops, "write": {"dtype": "f32", "layout": "packed"}}
    return {"frames": [fr], "items": [whole_frame_item(fr)], "chain": chain, "seed": seed}


def cast_chain_batch(batch: int = 50, in_dtype: str = "u8", out_dtype: str = "f32", seed: int = 0,
                     hw=(120, 60)) -> dict:
    """Sections VI-C and VI-I: `batch` single-channel images of hw (height,
    width) in one frame: columns of up to 512 images stacked vertically
    (image b at column b // 512, rows [(b % 512) h, (b % 512 + 1) h)), chain
    Read -> Cast -> Multiply -> Subtract -> Divide -> Write.  Constants:
    mul uniform in [0.5, 1.5), sub in [-1, 1), div in [0.5, 1.5), drawn after
    the frame values."""
    g = rng(seed)
    h, w = hw
    per_col = 512
    cols = (batch + per_col - 1) // per_col
    fr = frame(g, min(batch, per_col) * h, cols * w, 1, dtype=in_dtype)
    ops = [{"kind": "cvt", "k": []}, {"kind": "mul", "k": [f32(g.uniform(0.5, 1.5))]},
           {"kind": "sub", "k": [f32(g.uniform(-1.0, 1.0))]}, {"kind": "div", "k": [f32(g.uniform(0.5, 1.5))]}]
    chain = {"read": {"kind": "plain", "dtype": in_dtype, "channels": 1, "out_w": 0, "out_h": 0},
             "ops": ops, "write": {"dtype": out_dtype, "layout": "packed"}}
    items = [{"frame": 0, "x": (b // per_col) * w, "y": (b % per_col) * h, "w": w, "h": h, "out_w": w, "out_h": h}
             for b in range(batch)]
    return {"frames": [fr], "items": items, "chain": chain, "seed": seed}


def nv12_frame(g: np.random.Generator, h: int, w: int) -> np.ndarray:
    """An NV12 frame of h x w luma pixels (h, w even) as (3h/2, w) bytes:
    h luma rows, then h/2 rows of w/2 (U, V) pairs; every byte uniform in
    0..255."""
    assert h % 2 == 0 and w % 2 == 0
    return g.integers(0, 256, size=(h * 3 // 2, w), dtype=np.uint8)


def whole_frame_item(fr: np.ndarray, frame_index: int = 0) -> dict:
    h, w = fr.shape[:2]
    return {"frame": frame_index, "x": 0, "y": 0, "w": w, "h": h, "out_w": w, "out_h": h}


# ---------------------------------------------------------------------------
# The five benchmark workloads (small and full sizes share one recipe).
# ---------------------------------------------------------------------------

def config0(seed: int = 0, frame_hw=(1080, 1920), crop=(100, 200, 512, 512), out=(224, 224)) -> dict:
    """One BGR u8 frame (uniform bytes); crop (x, y, w, h) bilinear-resized to
    out=(out_w, out_h), normalised, written planar fp32."""
    g = rng(seed)
    fr = frame(g, frame_hw[0], frame_hw[1], 3)
    x, y, w, h = crop
    items = [{"frame": 0, "x": x, "y": y, "w": w, "h": h, "out_w": out[0], "out_h": out[1]}]
    return {"frames": [fr], "items": items, "chain": normalize_chain(out[0], out[1]), "seed": seed}


def config1(n_ops: int, seed: int = 0, frame_hw=(2160, 3840)) -> dict:
    """One u8 frame; cvt then n_ops alternating mul/add; packed HWC fp32."""
    g = rng(seed)
    fr = frame(g, frame_hw[0], frame_hw[1], 3)
    chain = muladd_chain(n_ops, g)
    return {"frames": [fr], "items": [whole_frame_item(fr)], "chain": chain, "seed": seed}


def random_crops(g: np.random.Generator, n: int, frame_w: int, frame_h: int,
                 lo: int = 60, hi: int = 600, out=(64, 128), frame_index: int = 0) -> list:
    """n crops with sides uniform in lo..hi (clipped to the frame), positions
    uniform over the valid range; drawn per crop in the order w, h, x, y."""
    items = []
    for _ in range(n):
        w = int(g.integers(lo, min(hi, frame_w) + 1))
        h = int(g.integers(lo, min(hi, frame_h) + 1))
        x = int(g.integers(0, frame_w - w + 1))
        y = int(g.integers(0, frame_h - h + 1))
        items.append({"frame": frame_index, "x": x, "y": y, "w": w, "h": h,
                      "out_w": out[0], "out_h": out[1]})
    return items


def config2(batch: int, seed: int = 0, frame_hw=(2160, 3840), out=(64, 128),
            side=(60, 600)) -> dict:
    """One u8 frame, `batch` uneven crops, each resized to out=(64 wide,
    128 high), normalised and split into one contiguous [B][3][128][64]
    output."""
    g = rng(seed)
    fr = frame(g, frame_hw[0], frame_hw[1], 3)
    items = random_crops(g, batch, frame_hw[1], frame_hw[0], side[0], side[1], out)
    return {"frames": [fr], "items": items, "chain": normalize_chain(out[0], out[1]), "seed": seed}


# --- random chains for the launch-configuration cost model -----------------

OUT_SIZES = [(64, 128), (128, 128), (224, 224), (256, 256), (512, 512)]
OP_KINDS = ["swap", "cvt", "mul", "add", "sub", "div"]


def log_uniform_int(g: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))


def random_chain_spec(g: np.random.Generator, max_ops: int = 64,
                      side=(64, 4096), max_batch: int = 256,
                      max_input_bytes: int = 1 << 30) -> dict:
    """One random chain with its input geometry (no pixel data).

    Read op: crop+resize or plain read (p = 1/2).  1..max_ops compute ops
    uniform over {swap, cvt, mul, add, sub, div}; scalar or per-channel
    constants (p = 1/2), mul/div constants uniform in [0.5, 1.5), add/sub in
    [-1, 1).  Input sides log-uniform in `side`, dtype uniform over
    u8/f16/f32, channels uniform over 1/3/4, batch log-uniform in
    1..max_batch, shrunk so that the batch's input bytes stay within
    max_input_bytes.  Crop+resize items draw an ROI with sides >= 16 px and
    an output size from OUT_SIZES.  Output fp32/fp16, packed or planar."""
    read_kind = "crop_resize" if g.uniform() < 0.5 else "plain"
    in_dtype = ["u8", "f16", "f32"][int(g.integers(0, 3))]
    channels = [1, 3, 4][int(g.integers(0, 3))]
    fw = log_uniform_int(g, side[0], side[1])
    fh = log_uniform_int(g, side[0], side[1])
    esize = np.dtype(DTYPES[in_dtype]).itemsize
    batch = log_uniform_int(g, 1, max_batch)
    per_frame = fw * fh * channels * esize
    batch = max(1, min(batch, max_input_bytes // max(per_frame, 1)))
    n_ops = int(g.integers(1, max_ops + 1))
    ops = []
    for _ in range(n_ops):
        kind = OP_KINDS[int(g.integers(0, len(OP_KINDS)))]
        k: list = []
        if kind in ("mul", "div", "add", "sub"):
            n_k = 1 if (channels == 1 or g.uniform() < 0.5) else channels
            lo, hi = (0.5, 1.5) if kind in ("mul", "div") else (-1.0, 1.0)
            k = [f32(g.uniform(lo, hi)) for _ in range(n_k)]
        ops.append({"kind": kind, "k": k})
    out_dtype = "f32" if g.uniform() < 0.5 else "f16"
    layout = "packed" if g.uniform() < 0.5 else "planar"
    items = []
    if read_kind == "crop_resize":
        ow, oh = OUT_SIZES[int(g.integers(0, len(OUT_SIZES)))]
        for b in range(batch):
            w = int(g.integers(16, fw + 1))
            h = int(g.integers(16, fh + 1))
            x = int(g.integers(0, fw - w + 1))
            y = int(g.integers(0, fh - h + 1))
            items.append({"frame": b, "x": x, "y": y, "w": w, "h": h, "out_w": ow, "out_h": oh})
    else:
        ow, oh = 0, 0
        for b in range(batch):
            items.append({"frame": b, "x": 0, "y": 0, "w": fw, "h": fh, "out_w": fw, "out_h": fh})
    chain = {"read": {"kind": read_kind, "dtype": in_dtype, "channels": channels,
                      "out_w": ow, "out_h": oh},
             "ops": ops, "write": {"dtype": out_dtype, "layout": layout}}
    return {"chain": chain, "frame_hw": (fh, fw), "batch": batch, "items": items}


# --- serving workload ------------------------------------------------------

def poisson_requests(g: np.random.Generator, rate_hz: float, n: int,
                     w_range=(640, 3840), h_range=(480, 2160), max_crops: int = 64,
                     min_crops: int = 1, out_size=None) -> list:
    """Open-loop Poisson arrivals (exponential gaps) of requests, each one
    uint8 BGR frame with uniform sides and min_crops..max_crops crops; each
    crop's sides are uniform in 60..min(600, W, H) and its output is
    224x224 or 64 wide x 128 high with probability 1/2 each, or `out_size`
    (width, height) for every crop when given."""
    t = 0.0
    reqs = []
    for i in range(n):
        t += float(g.exponential(1.0 / rate_hz))
        fw = int(g.integers(w_range[0], w_range[1] + 1))
        fh = int(g.integers(h_range[0], h_range[1] + 1))
        n_crops = int(g.integers(min_crops, max_crops + 1))
        hi = min(600, fw, fh)
        crops = []
        for _ in range(n_crops):
            w = int(g.integers(60, hi + 1))
            h = int(g.integers(60, hi + 1))
            x = int(g.integers(0, fw - w + 1))
            y = int(g.integers(0, fh - h + 1))
            if out_size is not None:
                out = tuple(out_size)
            else:
                out = (224, 224) if g.uniform() < 0.5 else (64, 128)
            crops.append({"x": x, "y": y, "w": w, "h": h, "out_w": out[0], "out_h": out[1]})
        reqs.append({"id": i, "t_arrival": t, "frame_hw": (fh, fw), "crops": crops,
                     "frame_seed": int(g.integers(0, 2**31 - 1))})
    return reqs
