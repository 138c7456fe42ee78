"""CPU oracle for the fused preprocessing chain -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library (the package
``paper_2508_07071_amd``) never imports it, and this package imports nothing
from the GPU library; both read their inputs from the ``datagen`` module.

The arithmetic lives in ``fk_oracle.c`` (plain C, no HIP): every op of a
chain runs unfused over the whole image with fp32 intermediates, next to an
fp64 shadow and a running maximum magnitude per element.  This module only
builds that C file, marshals numpy arrays into it and returns the results.
``mlp.py`` holds the oracle of the cost model's network.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fk_oracle.c")
LIB = os.path.join(HERE, "libfkoracle.so")

_DT = {"u8": 0, "f16": 1, "f32": 2, "f64": 3}
_READ = {"plain": 0, "crop_resize": 1, "crop_nearest": 2, "nv12": 3, "nv12_resize": 4}
_RESIZING = ("crop_resize", "crop_nearest", "nv12_resize")
_NV12 = ("nv12", "nv12_resize")
_OP = {"swap": 0, "cvt": 1, "mul": 2, "add": 3, "sub": 4, "div": 5, "loop": 6}
_LAYOUT = {"packed": 0, "planar": 1, "stats": 2}
_NP_OUT = {"f32": np.float32, "f16": np.float16, "f64": np.float64}


class _Op(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nconst", C.c_int32), ("k", C.c_float * 4),
                ("span", C.c_int32), ("count", C.c_int32)]


class _Chain(C.Structure):
    _fields_ = [("read_kind", C.c_int32), ("in_dtype", C.c_int32), ("channels", C.c_int32),
                ("ops", C.POINTER(_Op)), ("n_ops", C.c_int32), ("out_dtype", C.c_int32),
                ("layout", C.c_int32)]


class _Item(C.Structure):
    _fields_ = [("src", C.c_void_p), ("W", C.c_int32), ("H", C.c_int32), ("pitch", C.c_int64),
                ("x", C.c_int32), ("y", C.c_int32), ("w", C.c_int32), ("h", C.c_int32),
                ("ow", C.c_int32), ("oh", C.c_int32), ("dst", C.c_void_p),
                ("v64", C.c_void_p), ("smax", C.c_void_p)]


def build(force: bool = False) -> str:
    """Compile fk_oracle.c with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off",
                               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        L.orc_run.argtypes = [C.POINTER(_Chain), C.POINTER(_Item), C.c_int32]
        L.orc_validate.argtypes = [C.POINTER(_Chain), C.POINTER(_Item), C.c_int32]
        L.orc_resize_f32.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                     C.c_int32, C.c_int32]
        L.orc_half_to_float.argtypes = [C.c_uint16]
        L.orc_half_to_float.restype = C.c_float
        L.orc_float_to_half.argtypes = [C.c_float]
        L.orc_float_to_half.restype = C.c_uint16
        _lib = L
    return _lib


def _chain_struct(chain: dict):
    ops = chain["ops"]
    arr = (_Op * max(1, len(ops)))()
    for i, op in enumerate(ops):
        arr[i].kind = _OP[op["kind"]]
        ks = list(op.get("k", []))
        arr[i].nconst = len(ks)
        for j, v in enumerate(ks[:4]):
            arr[i].k[j] = v
        arr[i].span = op.get("span", 0)
        arr[i].count = op.get("count", 0)
    ch = _Chain()
    ch.read_kind = _READ[chain["read"]["kind"]]
    ch.in_dtype = _DT[chain["read"]["dtype"]]
    ch.channels = chain["read"]["channels"]
    ch.ops = arr
    ch.n_ops = len(ops)
    ch.out_dtype = _DT[chain["write"]["dtype"]]
    ch.layout = _LAYOUT[chain["write"]["layout"]]
    return ch, arr


def _frame_hw(chain: dict, fr: np.ndarray) -> tuple:
    """Image height and width of a frame array; an NV12 frame is held as
    (3H/2, W) bytes (luma rows, then chroma rows)."""
    if chain["read"]["kind"] in _NV12:
        return fr.shape[0] * 2 // 3, fr.shape[1]
    return fr.shape[0], fr.shape[1]


def out_shape(chain: dict, item: dict) -> tuple:
    C_ = chain["read"]["channels"]
    if chain["write"]["layout"] == "stats":
        return (C_, 4)  # per channel: min, max, sum, mean
    if chain["read"]["kind"] in _RESIZING:
        oh, ow = item["out_h"], item["out_w"]
    else:
        oh, ow = item["h"], item["w"]
    return (C_, oh, ow) if chain["write"]["layout"] == "planar" else (oh, ow, C_)


def run_chain(chain: dict, frames: list, items: list, shadow: bool = True) -> list:
    """Run `chain` on each item.  Returns one dict per item with ``out`` (the
    chain's output dtype and layout), and, if `shadow`, ``v64`` (fp64 shadow)
    and ``smax`` (largest |value| the element took), same shape as ``out``.
    A stats write gives ``out`` of shape (C, 4) = per channel min, max, sum,
    mean, and no shadow.  Raises ValueError if the oracle rejects the chain
    or an item."""
    L = lib()
    shadow = shadow and chain["write"]["layout"] != "stats"
    ch, _keep = _chain_struct(chain)
    frames = [np.ascontiguousarray(f) for f in frames]
    results = []
    structs = (_Item * max(1, len(items)))()
    for b, it in enumerate(items):
        fr = frames[it["frame"]]
        shape = out_shape(chain, it)
        res = {"out": np.zeros(shape, dtype=_NP_OUT[chain["write"]["dtype"]])}
        if shadow:
            res["v64"] = np.zeros(shape, dtype=np.float64)
            res["smax"] = np.zeros(shape, dtype=np.float32)
        s = structs[b]
        s.src = fr.ctypes.data
        s.H, s.W = _frame_hw(chain, fr)
        s.pitch = fr.strides[0]
        s.x, s.y, s.w, s.h = it["x"], it["y"], it["w"], it["h"]
        s.ow, s.oh = it.get("out_w", it["w"]), it.get("out_h", it["h"])
        s.dst = res["out"].ctypes.data
        s.v64 = res["v64"].ctypes.data if shadow else None
        s.smax = res["smax"].ctypes.data if shadow else None
        results.append(res)
    rc = L.orc_run(C.byref(ch), structs, len(items))
    if rc != 0:
        raise ValueError(f"oracle rejected the chain or an item (status {rc})")
    return results


def validate(chain: dict, frames: list, items: list) -> int:
    """Status of the oracle's argument check (0 = valid, negative = invalid)."""
    L = lib()
    ch, _keep = _chain_struct(chain)
    structs = (_Item * max(1, len(items)))()
    dummy = np.zeros(1, np.uint8)
    for b, it in enumerate(items):
        fr = frames[it["frame"]]
        s = structs[b]
        s.src = fr.ctypes.data
        s.H, s.W = _frame_hw(chain, fr)
        s.pitch = fr.strides[0]
        s.x, s.y, s.w, s.h = it["x"], it["y"], it["w"], it["h"]
        s.ow, s.oh = it.get("out_w", it["w"]), it.get("out_h", it["h"])
        s.dst = dummy.ctypes.data
    return int(L.orc_validate(C.byref(ch), structs, len(items)))


def resize_f32(src: np.ndarray, out_w: int, out_h: int) -> np.ndarray:
    """The resize step alone on a packed (h, w, C) fp32 image."""
    src = np.ascontiguousarray(src, dtype=np.float32)
    if src.ndim == 2:
        src = src[:, :, None]
    h, w, c = src.shape
    dst = np.zeros((out_h, out_w, c), np.float32)
    rc = lib().orc_resize_f32(src.ctypes.data, w, h, c, dst.ctypes.data, out_w, out_h)
    if rc != 0:
        raise ValueError("bad resize arguments")
    return dst


def half_to_float(bits: np.ndarray) -> np.ndarray:
    L = lib()
    return np.array([L.orc_half_to_float(int(b)) for b in np.asarray(bits).ravel()], np.float32)


def float_to_half(vals: np.ndarray) -> np.ndarray:
    L = lib()
    return np.array([L.orc_float_to_half(float(v)) for v in np.asarray(vals, np.float32).ravel()],
                    np.uint16)
