"""Python binding of libfkmi.so, the MI355X fused preprocessing-chain library.

Argument marshalling only: every step of a chain runs in the library's HIP
kernels.  The functions keep the C ABI's names (``fk_plan_create``,
``fk_run``, ...) and take ctypes structures or plain Python values; the
helpers ``chain_desc`` and ``make_items`` build those structures from the
chain/item dicts used throughout the project, with torch tensors as device
buffers.  PyTorch provides device memory and streams only.

The library is loaded after ``import torch`` so that both share torch's HIP
runtime; loading fails loudly if the library is missing or if two HIP
runtimes end up in the process.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (must own the process's HIP runtime before the library loads)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfkmi.so")

FK_OK = 0
FK_ERR_INVALID_ARG = -1
FK_ERR_UNSUPPORTED = -2
FK_ERR_OUT_OF_MEMORY = -3
FK_ERR_HIP = -4
FK_ERR_BAD_STATE = -5
FK_ERR_BUDGET = -6

FK_U8, FK_F16, FK_F32, FK_F64 = 0, 1, 2, 3
FK_PACKED, FK_PLANAR, FK_STATS = 0, 1, 2
FK_READ_PLAIN, FK_READ_CROP_RESIZE, FK_READ_CROP_NEAREST, FK_READ_NV12, FK_READ_NV12_RESIZE = range(5)
FK_OP_SWAP_RB, FK_OP_CVT_F32, FK_OP_MUL, FK_OP_ADD, FK_OP_SUB, FK_OP_DIV, FK_OP_LOOP = range(7)
FK_CONFIG_DEFAULT, FK_CONFIG_MANUAL, FK_CONFIG_AUTOTUNE, FK_CONFIG_MODEL = range(4)
FK_TIER_AUTO, FK_TIER_RUNTIME = 0, 1
FK_GATHER_DIRECT, FK_GATHER_LDS = 0, 1

DTYPE = {"u8": FK_U8, "f16": FK_F16, "f32": FK_F32, "f64": FK_F64}
LAYOUT = {"packed": FK_PACKED, "planar": FK_PLANAR, "stats": FK_STATS}
READ = {"plain": FK_READ_PLAIN, "crop_resize": FK_READ_CROP_RESIZE, "crop_nearest": FK_READ_CROP_NEAREST,
        "nv12": FK_READ_NV12, "nv12_resize": FK_READ_NV12_RESIZE}
RESIZING = ("crop_resize", "crop_nearest", "nv12_resize")
NV12 = ("nv12", "nv12_resize")
OP = {"swap": FK_OP_SWAP_RB, "cvt": FK_OP_CVT_F32, "mul": FK_OP_MUL, "add": FK_OP_ADD,
      "sub": FK_OP_SUB, "div": FK_OP_DIV, "loop": FK_OP_LOOP}
TORCH_DTYPE = {"u8": torch.uint8, "f16": torch.float16, "f32": torch.float32, "f64": torch.float64}


class fk_read_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("in_dtype", C.c_int32), ("channels", C.c_int32)]


class fk_op_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_consts", C.c_int32), ("consts", C.c_float * 4),
                ("loop_span", C.c_int32), ("loop_count", C.c_int32)]


class fk_write_desc(C.Structure):
    _fields_ = [("out_dtype", C.c_int32), ("layout", C.c_int32)]


class fk_chain_desc(C.Structure):
    _fields_ = [("read", fk_read_desc), ("ops", C.POINTER(fk_op_desc)), ("n_ops", C.c_int32),
                ("write", fk_write_desc)]


class fk_image(C.Structure):
    _fields_ = [("ptr", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32),
                ("pitch_bytes", C.c_int64)]


class fk_item(C.Structure):
    _fields_ = [("src", fk_image), ("x", C.c_int32), ("y", C.c_int32), ("w", C.c_int32),
                ("h", C.c_int32), ("dst", C.c_void_p), ("out_w", C.c_int32), ("out_h", C.c_int32)]


class fk_launch_config(C.Structure):
    _fields_ = [("block_threads", C.c_int32), ("coarsen", C.c_int32)]

    def __repr__(self):
        return f"fk_launch_config({self.block_threads}, {self.coarsen})"


class fk_plan_opts(C.Structure):
    _fields_ = [("config_source", C.c_int32), ("manual", fk_launch_config), ("use_graph", C.c_int32),
                ("strict_fp", C.c_int32), ("tier", C.c_int32), ("unfused_loop_kernel", C.c_int32),
                ("gather", C.c_int32)]


class fk_crop(C.Structure):
    _fields_ = [("x", C.c_int32), ("y", C.c_int32), ("w", C.c_int32), ("h", C.c_int32),
                ("out_w", C.c_int32), ("out_h", C.c_int32)]


class fk_request(C.Structure):
    _fields_ = [("frame", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32),
                ("pitch_bytes", C.c_int64), ("crops", C.POINTER(fk_crop)), ("n_crops", C.c_int32),
                ("t_arrival", C.c_double), ("frame_on_device", C.c_int32)]


class fk_server_opts(C.Structure):
    _fields_ = [("chain", C.POINTER(fk_chain_desc)), ("arena", C.c_void_p), ("arena_bytes", C.c_int64),
                ("budget_bytes", C.c_int64), ("max_batch_items", C.c_int32), ("max_inflight", C.c_int32),
                ("mode", C.c_int32), ("strict_fp", C.c_int32), ("config", fk_launch_config)]


class fk_completion(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int32), ("n_crops", C.c_int32),
                ("outputs", C.c_void_p), ("output_bytes", C.c_int64), ("t_arrival", C.c_double),
                ("t_admit", C.c_double), ("t_launch", C.c_double), ("t_done", C.c_double)]


class fk_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("launches", C.c_int64), ("crops_launched", C.c_int64), ("bytes_in_use", C.c_int64),
                ("peak_bytes", C.c_int64), ("pending", C.c_int64)]


FK_SERVER_BATCHED, FK_SERVER_PER_REQUEST, FK_SERVER_UNFUSED = 0, 1, 2


class FKError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def _hip_runtimes() -> set:
    with open("/proc/self/maps") as f:
        return {ln.split()[-1] for ln in f if "libamdhip64" in ln}


def lib():
    """Load libfkmi.so (built by ``__graft_entry__.build()``).  Raises if it
    is missing: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise ImportError(f"more than one HIP runtime loaded: {sorted(runtimes)}")
    P = C.c_void_p
    sig = {
        "fk_status_string": ([C.c_int32], C.c_char_p),
        "fk_last_error": ([], C.c_char_p),
        "fk_version": ([], C.c_char_p),
        "fk_chain_validate": ([C.POINTER(fk_chain_desc)], C.c_int32),
        "fk_items_validate": ([C.POINTER(fk_chain_desc), C.POINTER(fk_item), C.c_int32], C.c_int32),
        "fk_plan_create": ([C.POINTER(fk_chain_desc), C.c_int32, C.POINTER(fk_plan_opts),
                            C.POINTER(P)], C.c_int32),
        "fk_plan_destroy": ([P], C.c_int32),
        "fk_plan_get_config": ([P, C.POINTER(fk_launch_config)], C.c_int32),
        "fk_plan_set_config": ([P, C.POINTER(fk_launch_config)], C.c_int32),
        "fk_plan_get_tier": ([P, C.POINTER(C.c_int32)], C.c_int32),
        "fk_run": ([P, C.POINTER(fk_item), C.c_int32, P], C.c_int32),
        "fk_run_timed": ([P, C.POINTER(fk_item), C.c_int32, P, P, P], C.c_int32),
        "fk_unfused_scratch_bytes": ([P, C.POINTER(fk_item), C.c_int32, C.POINTER(C.c_int64)],
                                     C.c_int32),
        "fk_run_unfused": ([P, C.POINTER(fk_item), C.c_int32, P, C.c_int64, P], C.c_int32),
        "fk_run_unfused_noalloc": ([P, C.POINTER(fk_item), C.c_int32, P], C.c_int32),
        "fk_autotune_space": ([C.POINTER(fk_launch_config), C.c_int32], C.c_int32),
        "fk_autotune": ([P, C.POINTER(fk_item), C.c_int32, C.c_int32, C.POINTER(C.c_float),
                         C.POINTER(fk_launch_config)], C.c_int32),
        "fk_model_create": ([C.c_int32, C.c_uint64, C.POINTER(P)], C.c_int32),
        "fk_model_destroy": ([P], C.c_int32),
        "fk_model_param_count": ([P], C.c_int64),
        "fk_model_get_params": ([P, P, C.c_int64], C.c_int32),
        "fk_model_set_params": ([P, P, C.c_int64], C.c_int32),
        "fk_model_get_normalization": ([P, P, P], C.c_int32),
        "fk_model_set_normalization": ([P, P, P], C.c_int32),
        "fk_model_features": ([P, C.POINTER(fk_item), C.c_int32, P], C.c_int32),
        "fk_model_train": ([P, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_uint64, P],
                           C.c_int32),
        "fk_model_train_device": ([P, P, P, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_uint64,
                                   P, P], C.c_int32),
        "fk_mlp_workspace_floats": ([P, C.c_int32], C.c_int64),
        "fk_mlp_forward": ([P, P, C.c_int32, P, P, P], C.c_int32),
        "fk_mlp_backward": ([P, P, C.c_int32, P, P, P, P], C.c_int32),
        "fk_mlp_mse": ([P, P, C.c_int32, P, P, P], C.c_int32),
        "fk_mlp_step": ([P, P, C.c_float, P], C.c_int32),
        "fk_model_predict_batch": ([P, P, C.c_int32, P], C.c_int32),
        "fk_model_loss_grad": ([P, P, P, C.c_int32, P, P], C.c_int32),
        "fk_model_predict": ([P, P, C.POINTER(fk_item), C.c_int32, C.POINTER(fk_launch_config)],
                             C.c_int32),
        "fk_plan_use_model": ([P, P, C.POINTER(fk_item), C.c_int32], C.c_int32),
        "fk_model_save": ([P, C.c_char_p], C.c_int32),
        "fk_model_load": ([C.c_char_p, C.POINTER(P)], C.c_int32),
        "fk_server_clock": ([], C.c_double),
        "fk_server_create": ([C.POINTER(fk_server_opts), C.POINTER(P)], C.c_int32),
        "fk_server_submit": ([P, C.POINTER(fk_request), C.POINTER(C.c_uint64)], C.c_int32),
        "fk_server_poll": ([P, C.POINTER(fk_completion), C.c_int32, C.POINTER(C.c_int32)], C.c_int32),
        "fk_server_release": ([P, C.c_uint64], C.c_int32),
        "fk_server_stats_get": ([P, C.POINTER(fk_server_stats)], C.c_int32),
        "fk_server_destroy": ([P], C.c_int32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


# Symbols the header declares; tests check the library exports each one.
EXPORTS = [
    "fk_status_string", "fk_last_error", "fk_version", "fk_chain_validate", "fk_items_validate",
    "fk_plan_create", "fk_plan_destroy", "fk_plan_get_config", "fk_plan_set_config",
    "fk_plan_get_tier", "fk_run", "fk_run_timed", "fk_unfused_scratch_bytes", "fk_run_unfused",
    "fk_run_unfused_noalloc",
    "fk_autotune_space", "fk_autotune",
    "fk_model_create", "fk_model_destroy", "fk_model_param_count", "fk_model_get_params",
    "fk_model_set_params", "fk_model_get_normalization", "fk_model_set_normalization",
    "fk_model_features", "fk_model_train", "fk_model_train_device", "fk_mlp_workspace_floats",
    "fk_mlp_forward", "fk_mlp_backward", "fk_mlp_mse", "fk_mlp_step",
    "fk_model_predict_batch", "fk_model_loss_grad",
    "fk_model_predict", "fk_plan_use_model", "fk_model_save", "fk_model_load",
    "fk_server_clock", "fk_server_create", "fk_server_submit", "fk_server_poll", "fk_server_release",
    "fk_server_stats_get", "fk_server_destroy",
]

FK_MODEL_FEATURES = 32
FK_MODEL_OUTPUTS = 20


def check(status: int) -> int:
    if status != FK_OK:
        L = lib()
        raise FKError(status, f"{L.fk_status_string(status).decode()}: {L.fk_last_error().decode()}")
    return status


# ------------------------------------------------------------ marshalling --

def chain_desc(chain: dict):
    """fk_chain_desc for a chain dict; the returned object keeps its op array
    alive (attribute ``_ops``)."""
    ops = chain["ops"]
    arr = (fk_op_desc * max(1, len(ops)))()
    for i, op in enumerate(ops):
        arr[i].kind = OP[op["kind"]]
        ks = list(op.get("k", []))
        arr[i].n_consts = len(ks)
        for j, v in enumerate(ks[:4]):
            arr[i].consts[j] = v
        arr[i].loop_span = op.get("span", 0)
        arr[i].loop_count = op.get("count", 0)
    d = fk_chain_desc()
    d.read.kind = READ[chain["read"]["kind"]]
    d.read.in_dtype = DTYPE[chain["read"]["dtype"]]
    d.read.channels = chain["read"]["channels"]
    d.ops = arr
    d.n_ops = len(ops)
    d.write.out_dtype = DTYPE[chain["write"]["dtype"]]
    d.write.layout = LAYOUT[chain["write"]["layout"]]
    d._ops = arr
    return d


def make_items(chain: dict, frames: list, items: list, outs: list):
    """fk_item array: `frames` are device tensors (H, W, C) (any row pitch in
    their stride; NV12 frames are (3H/2, W) bytes), `outs` device tensors
    receiving each item's output."""
    arr = (fk_item * max(1, len(items)))()
    nv12 = chain["read"]["kind"] in NV12
    for fr in frames:
        _check_frame(chain, fr)
    for b, it in enumerate(items):
        _check_out(chain, it, outs[b])
    if not all(t.is_cuda for t in list(frames) + list(outs[:len(items)])):
        raise ValueError("frames and outputs must be device tensors")
    for b, it in enumerate(items):
        fr = frames[it["frame"]]
        a = arr[b]
        a.src.ptr = fr.data_ptr()
        a.src.height = int(fr.shape[0]) * 2 // 3 if nv12 else int(fr.shape[0])
        a.src.width = int(fr.shape[1])
        a.src.pitch_bytes = int(fr.stride(0)) * fr.element_size()
        a.x, a.y, a.w, a.h = it["x"], it["y"], it["w"], it["h"]
        a.dst = outs[b].data_ptr()
        if chain["read"]["kind"] in RESIZING:
            a.out_w, a.out_h = it["out_w"], it["out_h"]
        else:
            a.out_w, a.out_h = 0, 0
    return arr


def _check_frame(chain: dict, fr) -> None:
    """A frame must be a device tensor of the read's dtype laid out packed
    HWC (rows may carry padding: any stride(0)); NV12 and one-channel frames
    may be 2-D (H, W) with unit column stride."""
    c = chain["read"]["channels"]
    nv12 = chain["read"]["kind"] in NV12
    want = torch.uint8 if nv12 else TORCH_DTYPE[chain["read"]["dtype"]]
    if fr.dim() == 3:
        ok = fr.shape[2] == c and fr.stride(2) == 1 and fr.stride(1) == c and not nv12
    elif fr.dim() == 2:
        ok = (nv12 or c == 1) and fr.stride(1) == 1
    else:
        ok = False
    if not ok:
        raise ValueError(f"frame of shape {tuple(fr.shape)} and strides {fr.stride()} is not a "
                         f"packed {'NV12' if nv12 else f'HWC x{c}'} image")
    if fr.dtype != want:
        raise ValueError(f"frame dtype {fr.dtype}, the chain reads {want}")


def _check_out(chain: dict, item: dict, out) -> None:
    """An output must be a contiguous device tensor of the write's dtype
    holding exactly the item's output elements."""
    want = TORCH_DTYPE[chain["write"]["dtype"]]
    n = 1
    for d in out_shape(chain, item):
        n *= d
    if not out.is_contiguous():
        raise ValueError("outputs must be contiguous")
    if out.dtype != want:
        raise ValueError(f"output dtype {out.dtype}, the chain writes {want}")
    if out.numel() != n:
        raise ValueError(f"output holds {out.numel()} elements, the item writes {n}")


def out_shape(chain: dict, item: dict) -> tuple:
    c = chain["read"]["channels"]
    if chain["write"]["layout"] == "stats":
        return (c, 4)  # per channel: min, max, sum, mean (fp64)
    if chain["read"]["kind"] in RESIZING:
        oh, ow = item["out_h"], item["out_w"]
    else:
        oh, ow = item["h"], item["w"]
    return (c, oh, ow) if chain["write"]["layout"] == "planar" else (oh, ow, c)


def stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# ------------------------------------------------------------- C ABI calls --

def fk_status_string(s: int) -> str:
    return lib().fk_status_string(s).decode()


def fk_last_error() -> str:
    return lib().fk_last_error().decode()


def fk_version() -> str:
    return lib().fk_version().decode()


def fk_chain_validate(desc) -> int:
    return lib().fk_chain_validate(C.byref(desc))


def fk_items_validate(desc, items, n: int) -> int:
    return lib().fk_items_validate(C.byref(desc), items, n)


def fk_plan_create(desc, max_batch: int, opts=None) -> int:
    """Returns the plan handle (an int); raises FKError on failure."""
    h = C.c_void_p()
    check(lib().fk_plan_create(C.byref(desc), max_batch, C.byref(opts) if opts is not None else None,
                               C.byref(h)))
    return h.value


def fk_plan_destroy(plan: int) -> None:
    check(lib().fk_plan_destroy(plan))


def fk_plan_get_config(plan: int) -> fk_launch_config:
    c = fk_launch_config()
    check(lib().fk_plan_get_config(plan, C.byref(c)))
    return c


def fk_plan_set_config(plan: int, cfg: fk_launch_config) -> None:
    check(lib().fk_plan_set_config(plan, C.byref(cfg)))


def fk_plan_get_tier(plan: int) -> int:
    v = C.c_int32()
    check(lib().fk_plan_get_tier(plan, C.byref(v)))
    return v.value


def fk_run(plan: int, items, n: int, stream: int) -> None:
    check(lib().fk_run(plan, items, n, stream))


def fk_run_timed(plan: int, items, n: int, stream: int, start_event: int, stop_event: int) -> None:
    """fk_run whose launch records the two hipEvent_t handles (e.g. a
    torch.cuda.Event's ``cuda_event``) as its kernel starts and ends."""
    check(lib().fk_run_timed(plan, items, n, stream, start_event, stop_event))


def fk_unfused_scratch_bytes(plan: int, items, n: int) -> int:
    v = C.c_int64()
    check(lib().fk_unfused_scratch_bytes(plan, items, n, C.byref(v)))
    return v.value


def fk_run_unfused(plan: int, items, n: int, scratch_ptr: int, scratch_bytes: int, stream: int) -> None:
    check(lib().fk_run_unfused(plan, items, n, scratch_ptr, scratch_bytes, stream))


# workspace the library holds for fk_run_unfused_noalloc (include/fk.h)
FK_NOALLOC_SCRATCH_BYTES = 32 << 20


def fk_run_unfused_noalloc(plan: int, items, n: int, stream: int) -> None:
    """fk_run_unfused with the library's own device workspace (no device
    allocation in the call)."""
    check(lib().fk_run_unfused_noalloc(plan, items, n, stream))


def fk_autotune_space() -> list:
    n = lib().fk_autotune_space(None, 0)
    arr = (fk_launch_config * n)()
    lib().fk_autotune_space(arr, n)
    return [fk_launch_config(a.block_threads, a.coarsen) for a in arr]


def fk_autotune(plan: int, items, n: int, reps: int):
    """Returns (best config, list of 20 median times in ms)."""
    space = lib().fk_autotune_space(None, 0)
    times = (C.c_float * space)()
    best = fk_launch_config()
    check(lib().fk_autotune(plan, items, n, reps, times, C.byref(best)))
    return best, list(times)


# ----------------------------------------------------------- cost model --

def _f32(a):
    import numpy as np
    return np.ascontiguousarray(a, dtype=np.float32)


def fk_model_create(hidden: int = 128, seed: int = 0) -> int:
    h = C.c_void_p()
    check(lib().fk_model_create(hidden, seed, C.byref(h)))
    return h.value


def fk_model_destroy(model: int) -> None:
    check(lib().fk_model_destroy(model))


def fk_model_param_count(model: int) -> int:
    return int(lib().fk_model_param_count(model))


def fk_model_get_params(model: int):
    import numpy as np
    out = np.zeros(fk_model_param_count(model), np.float32)
    check(lib().fk_model_get_params(model, out.ctypes.data, out.size))
    return out


def fk_model_set_params(model: int, params) -> None:
    p = _f32(params)
    check(lib().fk_model_set_params(model, p.ctypes.data, p.size))


def fk_model_get_normalization(model: int):
    import numpy as np
    mean = np.zeros(FK_MODEL_FEATURES, np.float32)
    std = np.zeros(FK_MODEL_FEATURES, np.float32)
    check(lib().fk_model_get_normalization(model, mean.ctypes.data, std.ctypes.data))
    return mean, std


def fk_model_set_normalization(model: int, mean, std) -> None:
    m, s = _f32(mean), _f32(std)
    check(lib().fk_model_set_normalization(model, m.ctypes.data, s.ctypes.data))


def fk_model_features(plan: int, items, n: int):
    import numpy as np
    out = np.zeros(FK_MODEL_FEATURES, np.float32)
    check(lib().fk_model_features(plan, items, n, out.ctypes.data))
    return out


def fk_model_train(model: int, features, targets, epochs: int, batch: int, lr: float, seed: int = 0):
    """Returns the per-epoch mean mini-batch loss."""
    import numpy as np
    x, t = _f32(features), _f32(targets)
    curve = np.zeros(max(epochs, 1), np.float32)
    check(lib().fk_model_train(model, x.ctypes.data, t.ctypes.data, x.shape[0], epochs, batch, lr, seed,
                               curve.ctypes.data))
    return curve[:epochs]


def fk_model_train_device(model: int, d_features, d_targets, epochs: int, batch: int, lr: float,
                          seed: int = 0, d_loss_curve=None, stream=None) -> None:
    """Queue a training run on device tensors (fp32, contiguous) on `stream`
    (default: torch's current stream)."""
    for t in (d_features, d_targets) + ((d_loss_curve,) if d_loss_curve is not None else ()):
        _check_dev_f32(t)
    check(lib().fk_model_train_device(model, d_features.data_ptr(), d_targets.data_ptr(),
                                      d_features.shape[0], epochs, batch, lr, seed,
                                      d_loss_curve.data_ptr() if d_loss_curve is not None else None,
                                      stream_handle(stream)))


def _check_dev_f32(t) -> None:
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 device tensor")


def fk_mlp_workspace_floats(model: int, n: int) -> int:
    v = int(lib().fk_mlp_workspace_floats(model, n))
    if v < 0:
        raise FKError(FK_ERR_INVALID_ARG, "fk_mlp_workspace_floats: bad argument")
    return v


def fk_mlp_forward(model: int, d_x, d_ws, d_y, stream=None) -> None:
    for t in (d_x, d_ws, d_y):
        _check_dev_f32(t)
    check(lib().fk_mlp_forward(model, d_x.data_ptr(), d_x.shape[0], d_ws.data_ptr(), d_y.data_ptr(),
                               stream_handle(stream)))


def fk_mlp_backward(model: int, d_x, d_ws, d_dy, d_grad, stream=None) -> None:
    for t in (d_x, d_ws, d_dy, d_grad):
        _check_dev_f32(t)
    check(lib().fk_mlp_backward(model, d_x.data_ptr(), d_x.shape[0], d_ws.data_ptr(), d_dy.data_ptr(),
                                d_grad.data_ptr(), stream_handle(stream)))


def fk_mlp_mse(d_y, d_t, d_dy, d_loss, stream=None) -> None:
    for t in (d_y, d_t, d_dy, d_loss):
        _check_dev_f32(t)
    check(lib().fk_mlp_mse(d_y.data_ptr(), d_t.data_ptr(), d_y.shape[0], d_dy.data_ptr(),
                           d_loss.data_ptr(), stream_handle(stream)))


def fk_mlp_step(model: int, d_grad, lr: float, stream=None) -> None:
    _check_dev_f32(d_grad)
    check(lib().fk_mlp_step(model, d_grad.data_ptr(), lr, stream_handle(stream)))


def fk_model_predict_batch(model: int, features):
    import numpy as np
    x = _f32(features)
    out = np.zeros((x.shape[0], FK_MODEL_OUTPUTS), np.float32)
    check(lib().fk_model_predict_batch(model, x.ctypes.data, x.shape[0], out.ctypes.data))
    return out


def fk_model_loss_grad(model: int, features, targets):
    import numpy as np
    x, t = _f32(features), _f32(targets)
    loss = np.zeros(1, np.float32)
    grad = np.zeros(fk_model_param_count(model), np.float32)
    check(lib().fk_model_loss_grad(model, x.ctypes.data, t.ctypes.data, x.shape[0], loss.ctypes.data,
                                   grad.ctypes.data))
    return float(loss[0]), grad


def fk_model_predict(model: int, plan: int, items, n: int) -> fk_launch_config:
    c = fk_launch_config()
    check(lib().fk_model_predict(model, plan, items, n, C.byref(c)))
    return c


def fk_plan_use_model(plan: int, model: int, items, n: int) -> None:
    check(lib().fk_plan_use_model(plan, model, items, n))


def fk_model_save(model: int, path: str) -> None:
    check(lib().fk_model_save(model, path.encode()))


def fk_model_load(path: str) -> int:
    h = C.c_void_p()
    check(lib().fk_model_load(path.encode(), C.byref(h)))
    return h.value


# -------------------------------------------------------------- server --

def fk_server_clock() -> float:
    return float(lib().fk_server_clock())


def fk_server_create(opts: fk_server_opts) -> int:
    h = C.c_void_p()
    check(lib().fk_server_create(C.byref(opts), C.byref(h)))
    return h.value


def fk_server_submit(srv: int, req: fk_request) -> int:
    t = C.c_uint64()
    check(lib().fk_server_submit(srv, C.byref(req), C.byref(t)))
    return t.value


def fk_server_poll(srv: int, max_n: int = 256) -> list:
    arr = (fk_completion * max_n)()
    n = C.c_int32()
    check(lib().fk_server_poll(srv, arr, max_n, C.byref(n)))
    return [arr[i] for i in range(n.value)]


def fk_server_release(srv: int, ticket: int) -> None:
    check(lib().fk_server_release(srv, ticket))


def fk_server_stats_get(srv: int) -> fk_server_stats:
    st = fk_server_stats()
    check(lib().fk_server_stats_get(srv, C.byref(st)))
    return st


def fk_server_destroy(srv: int) -> None:
    check(lib().fk_server_destroy(srv))


def server_opts(desc, arena, budget_bytes=0, max_batch_items=1024, max_inflight=3,
                mode=FK_SERVER_BATCHED, strict=False, config=(0, 0)) -> fk_server_opts:
    """Options for fk_server_create; `desc` from chain_desc() (kept alive by
    the returned object), `arena` a uint8 device tensor."""
    o = fk_server_opts()
    o.chain = C.pointer(desc)
    o.arena = arena.data_ptr()
    o.arena_bytes = arena.numel()
    o.budget_bytes = budget_bytes
    o.max_batch_items = max_batch_items
    o.max_inflight = max_inflight
    o.mode = mode
    o.strict_fp = int(bool(strict))
    o.config.block_threads, o.config.coarsen = config
    o._desc = desc
    return o


def make_request(frame, crops, t_arrival=None) -> fk_request:
    """fk_request for a frame tensor (H, W, C) and a list of crop dicts; keeps
    the crop array alive.  A host frame (pinned for async copies) is copied
    by the server; a device frame is read in place (frame_on_device)."""
    arr = (fk_crop * len(crops))()
    for i, c in enumerate(crops):
        arr[i].x, arr[i].y, arr[i].w, arr[i].h = c["x"], c["y"], c["w"], c["h"]
        arr[i].out_w, arr[i].out_h = c["out_w"], c["out_h"]
    r = fk_request()
    r.frame = frame.data_ptr()
    r.height, r.width = int(frame.shape[0]), int(frame.shape[1])
    r.pitch_bytes = int(frame.stride(0)) * frame.element_size()
    r.crops = arr
    r.n_crops = len(crops)
    r.t_arrival = fk_server_clock() if t_arrival is None else t_arrival
    r.frame_on_device = 1 if frame.is_cuda else 0
    r._crops = arr
    return r


def output_offsets(chain: dict, crops) -> list:
    """Byte offset of each crop's output inside a completion's buffer."""
    c = chain["read"]["channels"]
    es = {"f32": 4, "f16": 2}[chain["write"]["dtype"]]
    offs, off = [], 0
    for cr in crops:
        offs.append(off)
        off = (off + cr["out_w"] * cr["out_h"] * c * es + 255) // 256 * 256
    return offs


def plan_opts(config_source=FK_CONFIG_DEFAULT, manual=(256, 1), use_graph=False, strict=False,
              tier=FK_TIER_AUTO, unfused_loop_kernel=False, gather=FK_GATHER_DIRECT) -> fk_plan_opts:
    o = fk_plan_opts()
    o.gather = gather
    o.config_source = config_source
    o.manual.block_threads, o.manual.coarsen = manual
    o.use_graph = int(bool(use_graph))
    o.strict_fp = int(bool(strict))
    o.tier = tier
    o.unfused_loop_kernel = int(bool(unfused_loop_kernel))
    return o
