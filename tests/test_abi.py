"""The C ABI library on the host: it loads next to torch's HIP runtime,
exports every symbol include/fk.h declares, and rejects bad chains and
items before any device work (no GPU needed)."""
import ctypes as C
import os
import re

import pytest
import torch

import paper_2508_07071_amd as fk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "fk.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fk_\w+)\s*\(", text)))


def test_library_loads_with_one_hip_runtime():
    L = fk.lib()
    assert L is not None
    runtimes = fk._hip_runtimes()
    assert len(runtimes) <= 1
    assert "gfx950" in fk.fk_version()


def test_exports_every_declared_symbol():
    declared = header_functions()
    assert declared, "no declarations parsed"
    L = fk.lib()
    for name in declared:
        assert hasattr(L, name), f"{name} declared in fk.h but not exported"
    assert sorted(fk.EXPORTS) == declared


def test_status_strings():
    assert fk.fk_status_string(fk.FK_OK) == "ok"
    assert fk.fk_status_string(fk.FK_ERR_INVALID_ARG) == "invalid argument"
    assert fk.fk_status_string(fk.FK_ERR_HIP) == "HIP error"
    assert fk.fk_status_string(12345) == "unknown status"


def norm_chain():
    import datagen
    return datagen.normalize_chain(64, 128)


@pytest.mark.parametrize("mutate,status", [
    (lambda c: c["read"].update(kind="warp"), None),
    (lambda c: c["read"].update(channels=2), fk.FK_ERR_UNSUPPORTED),
    (lambda c: c["write"].update(dtype="u8"), fk.FK_ERR_UNSUPPORTED),
    (lambda c: c["ops"].__setitem__(2, {"kind": "mul", "k": [1.0, 2.0]}), fk.FK_ERR_INVALID_ARG),
    (lambda c: c["ops"].__setitem__(0, {"kind": "swap", "k": [1.0]}), fk.FK_ERR_INVALID_ARG),
])
def test_chain_validation_rejects(mutate, status):
    c = norm_chain()
    assert fk.fk_chain_validate(fk.chain_desc(c)) == fk.FK_OK
    try:
        mutate(c)
        d = fk.chain_desc(c)
    except KeyError:
        # unknown names cannot even be marshalled: build the bad code directly
        d = fk.chain_desc(norm_chain())
        d.read.kind = 7
        status = fk.FK_ERR_INVALID_ARG
    assert fk.fk_chain_validate(d) == status
    assert fk.fk_last_error()


def test_chain_validation_limits():
    d = fk.chain_desc(norm_chain())
    d.n_ops = 5000
    assert fk.fk_chain_validate(d) == fk.FK_ERR_INVALID_ARG
    d = fk.chain_desc(norm_chain())
    d.ops = None
    assert fk.fk_chain_validate(d) == fk.FK_ERR_INVALID_ARG
    assert fk.lib().fk_chain_validate(None) == fk.FK_ERR_INVALID_ARG


def fake_items(chain, n=1, **kw):
    arr = (fk.fk_item * n)()
    for a in arr:
        a.src.ptr = 0x10000
        a.src.width, a.src.height = 640, 480
        a.src.pitch_bytes = 640 * 3
        a.x, a.y, a.w, a.h = 10, 20, 100, 80
        a.dst = 0x20000
        a.out_w, a.out_h = 64, 128
        for k, v in kw.items():
            if k in ("ptr", "width", "height", "pitch_bytes"):
                setattr(a.src, k, v)
            else:
                setattr(a, k, v)
    return arr


@pytest.mark.parametrize("kw", [dict(x=-1), dict(y=-1), dict(w=0), dict(h=0), dict(x=541), dict(y=401),
                                dict(pitch_bytes=100), dict(ptr=None), dict(dst=None), dict(out_w=0),
                                dict(width=0)])
def test_item_validation_rejects(kw):
    d = fk.chain_desc(norm_chain())
    assert fk.fk_items_validate(d, fake_items(norm_chain()), 1) == fk.FK_OK
    assert fk.fk_items_validate(d, fake_items(norm_chain(), **kw), 1) == fk.FK_ERR_INVALID_ARG


def test_plain_read_output_size_must_match_roi():
    import datagen
    c = datagen.muladd_chain(4, datagen.rng(0))
    d = fk.chain_desc(c)
    assert fk.fk_items_validate(d, fake_items(c, out_w=0, out_h=0), 1) == fk.FK_OK
    assert fk.fk_items_validate(d, fake_items(c, out_w=100, out_h=80), 1) == fk.FK_OK
    assert fk.fk_items_validate(d, fake_items(c, out_w=64, out_h=128), 1) == fk.FK_ERR_INVALID_ARG


def test_autotune_space_order():
    space = fk.fk_autotune_space()
    assert len(space) == 20
    got = [(c.block_threads, c.coarsen) for c in space]
    assert got == [(t, k) for t in (64, 128, 256, 512, 1024) for k in (1, 2, 4, 8)]


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-GPU error path")
def test_plan_create_without_gpu_fails_cleanly():
    d = fk.chain_desc(norm_chain())
    with pytest.raises(fk.FKError) as e:
        fk.fk_plan_create(d, 4)
    assert e.value.status == fk.FK_ERR_HIP


LOOP_CASES = [
    ([{"kind": "mul", "k": [2.0]}, {"kind": "add", "k": [1.0]}, {"kind": "loop", "span": 2, "count": 9}], True),
    ([{"kind": "mul", "k": [2.0]}, {"kind": "loop", "span": 1, "count": 1}], True),
    ([{"kind": "cvt", "k": []}, {"kind": "div", "k": [3.0]}, {"kind": "loop", "span": 1, "count": 1 << 30},
      {"kind": "swap", "k": []}], True),
    ([{"kind": "loop", "span": 1, "count": 2}], False),
    ([{"kind": "mul", "k": [2.0]}, {"kind": "loop", "span": 2, "count": 2}], False),
    ([{"kind": "mul", "k": [2.0]}, {"kind": "loop", "span": 1, "count": 0}], False),
    ([{"kind": "swap", "k": []}, {"kind": "mul", "k": [2.0]}, {"kind": "loop", "span": 2, "count": 2}], False),
    ([{"kind": "cvt", "k": []}, {"kind": "loop", "span": 1, "count": 2}], False),
    ([{"kind": "mul", "k": [2.0]}, {"kind": "loop", "span": 1, "count": 2}, {"kind": "loop", "span": 2, "count": 2}],
     False),
    ([{"kind": "mul", "k": [2.0]}, {"kind": "loop", "span": 1, "count": 2, "k": [1.0]}], False),
]


@pytest.mark.parametrize("ops,ok", LOOP_CASES)
def test_loop_validation_agrees_with_oracle(ops, ok):
    import numpy as np
    import oracle
    ch = {"read": {"kind": "plain", "dtype": "u8", "channels": 3, "out_w": 0, "out_h": 0},
          "ops": ops, "write": {"dtype": "f32", "layout": "packed"}}
    lib_ok = fk.fk_chain_validate(fk.chain_desc(ch)) == fk.FK_OK
    fr = np.zeros((4, 4, 3), np.uint8)
    orc_ok = oracle.validate(ch, [fr], [{"frame": 0, "x": 0, "y": 0, "w": 4, "h": 4}]) == 0
    assert lib_ok == orc_ok == ok


@pytest.mark.parametrize("dtype,layout,ok", [
    ("f64", "stats", fk.FK_OK), ("f32", "stats", fk.FK_ERR_UNSUPPORTED),
    ("f64", "planar", fk.FK_ERR_UNSUPPORTED), ("f64", "packed", fk.FK_ERR_UNSUPPORTED),
])
def test_stats_write_validation(dtype, layout, ok):
    c = norm_chain()
    c["write"] = {"dtype": dtype, "layout": layout}
    assert fk.fk_chain_validate(fk.chain_desc(c)) == ok


@pytest.mark.parametrize("kind,dtype,C,ok", [
    ("nv12", "u8", 3, fk.FK_OK), ("nv12_resize", "u8", 3, fk.FK_OK), ("crop_nearest", "f16", 4, fk.FK_OK),
    ("nv12", "u8", 1, fk.FK_ERR_INVALID_ARG), ("nv12_resize", "f32", 3, fk.FK_ERR_INVALID_ARG),
])
def test_read_kind_validation(kind, dtype, C, ok):
    c = {"read": {"kind": kind, "dtype": dtype, "channels": C, "out_w": 0, "out_h": 0},
         "ops": [{"kind": "cvt", "k": []}], "write": {"dtype": "f32", "layout": "planar"}}
    assert fk.fk_chain_validate(fk.chain_desc(c)) == ok


def test_nv12_items_need_even_frames():
    c = {"read": {"kind": "nv12", "dtype": "u8", "channels": 3, "out_w": 0, "out_h": 0},
         "ops": [], "write": {"dtype": "f32", "layout": "packed"}}
    d = fk.chain_desc(c)
    it = (fk.fk_item * 1)()
    it[0].src.ptr, it[0].src.width, it[0].src.height, it[0].src.pitch_bytes = 4096, 64, 48, 64
    it[0].x, it[0].y, it[0].w, it[0].h, it[0].dst = 0, 0, 8, 8, 8192
    assert fk.lib().fk_items_validate(C.byref(d), it, 1) == fk.FK_OK
    it[0].src.width = 63
    assert fk.lib().fk_items_validate(C.byref(d), it, 1) == fk.FK_ERR_INVALID_ARG


@pytest.mark.parametrize("kw,status", [
    (dict(out_w=65535, out_h=2), fk.FK_OK),
    (dict(out_w=65536, out_h=1), fk.FK_ERR_UNSUPPORTED),
    (dict(out_w=4, out_h=1 << 25), fk.FK_ERR_UNSUPPORTED),
    (dict(width=65536, pitch_bytes=65536 * 3), fk.FK_ERR_UNSUPPORTED),
    (dict(out_w=65535, out_h=65535), fk.FK_ERR_UNSUPPORTED),  # above 2^28 pixels
])
def test_resize_output_sides_are_limited(kw, status):
    # the kernels take output rows and columns through 24-bit multiplies:
    # sides above 65535 must be refused, not computed wrongly
    d = fk.chain_desc(norm_chain())
    assert fk.fk_items_validate(d, fake_items(norm_chain(), **kw), 1) == status


def test_mlp_raw_exports_reject_bad_arguments():
    L = fk.lib()
    assert L.fk_mlp_workspace_floats(None, 4) == -1
    assert L.fk_mlp_forward(None, None, 1, None, None, None) == fk.FK_ERR_INVALID_ARG
    assert L.fk_mlp_backward(None, None, 1, None, None, None, None) == fk.FK_ERR_INVALID_ARG
    assert L.fk_mlp_mse(None, None, 1, None, None, None) == fk.FK_ERR_INVALID_ARG
    assert L.fk_mlp_step(None, None, 1e-3, None) == fk.FK_ERR_INVALID_ARG
    assert L.fk_model_train_device(None, None, None, 4, 1, 4, 1e-3, 0, None, None) == fk.FK_ERR_INVALID_ARG


def test_server_calls_reject_null():
    L = fk.lib()
    n = C.c_int32()
    assert L.fk_server_poll(None, None, 0, C.byref(n)) == fk.FK_ERR_INVALID_ARG
    assert L.fk_server_release(None, 1) == fk.FK_ERR_INVALID_ARG
    assert L.fk_server_destroy(None) == fk.FK_OK


class TestMakeItemsChecks:
    """make_items refuses tensors the library would read or write wrongly
    (checked before the device, so CPU tensors exercise each rule)."""

    def cfg(self):
        import datagen
        chain = datagen.normalize_chain(64, 128)
        item = {"frame": 0, "x": 0, "y": 0, "w": 32, "h": 16, "out_w": 64, "out_h": 128}
        return chain, item

    def test_strided_frame_view_is_refused(self):
        chain, item = self.cfg()
        fr = torch.zeros(16, 64, 3, dtype=torch.uint8)[:, ::2, :]  # column stride 6
        out = torch.zeros(3, 128, 64)
        with pytest.raises(ValueError, match="packed"):
            fk.make_items(chain, [fr], [item], [out])

    def test_channel_last_transposed_frame_is_refused(self):
        chain, item = self.cfg()
        fr = torch.zeros(3, 16, 32, dtype=torch.uint8).permute(1, 2, 0)  # (16, 32, 3), stride(2) != 1
        out = torch.zeros(3, 128, 64)
        with pytest.raises(ValueError, match="packed"):
            fk.make_items(chain, [fr], [item], [out])

    def test_frame_dtype_must_match_chain(self):
        chain, item = self.cfg()
        fr = torch.zeros(16, 32, 3, dtype=torch.float32)
        out = torch.zeros(3, 128, 64)
        with pytest.raises(ValueError, match="dtype"):
            fk.make_items(chain, [fr], [item], [out])

    def test_output_must_be_contiguous_and_sized(self):
        chain, item = self.cfg()
        fr = torch.zeros(16, 32, 3, dtype=torch.uint8)
        with pytest.raises(ValueError, match="contiguous"):
            fk.make_items(chain, [fr], [item], [torch.zeros(3, 64, 128).transpose(1, 2)])
        with pytest.raises(ValueError, match="elements"):
            fk.make_items(chain, [fr], [item], [torch.zeros(3, 127, 64)])
        with pytest.raises(ValueError, match="dtype"):
            fk.make_items(chain, [fr], [item], [torch.zeros(3, 128, 64, dtype=torch.float16)])

    def test_host_tensors_are_refused(self):
        chain, item = self.cfg()
        fr = torch.zeros(16, 32, 3, dtype=torch.uint8)
        with pytest.raises(ValueError, match="device"):
            fk.make_items(chain, [fr], [item], [torch.zeros(3, 128, 64)])
