"""Bounds of the dword-window reads (CPU only).  Three u8 reads fetch a
pixel's bytes as aligned dwords around them: the crop+resize read (a tap
pair, C = 1: 8 bytes, C >= 3: 12 bytes), the nearest read (one pixel of 3
or 4 channels, 8 bytes) and the NV12 resize read (a tap row's luma bytes
and its chroma pairs, 8 bytes each).  A window starts at the dword holding
its first byte, so it reads up to 3 bytes before and several after.  The
LDS-staged gather copies whole 16-byte chunks of the tap rows into LDS and
cuts each tap pair out of two aligned 8-byte LDS reads.  The
kernels use windows only for items their rule admits; this test restates
each rule and checks, over random frames, pitches and ROIs, that every
window an admitted item can issue (every tap column of every ROI row)
covers the bytes it serves and stays inside the frame's tightest
allocation: full rows at the pitch, the last row ending at its pixels."""
import os
import re

import numpy as np

G = np.random.default_rng(2024)


def resize_window_ok(C, fw, fh, x, y, w, h, base=0):
    WB = 8 if C == 1 else 12
    return base % 4 == 0 and C * fw >= WB and (y + h < fh or C * (x + w - 1) + WB <= C * fw)


def nv12_window_ok(fw, fh, x, y, w, h, base=0):
    if base % 4 or fw < 8:
        return False
    last_chroma_row = ((y + h - 1) >> 1) == (fh >> 1) - 1
    return not last_chroma_row or ((x + w - 1) & ~1) + 8 <= fw


def frame_geometry(C, nv12=False):
    fw = int(G.integers(1, 300))
    fh = int(G.integers(1, 40))
    if nv12:
        fw, fh = max(2, fw & ~1), max(2, fh & ~1)
    row = fw * C
    pitch = row + int(G.choice([0, 0, 1, 3, 4, 16]))
    rows = fh + fh // 2 if nv12 else fh
    alloc = (rows - 1) * pitch + row
    return fw, fh, pitch, alloc


def roi(fw, fh):
    x = int(G.integers(0, fw))
    w = int(G.integers(1, fw - x + 1))
    y = int(G.integers(0, fh))
    h = int(G.integers(1, fh - y + 1))
    return x, y, w, h


def test_crop_resize_and_nearest_windows_stay_in_the_frame():
    admitted = 0
    for trial in range(3000):
        C = int(G.choice([1, 3, 4]))
        fw, fh, pitch, alloc = frame_geometry(C)
        x, y, w, h = roi(fw, fh)
        if not resize_window_ok(C, fw, fh, x, y, w, h):
            continue
        admitted += 1
        WB = 8 if C == 1 else 12
        rows = np.arange(y, y + h)[:, None]
        cols = np.arange(x, x + w)[None, :]
        first = rows * pitch + cols * C                # first byte of the tap pair / pixel
        start = first & ~3
        # crop+resize: the pair's 2C bytes (or C when clamped) in [start, start + WB)
        assert np.all(first + 2 * C <= start + WB) or C == 1 and np.all(first + 2 <= start + WB)
        assert start.min() >= 0 and (start + WB).max() <= alloc, (C, fw, fh, pitch, x, y, w, h)
        if C >= 3:
            # nearest: C bytes of one pixel in an 8-byte window, under the same rule
            assert np.all(first + C <= start + 8)
            assert (start + 8).max() <= alloc
    assert admitted > 1000


def test_nv12_resize_windows_stay_in_the_frame():
    admitted = 0
    for trial in range(3000):
        fw, fh, pitch, alloc = frame_geometry(1, nv12=True)
        x, y, w, h = roi(fw, fh)
        if not nv12_window_ok(fw, fh, x, y, w, h):
            continue
        admitted += 1
        Y = np.arange(y, y + h)[:, None]
        X0 = np.arange(x, x + w)[None, :]
        X1 = np.minimum(X0 + 1, x + w - 1)
        luma = Y * pitch + X0
        ls = luma & ~3
        c0 = X0 & ~1
        chroma = (fh + (Y >> 1)) * pitch + c0
        cs = chroma & ~3
        # the luma bytes X0, X1 and the chroma pairs at X0 & ~1, X1 & ~1
        assert np.all(luma + (X1 - X0) < ls + 8)
        assert np.all(chroma + ((X1 & ~1) - c0) + 1 < cs + 8)
        assert ls.min() >= 0 and (ls + 8).max() <= alloc, (fw, fh, pitch, x, y, w, h)
        assert cs.min() >= 0 and (cs + 8).max() <= alloc, (fw, fh, pitch, x, y, w, h)
    assert admitted > 1000


def test_rules_refuse_the_items_that_would_read_past_the_frame():
    """The rules are not vacuous: an item ending on the last row at the
    frame's right edge is refused where its last window would pass the
    end, and admitted once a row below follows."""
    assert not resize_window_ok(3, 100, 10, 90, 0, 10, 10)     # last row, last pixel
    assert resize_window_ok(3, 100, 10, 90, 0, 10, 9)          # a row below follows
    assert not resize_window_ok(3, 100, 10, 0, 0, 1, 1, base=2)
    assert not nv12_window_ok(100, 10, 94, 8, 6, 2)            # last chroma row, right edge
    assert nv12_window_ok(100, 10, 94, 6, 6, 2)                # chroma row 3 of 5: not the last
    assert not nv12_window_ok(6, 10, 0, 0, 6, 2)               # rows under 8 bytes


def test_restated_rules_match_the_kernel_source():
    """The rules above restate the kernels' own conditions; this fails when
    a condition in the device source changes without the restatement."""
    src = open(os.path.join(os.path.dirname(__file__), "..", "paper_2508_07071_amd", "csrc",
                            "fk_device.hpp")).read()
    flat = re.sub(r"\s+", " ", src)
    assert ("(it.src % 4 == 0) && C * (int)it.fw >= WB && "
            "(it.y + it.h < (int)it.fh || C * (it.x + it.w - 1) + WB <= C * (int)it.fw)") in flat
    assert "ReadCropResize<DT_U8, C>::window_ok(it)" in flat
    assert "if ((it.src & 3u) || (int)it.fw < 8) return false;" in flat
    assert "const bool last_chroma_row = (last_y >> 1) == ((int)it.fh >> 1) - 1;" in flat
    assert "return !last_chroma_row || ((it.x + it.w - 1) & ~1) + 8 <= (int)it.fw;" in flat


# ------------------------------------------------- LDS-staged bilinear gather --

def bilinear_taps(o, scale, n):
    """Source indices i0, i1 of output index o: max(fma(o + 0.5, scale,
    -0.5), 0) in fp32 (the product of two fp32 values is exact in double)."""
    s_ = max(float(np.float32((o + 0.5) * float(scale) - 0.5)), 0.0)
    i0 = int(np.floor(s_))
    return i0, min(i0 + 1, n - 1)


def lds_plan(C, fw, fh, pitch, base, x, y, w, h, lds):
    """The staging plan (None where the item reads directly)."""
    if base % 16 or pitch % 16:
        return None
    b0, b1 = x * C, (x + w) * C
    start = b0 & ~15
    end = (b1 + 15) & ~15
    if y + h >= fh and end > fw * C:
        return None
    n16 = (end - start) >> 4
    stride = end - start + 16
    band = lds // (2 * stride)
    return (start, n16, stride, band) if band >= 1 else None


def test_lds_gather_staging_stays_in_the_frame_and_in_lds():
    """Every 16-byte chunk a block stages lies inside the frame's tightest
    allocation; every LDS read (two 8-byte reads per tap row) lies inside
    its staged row's slot and the band inside the block's LDS; the tap
    bytes are among the staged ones."""
    g = np.random.default_rng(11)
    planned = 0
    for trial in range(3000):
        C = int(g.choice([1, 3, 4]))
        fw, fh = int(g.integers(1, 400)), int(g.integers(1, 40))
        pitch = ((fw * C + 15) & ~15) + 16 * int(g.choice([0, 0, 1, 4]))
        x, w = int(g.integers(0, fw)), 0
        w = int(g.integers(1, fw - x + 1))
        y = int(g.integers(0, fh))
        h = int(g.integers(1, fh - y + 1))
        T = int(g.choice([64, 128, 256, 512, 1024]))
        lds = min(T * 128, 65536)
        plan = lds_plan(C, fw, fh, pitch, 0, x, y, w, h, lds)
        if plan is None:
            continue
        planned += 1
        start, n16, stride, band = plan
        alloc = (fh - 1) * pitch + fw * C
        # global chunks of every tap row the item can stage
        for sy in range(y, y + h):
            assert sy * pitch + start >= 0
            assert sy * pitch + start + 16 * n16 <= alloc, (C, fw, fh, pitch, x, y, w, h)
        assert 2 * band * stride <= lds
        ow = int(g.integers(1, 300))
        sx = np.float32(w) / np.float32(ow)
        for ox in range(ow):
            x0, x1 = bilinear_taps(ox, sx, w)
            off = (x + x0) * C - start
            a8 = off & ~7
            assert a8 >= 0 and a8 + 16 <= stride, (off, stride)     # inside the row's slot
            assert off + (2 if x1 != x0 else 1) * C <= 16 * n16      # tap bytes were staged
    assert planned > 1000


def test_lds_restatement_matches_the_device_source():
    src = open(os.path.join(os.path.dirname(__file__), "..", "paper_2508_07071_amd", "csrc",
                            "fk_device.hpp")).read()
    start = src.index("__device__ __forceinline__ bool lds_gather_plan(")
    flat = re.sub(r"\s+", " ", src[start:src.index("return g.band >= 1;", start)])
    for line in ("if ((it.src & 15u) || (it.pitch & 15)) return false;",
                 "g.start = b0 & ~15u;", "const uint32_t end = (b1 + 15u) & ~15u;",
                 "if (it.y + it.h >= (int)it.fh && end > (uint32_t)it.fw * C) return false;",
                 "g.n16 = (end - g.start) >> 4;", "g.stride = end - g.start + 16u;",
                 "g.band = lds / (2u * g.stride);"):
        assert line in flat, line
    internal = open(os.path.join(os.path.dirname(__file__), "..", "paper_2508_07071_amd", "csrc",
                                 "fk_internal.hpp")).read()
    assert "return T * 128u < 65536u ? T * 128u : 65536u;" in internal
