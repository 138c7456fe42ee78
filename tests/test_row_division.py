"""The kernels' row division (CPU only): a work-unit index u is split into
row u // d and column by a double-precision reciprocal estimate corrected
once by 24-bit integer products (RowDiv in the device header).  This test
restates it in IEEE double arithmetic (the GPU's fp64 divide and multiply
are correctly rounded, the conversion truncates) and checks it exact
against integer division on random and edge cases over the whole range the
kernels use: d < 2^16 indices per row, fewer than 2^16 rows (output and
frame sides are at most 65535) and u < 2^28.  It also checks the
restatement against the source text, and that quotients of 2^16 and more,
which the kernels never form, are outside what the 24-bit products hold."""
import os
import re

import numpy as np

D_MAX = (1 << 16) - 1
ROWS_MAX = (1 << 16) - 1
U_MAX = 1 << 28


def umul24(a, b):
    return ((a & 0xFFFFFF) * (b & 0xFFFFFF)) & 0xFFFFFFFF


def rowdiv(u, d):
    """u, d: int64 arrays; returns the quotients as the device code does."""
    rcp = 1.0 / d.astype(np.float64)
    q = (u.astype(np.float64) * rcp).astype(np.int64)  # truncation toward zero
    up = umul24(q + 1, d) <= u
    down = ~up & (umul24(q, d) > u)
    return q + up - down


def check(u, d):
    got = rowdiv(u, d)
    want = u // d
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(int(u[i]), int(d[i]), int(got[i]), int(want[i])) for i in bad[:5]]


def test_random_indices_and_row_lengths():
    g = np.random.default_rng(7)
    for _ in range(10):
        d = g.integers(1, D_MAX + 1, size=1_000_000, dtype=np.int64)
        rows = g.integers(1, ROWS_MAX + 1, size=d.size, dtype=np.int64)
        limit = np.minimum(d * rows, U_MAX)
        u = (g.random(d.size) * limit).astype(np.int64)
        check(u, d)


def test_row_boundaries_and_extremes():
    g = np.random.default_rng(8)
    ds = np.concatenate([np.arange(1, 2050), [2 ** k + e for k in range(11, 16) for e in (-1, 0, 1)],
                         [D_MAX, D_MAX - 1, 3 * 5 * 7 * 11 * 13, 960, 1920, 3840 // 4, 65521],
                         g.integers(1, D_MAX + 1, size=2000)]).astype(np.int64)
    ds = ds[(ds >= 1) & (ds <= D_MAX)]
    for d in ds:
        kmax = min((U_MAX - 1) // int(d), ROWS_MAX - 1)
        ks = np.unique(np.concatenate([np.arange(0, 64), kmax - np.arange(0, 64),
                                       g.integers(0, kmax + 1, size=256)]))
        ks = ks[(ks >= 0) & (ks <= kmax)]
        u = np.concatenate([ks * d - 1, ks * d, ks * d + 1, ks * d + d - 1])
        u = u[(u >= 0) & (u < U_MAX) & (u // d <= ROWS_MAX - 1)]
        check(u, np.full(u.shape, d, dtype=np.int64))


def test_restatement_matches_the_device_source():
    src = open(os.path.join(os.path.dirname(__file__), "..", "paper_2508_07071_amd", "csrc",
                            "fk_device.hpp")).read()
    body = re.sub(r"\s+", " ", src[src.index("struct RowDiv {"):src.index("};", src.index("struct RowDiv {"))])
    for line in ("rcp(1.0 / (double)d)", "uint32_t q = (uint32_t)((double)u * rcp);",
                 "if (__umul24(q + 1, upr) <= u) ++q;", "else if (__umul24(q, upr) > u) --q;"):
        assert line in body, line


def test_quotients_beyond_the_row_limit_are_outside_the_domain():
    """Why the row limit matters: with 2^24 or more in a 24-bit product the
    correction breaks (u = 2^25, d = 2 gives a wrong row), which the item
    limits rule out."""
    u = np.array([1 << 25], dtype=np.int64)
    d = np.array([2], dtype=np.int64)
    assert rowdiv(u, d)[0] != u[0] // d[0]
