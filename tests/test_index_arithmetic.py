"""Index arithmetic of the kernels (CPU only).

Row division: a work-unit index u is split into
row u // d and column by a double-precision reciprocal estimate corrected
once by 24-bit integer products (RowDiv in the device header).  This test
restates it in IEEE double arithmetic (the GPU's fp64 divide and multiply
are correctly rounded, the conversion truncates) and checks it exact
against integer division on random and edge cases over the whole range the
kernels use: d < 2^16 indices per row, fewer than 2^16 rows (output and
frame sides are at most 65535) and u < 2^28.  It also checks the
restatement against the source text, and that quotients of 2^16 and more,
which the kernels never form, are outside what the 24-bit products hold.

Nearest-neighbour source index: floor((2o + 1) in / (2 out)) from an fp32
estimate of the quotient corrected once by exact 64-bit products
(nearest_index in the device header), restated in numpy float32 (round to
nearest even; the library is built with correctly rounded fp32 division)
and checked exact for every input and output side up to 65535.

Tile to item: the owning batch slot of a tile, by binary search over the
tile offsets with a first probe where equal items would put it
(find_item_guess), against bisection on random batches."""
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


def nearest_index(o, n_in, n_out):
    num = (2 * o + 1) * n_in
    den = 2 * n_out
    est = (num.astype(np.float32) * (np.float32(1.0) / den.astype(np.float32))).astype(np.int64)
    down = est * den > num
    up = ~down & ((est + 1) * den <= num)
    return est - down + up


def test_nearest_index_is_exact():
    g = np.random.default_rng(9)
    n_in = g.integers(1, 65536, size=2_000_000, dtype=np.int64)
    n_out = g.integers(1, 65536, size=n_in.size, dtype=np.int64)
    o = (g.random(n_in.size) * n_out).astype(np.int64)
    edges = []
    for a in (1, 2, 3, 7, 255, 4096, 65534, 65535):
        for b in (1, 2, 3, 5, 224, 4095, 65534, 65535):
            for oo in {0, 1, b // 2, b - 2, b - 1}:
                if 0 <= oo < b:
                    edges.append((oo, a, b))
    e = np.array(edges, dtype=np.int64)
    o, n_in, n_out = (np.concatenate([o, e[:, 0]]), np.concatenate([n_in, e[:, 1]]),
                      np.concatenate([n_out, e[:, 2]]))
    got = nearest_index(o, n_in, n_out)
    want = ((2 * o + 1) * n_in) // (2 * n_out)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(int(o[i]), int(n_in[i]), int(n_out[i]), int(got[i]), int(want[i])) for i in bad[:5]]
    assert (want >= 0).all() and (want < n_in).all()


def test_nearest_restatement_matches_the_device_source():
    src = open(os.path.join(os.path.dirname(__file__), "..", "paper_2508_07071_amd", "csrc",
                            "fk_device.hpp")).read()
    start = src.index("int nearest_index(int o, int in, int out)")
    body = re.sub(r"\s+", " ", src[start:src.index("return q;", start)])
    for line in ("const uint64_t num = (uint64_t)(2 * o + 1) * (uint64_t)in;",
                 "const uint64_t den = 2ull * (uint64_t)out;",
                 "int q = (int)((float)num * (1.0f / (float)den));",
                 "if ((uint64_t)q * den > num) --q;", "else if ((uint64_t)(q + 1) * den <= num) ++q;"):
        assert line in body, line


# ---------------------------------------------------- tile -> item lookup --

def find_item(tb, n, tile):
    lo, hi = 0, n - 1
    while lo < hi:
        mid = (lo + hi + 1) >> 1
        if tb[mid] <= tile:
            lo = mid
        else:
            hi = mid - 1
    return lo


def find_item_guess(tb, n, tile, total):
    if n <= 4:
        return find_item(tb, n, tile)
    lo, hi = 0, n - 1
    g = (tile * n) // total
    if tb[g] <= tile:
        if tb[g + 1] > tile:
            return g
        lo = g + 1
    else:
        hi = g - 1
    while lo < hi:
        mid = (lo + hi + 1) >> 1
        if tb[mid] <= tile:
            lo = mid
        else:
            hi = mid - 1
    return lo


def test_tile_lookup_finds_the_owning_item():
    """Every tile of random batches (equal, uneven and skewed tile counts,
    1 to 1,191 items) maps to the item whose tile range holds it, by the
    plain search and by the search with a first probe."""
    import bisect
    g = np.random.default_rng(12)
    for trial in range(400):
        n = int(g.choice([1, 2, 3, 4, 5, 7, 50, 256, 1191]))
        kind = trial % 3
        if kind == 0:
            counts = np.full(n, int(g.integers(1, 9)))
        elif kind == 1:
            counts = g.integers(1, 40, size=n)
        else:
            counts = np.where(g.random(n) < 0.1, g.integers(100, 1000, size=n), 1)
        tb = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64).tolist()
        total = tb[-1]
        tiles = range(total) if total <= 4000 else g.integers(0, total, size=4000).tolist()
        for t in tiles:
            want = bisect.bisect_right(tb, t) - 1
            assert find_item(tb, n, t) == want
            assert find_item_guess(tb, n, t, total) == want, (n, t, total)


def test_tile_lookup_restatement_matches_the_device_source():
    src = open(os.path.join(os.path.dirname(__file__), "..", "paper_2508_07071_amd", "csrc",
                            "fk_device.hpp")).read()
    start = src.index("int find_item_guess(")
    flat = re.sub(r"\s+", " ", src[start:src.index("return lo;", start)])
    for line in ("if (n_items <= 4) return find_item(tb, n_items, tile);",
                 "const int g = (int)(((uint64_t)tile * (uint64_t)n_items) / total);",
                 "if (tb[g] <= tile) { if (tb[g + 1] > tile) return g; lo = g + 1; } else { hi = g - 1; }",
                 "const int mid = (lo + hi + 1) >> 1; if (tb[mid] <= tile) lo = mid; else hi = mid - 1;"):
        assert line in flat, line
