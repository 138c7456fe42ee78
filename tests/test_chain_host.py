"""Plan-time chain rewriting (host C++, built here with g++): the run-time
tier's normalised op list must compute what the chain computes.  The list
is evaluated here in numpy fp32, one IEEE operation per op, and compared
with the oracle on the same frames: bit for bit in the strict mode, within
the fp32 tolerance when MUL+ADD pairs are contracted to FMA."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import datagen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_07071_amd", "csrc")
KINDS = {k: i for i, k in enumerate(datagen.OP_KINDS)}  # same order as FK_OP_*

DRIVER = r"""
#include "fk_chain.hpp"
#include <cstdio>
#include <vector>
int main() {
    int C, n, strict, rk, dt, odt, lay;
    while (std::scanf("%d %d %d %d %d %d %d", &C, &n, &strict, &rk, &dt, &odt, &lay) == 7) {
        std::vector<fk_op_desc> ops(n);
        for (auto &o : ops)
            std::scanf("%d %d %a %a %a %a %d %d", &o.kind, &o.n_consts, &o.consts[0], &o.consts[1],
                       &o.consts[2], &o.consts[3], &o.loop_span, &o.loop_count);
        fk_chain_desc ch{};
        ch.read.kind = rk; ch.read.in_dtype = dt; ch.read.channels = C;
        ch.ops = ops.data(); ch.n_ops = n;
        ch.write.out_dtype = odt; ch.write.layout = lay;
        std::vector<fk::OpRec> rec;
        int32_t swap = 0;
        fk::normalise_chain(&ch, strict != 0, rec, swap);
        std::vector<float> k;
        int sn = 0;
        int fam = fk::match_static(&ch, k, sn);
        double cnt[4];
        fk::executed_counts(rec, cnt);
        std::printf("%d %zu %d %d %zu %.0f %.0f %.0f %.0f\n", swap, rec.size(), fam, sn, k.size(), cnt[0],
                    cnt[1], cnt[2], cnt[3]);
        for (auto &r : rec)
            std::printf("%d %a %a %a %a %a %a %a %a %d %d\n", r.code, r.a[0], r.a[1], r.a[2], r.a[3],
                        r.b[0], r.b[1], r.b[2], r.b[3], r.span, r.count);
        for (float v : k) std::printf("%a\n", v);
    }
    return 0;
}
"""

OPC_MUL, OPC_ADD, OPC_DIV, OPC_FMA, OPC_LOOP = 0, 1, 2, 3, 4
FAM_RUNTIME, FAM_NORMALIZE, FAM_MULADD, FAM_MULADD_LOOP = 0, 1, 2, 3


@pytest.fixture(scope="module")
def driver():
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "drv.cpp"), os.path.join(d, "drv")
        open(src, "w").write(DRIVER)
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-ffp-contract=off", "-fsanitize=undefined",
                               "-fno-sanitize-recover=undefined", "-I", CSRC, "-o", exe,
                               src, os.path.join(CSRC, "fk_chain.cpp")])

        def run(chains):
            """[(chain dict, strict)] -> [(swap, ops, family, consts)]"""
            lines = []
            for ch, strict in chains:
                r, w = ch["read"], ch["write"]
                lines.append(f"{r['channels']} {len(ch['ops'])} {int(strict)} "
                             f"{int(r['kind'] == 'crop_resize')} {['u8', 'f16', 'f32'].index(r['dtype'])} "
                             f"{['u8', 'f16', 'f32'].index(w['dtype'])} {int(w['layout'] == 'planar')}")
                for o in ch["ops"]:
                    k = list(o.get("k", [])) + [0.0] * (4 - len(o.get("k", [])))
                    lines.append(f"{KINDS.get(o['kind'], 6)} {len(o.get('k', []))} " + " ".join(float(v).hex() for v in k)
                                 + f" {o.get('span', 0)} {o.get('count', 0)}")
            out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                                 check=True).stdout.split("\n")
            res, i = [], 0
            for _ in chains:
                f0 = out[i].split()
                swap, n, fam, sn, nk = (int(v) for v in f0[:5])
                executed = [float(v) for v in f0[5:9]]
                i += 1
                ops = []
                for _ in range(n):
                    f = out[i].split()
                    ops.append((int(f[0]), np.array([float.fromhex(v) for v in f[1:5]], np.float32),
                                np.array([float.fromhex(v) for v in f[5:9]], np.float32),
                                int(f[9]), int(f[10])))
                    i += 1
                ks = [float.fromhex(out[i + j]) for j in range(nk)]
                i += nk
                res.append((swap, ops, fam, sn, ks, executed))
            return res
        yield run


def evaluate(frame, C, swap, ops):
    """The normalised list applied to a packed frame, fp32 per operation; a
    LOOP record sends execution back over its `span` records until they
    have run `count` times."""
    x = frame.astype(np.float32).reshape(-1, C)
    if swap:
        x = x[:, [2, 1, 0] + list(range(3, C))]
    o, runs = 0, 1
    while o < len(ops):
        code, a, b, span, count = ops[o]
        o += 1
        if code == OPC_LOOP:
            if runs < count:
                runs += 1
                o -= span + 1
            else:
                runs = 1
            continue
        a, b = a[:C], b[:C]
        if code == OPC_MUL:
            x = x * a
        elif code == OPC_ADD:
            x = x + a
        elif code == OPC_DIV:
            x = x / a
        else:  # one rounding of the exact product-sum; exact for all but ties of a double rounding
            x = (x.astype(np.float64) * a + b).astype(np.float32)
    return x.reshape(frame.shape)


def random_chain(g, C, dtype, max_ops=24):
    spec = datagen.random_chain_spec(g, max_ops=max_ops)
    ch = spec["chain"]
    for o in ch["ops"]:  # re-draw per-channel constants for this C
        if len(o["k"]) > 1:
            o["k"] = [datagen.f32(g.uniform(*((0.5, 1.5) if o["kind"] in ("mul", "div") else (-1, 1))))
                      for _ in range(C)]
    ch["read"] = {"kind": "plain", "dtype": dtype, "channels": C, "out_w": 0, "out_h": 0}
    ch["write"] = {"dtype": "f32", "layout": "packed"}
    return ch


def add_loops(g, ops):
    """Insert loop ops after random runs of arithmetic ops."""
    out, run = [], 0
    for o in ops:
        out.append(o)
        run = run + 1 if o["kind"] in ("mul", "add", "sub", "div") else 0
        if run and g.uniform() < 0.3:
            out.append({"kind": "loop", "span": int(g.integers(1, run + 1)), "count": int(g.integers(1, 5))})
            run = 0
    return out


@pytest.mark.parametrize("strict", [True, False])
def test_normalised_list_matches_oracle(driver, strict):
    g = datagen.rng(11 + strict)
    cases = []
    for t in range(120):
        C = [1, 3, 4][t % 3]
        dtype = ["u8", "f32"][(t // 3) % 2]
        ch = random_chain(g, C, dtype)
        if t % 5 == 1:  # loops over runs of arithmetic ops
            ch["ops"] = add_loops(g, ch["ops"])
        if t % 7 == 0:  # swaps around per-channel constants
            ch["ops"] = [{"kind": "mul", "k": [1.5, 0.75, 0.625, 1.25][:C]}, {"kind": "swap", "k": []},
                         {"kind": "sub", "k": [0.25, -0.5, 0.125, 1.0][:C]}, {"kind": "swap", "k": []},
                         {"kind": "div", "k": [0.5, 0.875, 1.375, 1.0][:C]}, {"kind": "swap", "k": []}]
        if dtype == "u8":
            fr = datagen.frame(g, 5, 7, C)
        else:
            fr = (g.uniform(-300, 300, size=(5, 7, C))).astype(np.float32)
        cases.append((ch, fr))
    outs = driver([(ch, strict) for ch, _ in cases])
    for (ch, fr), (swap, ops, _, _, _, executed) in zip(cases, outs):
        C = ch["read"]["channels"]
        n_arith = sum(o["kind"] in ("mul", "add", "sub", "div") for o in ch["ops"])
        n_loops = sum(o["kind"] == "loop" for o in ch["ops"])
        # at most one record per op (contraction and merged repeats shorten it)
        assert len(ops) <= n_arith + n_loops
        assert all(op[0] != OPC_FMA for op in ops) or not strict
        # ops the chain executes (loops unrolled) = records run, before contraction
        runs = [1] * len(ch["ops"])
        for i, o in enumerate(ch["ops"]):
            if o["kind"] == "loop":
                for j in range(i - o["span"], i):
                    runs[j] = o["count"]
        n_exec = sum(r for o, r in zip(ch["ops"], runs) if o["kind"] in ("mul", "add", "sub", "div"))
        fma = executed[3]
        assert sum(executed) + fma == n_exec and (not strict or fma == 0)
        n_swaps = sum(o["kind"] == "swap" for o in ch["ops"])
        assert swap == (n_swaps % 2 if C >= 3 else 0)
        got = evaluate(fr, C, swap, ops)
        ref = oracle.run_chain(ch, [fr], [{"frame": 0, "x": 0, "y": 0, "w": 7, "h": 5}])[0]
        if strict:
            np.testing.assert_array_equal(got.view(np.uint32), ref["out"].view(np.uint32))
        else:
            tol = 1e-5 * np.maximum(np.abs(ref["out"]), ref["smax"]) + 1e-30
            assert np.all(np.abs(got - ref["out"]) <= tol)


def test_contraction_pairs_mul_then_add_only(driver):
    ch = {"read": {"kind": "plain", "dtype": "f32", "channels": 3, "out_w": 0, "out_h": 0},
          "write": {"dtype": "f32", "layout": "packed"},
          "ops": [{"kind": "mul", "k": [2.0]}, {"kind": "sub", "k": [1.0, 2.0, 3.0]},
                  {"kind": "add", "k": [4.0]}, {"kind": "mul", "k": [3.0]},
                  {"kind": "cvt", "k": []}, {"kind": "add", "k": [0.5]},
                  {"kind": "mul", "k": [5.0]}, {"kind": "div", "k": [2.0]}]}
    (swap, ops, fam, _, _, _), = driver([(ch, False)])
    codes = [op[0] for op in ops]
    # mul,sub -> fma(2,-k); add stays; mul,(cvt),add -> fma; mul; div
    assert codes == [OPC_FMA, OPC_ADD, OPC_FMA, OPC_MUL, OPC_DIV]
    np.testing.assert_array_equal(ops[0][1][:3], [2, 2, 2])
    np.testing.assert_array_equal(ops[0][2][:3], [-1, -2, -3])
    assert swap == 0 and fam == FAM_RUNTIME


def test_static_chain_match(driver):
    norm = datagen.normalize_chain(224, 224)
    mulsub = {**norm, "ops": [dict(o) for o in norm["ops"]]}
    mulsub["ops"][2] = {"kind": "mul", "k": [1.0, 2.0, 3.0]}  # per-channel scale: not the built-in chain
    f16 = {**norm, "write": {"dtype": "f16", "layout": "planar"}}
    cases = [(norm, True), (mulsub, True), (f16, True)]
    g = datagen.rng(0)
    for n in (1, 2, 4, 16, 64, 256, 257):
        cases.append((datagen.muladd_chain(n, g), True))
    loop3 = datagen.loop_chain(1000, g, channels=3)
    loop4 = datagen.loop_chain(7, g, channels=1)
    loop4["ops"][3]["span"] = 1
    f32loop = datagen.data_size_case(10, pairs=100)["chain"]
    f16loop = dict(f32loop, read=dict(f32loop["read"], dtype="f16"))
    cases += [(f32loop, True), (f16loop, True)]
    cases += [(datagen.loop_chain(10000, g), False), (loop3, True), (loop4, True)]
    res = driver(cases)
    r1, r3, r4 = res[-3:]
    assert res[-5][2] == FAM_MULADD_LOOP and res[-5][3] == 100 and res[-4][2] == FAM_RUNTIME
    assert r1[2] == FAM_MULADD_LOOP and r1[3] == 10000 and r3[2] == FAM_MULADD_LOOP and r3[3] == 1000
    assert r1[4] == [np.float32(cases[-3][0]["ops"][1]["k"][0]), np.float32(cases[-3][0]["ops"][2]["k"][0])]
    assert r4[2] == FAM_RUNTIME
    # contracted loop body: one FMA record, then LOOP(span 1, count P)
    assert [op[0] for op in r1[1]] == [OPC_FMA, OPC_LOOP] and r1[1][1][3:] == (1, 10000)
    assert [op[0] for op in r3[1]] == [OPC_MUL, OPC_ADD, OPC_LOOP] and r3[1][2][3:] == (2, 1000)
    # a loop over the add only: mul must not absorb it
    assert [op[0] for op in r4[1]] == [OPC_MUL, OPC_ADD, OPC_LOOP] and r4[1][2][3:] == (1, 7)
    res, cases = res[:-5], cases[:-5]
    assert res[0][2] == FAM_NORMALIZE and res[0][3] == 5
    k = res[0][4]
    assert k[0] == np.float32(norm["ops"][2]["k"][0])
    np.testing.assert_array_equal(k[1:4], np.float32(norm["ops"][3]["k"]))
    np.testing.assert_array_equal(k[4:7], np.float32(norm["ops"][4]["k"]))
    assert res[1][2] == FAM_RUNTIME and res[2][2] == FAM_RUNTIME
    for (ch, _), r, n in zip(cases[3:], res[3:], (1, 2, 4, 16, 64, 256, 257)):
        if n in (1, 4, 16, 64, 256):
            assert r[2] == FAM_MULADD and r[3] == n
            np.testing.assert_array_equal(r[4], [np.float32(o["k"][0]) for o in ch["ops"][1:]])
        else:
            assert r[2] == FAM_RUNTIME


def test_identical_records_merge_into_one_record_and_a_loop(driver):
    """Repeats of one op (same code and constants) outside multi-record loop
    bodies become one record and a one-record LOOP with the summed count;
    the list still computes the chain bit for bit (strict)."""
    C = 3
    m = {"kind": "mul", "k": [1.001]}
    a = {"kind": "add", "k": [0.5, -0.25, 0.125]}
    ops = ([{"kind": "cvt", "k": []}] + [m] * 7 + [{"kind": "loop", "span": 1, "count": 5}]
           + [m, a, {"kind": "loop", "span": 2, "count": 3}, m, m, a, a, {"kind": "swap", "k": []}, a])
    ch = {"read": {"kind": "plain", "dtype": "u8", "channels": C, "out_w": 0, "out_h": 0},
          "ops": ops, "write": {"dtype": "f32", "layout": "packed"}}
    (swap, recs, _, _, _, executed), = driver([(ch, True)])
    codes = [(r[0], r[-2], r[-1]) for r in recs]
    # 6 muls + one mul looped 5 times -> mul, LOOP(1, 11); the body of the
    # two-record loop stays; then mul x2, add x2 (the last add's constants
    # are permuted by the swap, so it differs) -> mul LOOP(1,2) add LOOP(1,2) add
    assert codes == [(OPC_MUL, 0, 0), (OPC_LOOP, 1, 11), (OPC_MUL, 0, 0), (OPC_ADD, 0, 0),
                     (OPC_LOOP, 2, 3), (OPC_MUL, 0, 0), (OPC_LOOP, 1, 2), (OPC_ADD, 0, 0),
                     (OPC_LOOP, 1, 2), (OPC_ADD, 0, 0)], codes
    assert executed[OPC_MUL] == 11 + 3 + 2 and executed[OPC_ADD] == 3 + 3
    g = datagen.rng(5)
    fr = datagen.frame(g, 4, 6, C)
    got = evaluate(fr, C, swap, recs)
    ref = oracle.run_chain(ch, [fr], [{"frame": 0, "x": 0, "y": 0, "w": 6, "h": 4}])[0]
    np.testing.assert_array_equal(got.view(np.uint32), ref["out"].view(np.uint32))
