"""The server's arena allocator (plain C++, built here with g++) against a
first-fit model with coalescing."""
import os
import subprocess
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_07071_amd", "csrc")

DRIVER = r"""
#include "fk_arena.hpp"
#include <cstdio>
int main() {
    fk::Arena a(1 << 20);
    char op; long long x, y;
    while (std::scanf(" %c", &op) == 1) {
        if (op == 'A') { std::scanf("%lld", &x); std::printf("%lld\n", (long long)a.alloc(x)); }
        else if (op == 'R') { std::scanf("%lld %lld", &x, &y); a.release(x, y); }
        else if (op == 'S') { std::printf("%lld %zu\n", (long long)a.free_bytes(), a.free_blocks()); }
    }
    return 0;
}
"""


class Model:
    def __init__(self, size):
        self.free = [(0, size)]

    def alloc(self, n):
        for i, (o, s) in enumerate(self.free):
            if s >= n:
                self.free[i:i + 1] = [(o + n, s - n)] if s > n else []
                return o
        return -1

    def release(self, o, n):
        self.free.append((o, n))
        self.free.sort()
        merged = []
        for blk in self.free:
            if merged and merged[-1][0] + merged[-1][1] == blk[0]:
                merged[-1] = (merged[-1][0], merged[-1][1] + blk[1])
            else:
                merged.append(blk)
        self.free = merged


def test_arena_matches_first_fit_model():
    g = np.random.default_rng(0)
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "drv.cpp")
        exe = os.path.join(d, "drv")
        open(src, "w").write(DRIVER)
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
                               "-I", CSRC, "-o", exe, src])
        model = Model(1 << 20)
        live, script, expect = [], [], []
        for _ in range(3000):
            if live and g.uniform() < 0.45:
                o, n = live.pop(int(g.integers(0, len(live))))
                script.append(f"R {o} {n}")
                model.release(o, n)
            else:
                n = int(g.integers(1, 40000)) // 256 * 256 + 256
                o = model.alloc(n)
                script.append(f"A {n}")
                expect.append(o)
                if o >= 0:
                    live.append((o, n))
        for o, n in live:
            script.append(f"R {o} {n}")
            model.release(o, n)
        script.append("S")
        out = subprocess.run([exe], input="\n".join(script), capture_output=True, text=True, check=True)
        lines = out.stdout.split("\n")
        got = [int(x) for x in lines[:len(expect)]]
        assert got == expect
        assert lines[len(expect)] == f"{1 << 20} 1"  # everything released: one free block
