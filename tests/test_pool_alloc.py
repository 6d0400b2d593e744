"""The request server's pool allocator (host C++, csrc/pool_alloc.hpp),
driven on the CPU: admission by HBM footprint carves each request's
workspace out of one device pool first-fit, 256-byte aligned, and merges
freed neighbours.  A small program built with g++ replays random admit/retire
sequences; a plain Python first-fit model of the same policy must give the
same offsets, no two live blocks may overlap, and retiring everything must
leave one free block of the whole pool."""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1911_04712_amd", "csrc")

REPLAY_SRC = r"""
#include <cstdio>
#include "pool_alloc.hpp"
int main() {
    dpd::PoolAlloc a;
    char op; unsigned long long x, y;
    while (std::scanf(" %c", &op) == 1) {
        if (op == 'R') { std::scanf("%llu", &x); a.reset(x); }
        else if (op == 'A') { std::scanf("%llu", &x); size_t off = 0; bool ok = a.alloc(x, &off);
                              std::printf("%d %llu\n", ok ? 1 : 0, (unsigned long long)off); }
        else if (op == 'F') { std::scanf("%llu %llu", &x, &y); a.release(x, y); }
        else if (op == 'L') { std::printf("%llu %llu\n", (unsigned long long)a.largest(),
                                          (unsigned long long)a.blocks()); }
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def replay(tmp_path_factory):
    d = tmp_path_factory.mktemp("pool")
    src, exe = d / "replay.cpp", d / "replay"
    src.write_text(REPLAY_SRC)
    # built with AddressSanitizer and UndefinedBehaviorSanitizer: every replay
    # below also checks the allocator for out-of-bounds access, use after free
    # and undefined behaviour
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


def _align(x):
    return (x + 255) & ~255


class FirstFit:
    """Reference: free list sorted by offset, lowest offset that fits."""

    def __init__(self, size):
        self.free = [[0, size]] if size else []

    def alloc(self, n):
        n = _align(n)
        for k, (o, l) in enumerate(self.free):
            if l >= n:
                if l == n:
                    del self.free[k]
                else:
                    self.free[k] = [o + n, l - n]
                return o
        return None

    def release(self, o, n):
        self.free.append([o, _align(n)])
        self.free.sort()
        merged = []
        for b in self.free:
            if merged and merged[-1][0] + merged[-1][1] == b[0]:
                merged[-1][1] += b[1]
            else:
                merged.append(b)
        self.free = merged


@pytest.mark.parametrize("seed", range(4))
def test_pool_matches_first_fit_model(replay, seed):
    rng = np.random.default_rng(seed)
    size = 1 << 24
    ops, model, live, expect = [f"R {size}"], FirstFit(size), [], []
    for _ in range(600):
        if live and rng.random() < 0.45:
            o, n = live.pop(int(rng.integers(len(live))))
            ops.append(f"F {o} {n}")
            model.release(o, n)
        else:
            n = int(rng.integers(1, 1 << 20))
            o = model.alloc(n)
            ops.append(f"A {n}")
            expect.append(o)
            if o is not None:
                live.append((o, n))
    for o, n in live:
        ops.append(f"F {o} {n}")
    ops.append("L")
    out = subprocess.run([replay], input="\n".join(ops) + "\n", capture_output=True, text=True, check=True)
    lines = out.stdout.split("\n")
    got = []
    for ln in lines[:len(expect)]:
        ok, off = ln.split()
        got.append(int(off) if ok == "1" else None)
    assert got == expect
    largest, blocks = (int(v) for v in lines[len(expect)].split())
    assert (largest, blocks) == (size, 1)          # everything retired: one free block again


def test_live_blocks_never_overlap(replay):
    rng = np.random.default_rng(9)
    size = 1 << 22
    ops, sizes = [f"R {size}"], []
    for _ in range(200):
        n = int(rng.integers(1, 1 << 16))
        ops.append(f"A {n}")
        sizes.append(n)
    out = subprocess.run([replay], input="\n".join(ops) + "\n", capture_output=True, text=True, check=True)
    blocks = []
    for ln, n in zip(out.stdout.split("\n"), sizes):
        ok, off = ln.split()
        if ok == "1":
            o = int(off)
            assert o % 256 == 0 and o + _align(n) <= size
            blocks.append((o, o + _align(n)))
    blocks.sort()
    assert all(a[1] <= b[0] for a, b in zip(blocks, blocks[1:]))
