"""Host bookkeeping of the request server, built with g++ and run on the CPU:
the arena allocator against a byte-map model under random alloc/release
sequences, and the nearest-rank percentile against its definition."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CORE = os.path.join(ROOT, "paper_2106_03503_amd", "csrc")

PROGRAM = r"""
#include "serve_core.h"
#include <cstdio>
#include <random>
#include <vector>

static int fail(const char* what, long a, long b) {
    std::printf("FAIL %s %ld %ld\n", what, a, b);
    return 1;
}

int main() {
    // allocator: random traffic, checked against a byte map of the arena
    for (int seed = 0; seed < 20; ++seed) {
        std::mt19937_64 rng(seed);
        const size_t size = 256 * (1 + rng() % 400);
        edt::Arena a(size + rng() % 256);  // the size is cut to whole units
        if (a.size() != size) return fail("size", a.size(), size);
        std::vector<int> owner(size / 256, -1);
        struct Blk { size_t off, bytes; int id; };
        std::vector<Blk> live;
        int next = 0;
        size_t used = 0, high = 0;
        for (int step = 0; step < 4000; ++step) {
            if (live.empty() || rng() % 2) {
                const size_t bytes = rng() % 3 == 0 ? rng() % 3000 : 1 + rng() % 600;
                size_t off = 0;
                const size_t units = (bytes == 0 ? 1 : (bytes + 255) / 256);
                // a model first-fit search: the lowest run of free units
                long want = -1;
                for (size_t u = 0, run = 0; u < owner.size(); ++u) {
                    run = owner[u] < 0 ? run + 1 : 0;
                    if (run == units) { want = (long)(u + 1 - units); break; }
                }
                const bool ok = a.alloc(bytes, &off);
                if (ok != (want >= 0)) return fail("alloc result", ok, want);
                if (!ok) continue;
                if ((long)(off / 256) != want || off % 256) return fail("first fit", off, want);
                for (size_t u = 0; u < units; ++u) owner[off / 256 + u] = next;
                live.push_back({off, bytes, next++});
                used += units * 256;
                if (used > high) high = used;
            } else {
                const size_t k = rng() % live.size();
                const Blk b = live[k];
                live.erase(live.begin() + k);
                const size_t units = (b.bytes == 0 ? 1 : (b.bytes + 255) / 256);
                for (size_t u = 0; u < units; ++u) {
                    if (owner[b.off / 256 + u] != b.id) return fail("owner", u, b.id);
                    owner[b.off / 256 + u] = -1;
                }
                a.release(b.off, b.bytes);
                used -= units * 256;
            }
            if (a.in_use() != used) return fail("in_use", a.in_use(), used);
            if (a.high_water() != high) return fail("high", a.high_water(), high);
            // free blocks are maximal runs: as many as the model's free runs
            size_t runs = 0, largest = 0;
            for (size_t u = 0, run = 0; u <= owner.size(); ++u) {
                if (u < owner.size() && owner[u] < 0) { ++run; continue; }
                if (run) { ++runs; if (run * 256 > largest) largest = run * 256; }
                run = 0;
            }
            if (a.free_blocks() != runs) return fail("coalesce", a.free_blocks(), runs);
            if (a.largest_free() != largest) return fail("largest", a.largest_free(), largest);
        }
    }
    // percentile: nearest rank, the smallest value with at least q of the data
    // at or below it
    std::vector<double> v;
    for (int k = 100; k >= 1; --k) v.push_back(k);
    if (edt::percentile(v, 0.50) != 50) return fail("p50", 0, 0);
    if (edt::percentile(v, 0.99) != 99) return fail("p99", 0, 0);
    if (edt::percentile(v, 1.0) != 100) return fail("p100", 0, 0);
    if (edt::percentile({7.0}, 0.99) != 7) return fail("single", 0, 0);
    if (edt::percentile({}, 0.5) != 0) return fail("empty", 0, 0);
    if (edt::percentile({1, 2, 3}, 0.5) != 2) return fail("odd", 0, 0);
    if (edt::percentile({1, 2, 3, 4}, 0.5) != 2) return fail("even", 0, 0);
    std::printf("OK\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_serve_core_host_logic(tmp_path):
    src = tmp_path / "core_check.cpp"
    exe = tmp_path / "core_check"
    src.write_text(PROGRAM)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", CORE, str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr
