"""Host bookkeeping of the request server, built with g++ and run on the CPU:
the arena allocator against a byte-map model under random alloc/release
sequences, the ticket book against an unbounded per-ticket model under random
issue/complete sequences, and the nearest-rank percentile against its
definition."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CORE = os.path.join(ROOT, "paper_2106_03503_amd", "csrc")

PROGRAM = r"""
#include "serve_core.h"
#include <algorithm>
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
    // ticket book: random issues and out-of-order completions (some failing)
    // against a model that keeps every ticket's status and every latency
    for (int seed = 0; seed < 8; ++seed) {
        std::mt19937_64 rng(100 + seed);
        edt::TicketBook book;
        std::vector<int> model;      // status of ticket t at t - 1
        std::vector<uint64_t> open;  // tickets in flight
        std::vector<double> lats;    // latencies in completion order
        const int steps = seed < 2 ? 300000 : 20000;  // the first two pass the window
        for (int step = 0; step < steps; ++step) {
            if (open.empty() || (open.size() < 64 && rng() % 2)) {
                const uint64_t t = book.issue();
                if (t != model.size() + 1) return fail("ticket order", (long)t, (long)model.size());
                model.push_back(edt::TicketBook::kPending);
                open.push_back(t);
            } else {
                const size_t k = rng() % open.size();
                const uint64_t t = open[k];
                open.erase(open.begin() + k);
                const int st = rng() % 97 == 0 ? -5 : 0;
                const double lat = (double)(rng() % 1000000);
                book.complete(t, st, lat);
                model[t - 1] = st;
                lats.push_back(lat);
            }
            if (step % 997 == 0 || step == steps - 1) {
                for (uint64_t t = 1; t <= model.size(); ++t)
                    if (book.status(t) != model[t - 1]) return fail("status", (long)t, model[t - 1]);
                if (book.known(0) || book.known(model.size() + 1) || !book.known(model.size()))
                    return fail("known", (long)model.size(), 0);
                size_t failed = 0;
                for (int v : model) failed += v != 0 && v != edt::TicketBook::kPending;
                // entries: from the oldest open ticket on, plus the failures
                const uint64_t oldest = open.empty() ? model.size() + 1
                                                     : *std::min_element(open.begin(), open.end());
                if (book.entries() > model.size() + 1 - oldest + failed)
                    return fail("bounded", (long)book.entries(), (long)(model.size() + 1 - oldest));
                if (book.completed() != lats.size()) return fail("count", (long)book.completed(), (long)lats.size());
                double sum = 0.0, mx = 0.0;
                for (double v : lats) { sum += v; mx = std::max(mx, v); }
                if (book.latency_sum() != sum || book.latency_max() != mx) return fail("sum/max", 0, 0);
                // the window holds exactly the last kWindow latencies
                const size_t w = std::min(lats.size(), edt::TicketBook::kWindow);
                std::vector<double> want(lats.end() - (long)w, lats.end()), got = book.window();
                std::sort(want.begin(), want.end());
                std::sort(got.begin(), got.end());
                if (got != want) return fail("window", (long)got.size(), (long)w);
            }
        }
        if (seed < 2 && lats.size() <= edt::TicketBook::kWindow) return fail("window passed", (long)lats.size(), 0);
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
