"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
every entry point of the C oracle on random, degenerate and pitched masks in
both polarities (with several threads), and the request server's host
bookkeeping (arena allocator, percentiles).  A sanitizer report or a
mismatch between oracle forms fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "edt_oracle.c")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_brute(const uint8_t *, int32_t, int32_t, int64_t, int32_t, int32_t, int32_t,
                     int32_t *, int32_t *);
int64_t oracle_brute_at(const uint8_t *, int32_t, int32_t, int64_t, int32_t, const int64_t *,
                        int64_t, int32_t, int32_t *, int32_t *);
void oracle_column_pass(const uint8_t *, int32_t, int32_t, int64_t, int32_t, int32_t, int32_t,
                        int32_t *, int64_t *);
int32_t oracle_row_envelope(const int64_t *, const int32_t *, int32_t, int32_t, int32_t *,
                            int32_t *);
void oracle_separable(const uint8_t *, int32_t, int32_t, int64_t, int32_t, int32_t, int32_t *,
                      int32_t *);
void oracle_basic_rows(const uint8_t *, int32_t, int32_t, int64_t, int32_t, int32_t, int32_t *,
                       int32_t *);
void oracle_sqrt_f32(const int32_t *, int64_t, float *);
int64_t oracle_brute_metric(const uint8_t *, int32_t, int32_t, int64_t, int32_t, int32_t,
                            int32_t *, int32_t *);
int64_t oracle_brute_metric_at(const uint8_t *, int32_t, int32_t, int64_t, int32_t, int32_t,
                               const int64_t *, int64_t, int32_t, int32_t *, int32_t *);
void oracle_cityblock_scans(const uint8_t *, int32_t, int32_t, int64_t, int32_t, int32_t,
                            int32_t *);
void oracle_chamfer_scans(const uint8_t *, int32_t, int32_t, int64_t, int32_t, int32_t,
                          int32_t *);
void oracle_regions(const uint8_t *, int32_t, int32_t, int64_t, int32_t, int32_t,
                    const int32_t *, int32_t *);
void oracle_danielsson(const uint8_t *, int32_t, int32_t, int64_t, int32_t, int32_t, int32_t *,
                       int32_t *);

static uint64_t st = 2106501;
static uint32_t rnd(void) { st = st * 6364136223846793005ull + 1442695040888963407ull; return (uint32_t)(st >> 33); }

static int same(const int32_t *a, const int32_t *b, int64_t n) { return memcmp(a, b, (size_t)n * 4) == 0; }

int main(void) {
    for (int it = 0; it < 160; ++it) {
        const int H = 1 + (int)(rnd() % (it < 20 ? 3 : 40)), W = 1 + (int)(rnd() % (it < 20 ? 3 : 40));
        const int pitch = W + (int)(rnd() % 5);
        const int pol = (int)(rnd() % 2), threads = 1 + (int)(rnd() % 3);
        const int kind = it % 4;  /* random, empty, full, sparse */
        uint8_t *m = (uint8_t *)malloc((size_t)H * pitch);
        for (int i = 0; i < H * pitch; ++i) {
            const uint32_t r = rnd() % 100;
            m[i] = kind == 1 ? 0 : kind == 2 ? 1 : kind == 3 ? (r < 2) : (r < 15 ? (uint8_t)(1 + r) : 0);
        }
        const int64_t n = (int64_t)H * W;
        int32_t *D0 = malloc(n * 4), *F0 = malloc(n * 4), *D1 = malloc(n * 4), *F1 = malloc(n * 4);
        int32_t *R = malloc(n * 4), *L = malloc(n * 4), *Rel = malloc(n * 4);
        int64_t *Dv = malloc(n * 8), *lin = malloc(n * 8);
        float *sq = malloc(n * 4);
        oracle_brute(m, H, W, pitch, pol, 0, threads, D0, F0);
        oracle_brute(m, H, W, pitch, pol, 1, threads, D1, F1);
        if (!same(D0, D1, n) || !same(F0, F1, n)) { printf("FAIL contour %d\n", it); return 1; }
        oracle_separable(m, H, W, pitch, pol, threads, D1, F1);
        if (!same(D0, D1, n) || !same(F0, F1, n)) { printf("FAIL separable %d\n", it); return 1; }
        oracle_basic_rows(m, H, W, pitch, pol, threads, D1, F1);
        if (!same(D0, D1, n) || !same(F0, F1, n)) { printf("FAIL basic %d\n", it); return 1; }
        for (int64_t q = 0; q < n; ++q) lin[q] = (q * 7919) % n;
        oracle_brute_at(m, H, W, pitch, pol, lin, n, threads, D1, F1);
        for (int64_t q = 0; q < n; ++q)
            if (D1[q] != D0[lin[q]] || F1[q] != F0[lin[q]]) { printf("FAIL at %d\n", it); return 1; }
        for (int sweeps = 1; sweeps <= 2; ++sweeps) oracle_column_pass(m, H, W, pitch, pol, sweeps, threads, R, Dv);
        for (int i = 0; i < H; ++i) {
            int32_t ks[64], js[64];
            for (int rule = 0; rule < 2; ++rule) oracle_row_envelope(Dv + (int64_t)i * W, R + (int64_t)i * W, W, rule, ks, js);
        }
        oracle_sqrt_f32(D0, n, sq);
        for (int metric = 1; metric <= 3; ++metric) {
            oracle_brute_metric(m, H, W, pitch, pol, metric, D0, F0);
            oracle_brute_metric_at(m, H, W, pitch, pol, metric, lin, n, threads, D1, F1);
            for (int64_t q = 0; q < n; ++q)
                if (D1[q] != D0[lin[q]] || F1[q] != F0[lin[q]]) { printf("FAIL metric at %d\n", it); return 1; }
        }
        oracle_brute_metric(m, H, W, pitch, pol, 1, D0, F0);
        for (int stages = 1; stages <= 4; ++stages) oracle_cityblock_scans(m, H, W, pitch, pol, stages, D1);
        if (!same(D0, D1, n)) { printf("FAIL cityblock scans %d\n", it); return 1; }
        oracle_brute_metric(m, H, W, pitch, pol, 3, D0, F0);
        for (int passes = 1; passes <= 2; ++passes) oracle_chamfer_scans(m, H, W, pitch, pol, passes, D1);
        if (!same(D0, D1, n)) { printf("FAIL chamfer scans %d\n", it); return 1; }
        oracle_separable(m, H, W, pitch, pol, threads, D0, F0);
        oracle_regions(m, H, W, pitch, pol, 4, F0, L);
        oracle_regions(m, H, W, pitch, pol, 8, F0, L);
        for (int passes = 1; passes <= 2; ++passes) oracle_danielsson(m, H, W, pitch, pol, passes, D1, Rel);
        free(m); free(D0); free(F0); free(D1); free(F1); free(R); free(L); free(Rel); free(Dv); free(lin); free(sq);
    }
    printf("OK\n");
    return 0;
}
"""


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    src = tmp_path / "driver.c"
    exe = tmp_path / "driver"
    src.write_text(DRIVER)
    subprocess.check_call(["gcc", "-std=c11", "-pthread"] + SAN +
                          [ORACLE_C, str(src), "-o", str(exe), "-lm"])
    out = _run(exe)
    assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr[-4000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_serve_host_bookkeeping_under_sanitizers(tmp_path):
    from tests.test_serve_core import CORE, PROGRAM
    src = tmp_path / "core_check.cpp"
    exe = tmp_path / "core_check"
    src.write_text(PROGRAM)
    subprocess.check_call(["g++", "-std=c++17"] + SAN + ["-I", CORE, str(src), "-o", str(exe)])
    out = _run(exe)
    assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr[-4000:]
