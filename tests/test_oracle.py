"""Pins of the CPU oracle against what the paper and the mathematics fix.

The oracle is checked here against: the values the paper prints for its worked
example (tests/golden/, each file citing its figure), closed forms, brute force
on tiny inputs, special cases that reduce to the one-dimensional problem, and
invariants of the exact transform.  None of these re-types the oracle's own
arithmetic.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests.golden_io import INF, keyed, table

INF_SQ = oracle.INF_SQ


def _inf_to_minus1(D):
    D = np.asarray(D, np.int64).copy()
    D[D == INF_SQ] = -1
    return D


# ---------------------------------------------------------------- paper tables

def test_example_mask_matches_initialisation():
    # Figure fig_EEDT(a): zeros exactly at the six object pixels of the listing.
    m = workloads.paper_example()
    init = table("fig_eedt_a_init.txt")
    assert m.shape == init.shape == (9, 10)
    assert np.array_equal(m.astype(bool), init == 0)
    D, _ = oracle.brute(m)
    assert np.array_equal(D == 0, init == 0)


def test_downward_sweep_matches_fig_eedt2():
    R, Dv = oracle.column_pass(workloads.paper_example(), sweeps=1)
    assert np.array_equal(Dv, table("fig_eedt2_downward.txt"))


def test_vertical_pass_matches_fig_eedt_b():
    R, Dv = oracle.column_pass(workloads.paper_example(), sweeps=2)
    assert np.array_equal(Dv, table("fig_eedt_b_vertical.txt"))
    # the carried site row reproduces the vertical distance
    i = np.arange(9)[:, None]
    fin = R >= 0
    assert np.array_equal(((i - R) ** 2)[fin], Dv[fin])


@pytest.mark.parametrize("fn", ["brute", "brute_contour", "separable", "basic_rows"])
def test_final_matches_fig_eedt_c(fn):
    m = workloads.paper_example()
    if fn == "brute_contour":
        D, F = oracle.brute(m, contour_only=True)
    else:
        D, F = getattr(oracle, fn)(m)
    assert np.array_equal(D, table("fig_eedt_c_final.txt"))


@pytest.mark.parametrize("fn", ["brute", "separable", "basic_rows"])
def test_single_site_matches_fig_euclidean(fn):
    m = np.zeros((9, 10), np.uint8)
    m[4, 4] = 1
    D, F = getattr(oracle, fn)(m)
    assert np.array_equal(D, table("fig_euclidean_b.txt"))
    assert np.all(F == 4 * 10 + 4)


def test_propagation_row1_parabolas_and_kstar():
    # Figure fig_propagation: the parabola of column k in row 1 is the distance
    # from the row-1 pixels to the nearest object pixel of column k alone.
    m = workloads.paper_example()
    g = keyed("fig_propagation_row1.txt")
    for key, vals in g.items():
        if key[0] != "D":
            continue
        k, dv = int(key[1]), int(key[2])
        only = np.zeros_like(m)
        only[:, k - 1] = m[:, k - 1]
        D, _ = oracle.brute(only)
        assert D[0, k - 1] == dv
        assert D[0].tolist() == [int(v) for v in vals]
    for fn in (oracle.brute, oracle.separable, oracle.basic_rows):
        D, F = fn(m)
        assert D[0].tolist() == [int(v) for v in g[("min",)]]
        for j, ks in enumerate(g[("kstar",)]):
            cols = [int(v) - 1 for v in ks.split("/")]
            # the assigned site lies in one of the printed columns ...
            assert F[0, j] % 10 in cols
            # ... and is the smallest linear index among the nearest sites of
            # those columns (ties broken by the smallest index)
            cand = []
            for c in cols:
                rows = np.nonzero(m[:, c])[0]
                for r in rows:
                    if (r - 0) ** 2 + (c - j) ** 2 == D[0, j]:
                        cand.append(r * 10 + c)
            assert F[0, j] == min(cand)
            if len(cols) > 1:
                assert len(cand) >= 2  # the paper's tie is a real tie


def test_envelope_trace_row1():
    # Section 3.3.1: the fast algorithm's contributors for row 1.  With ties to
    # the parabola further right (rounding the intersection up), column 5 owns
    # [1, 7) and column 8 owns [7, 11) (1-based); the virtual start parabola
    # at column 1 owns the empty range [1, 1).
    R, Dv = oracle.column_pass(workloads.paper_example())
    g = keyed("envelope_trace_row1.txt")
    ks_p = [int(v) for v in g["ks"]]
    js_p = [int(v) for v in g["js"]]
    ks, js = oracle.row_envelope(Dv[0], R[0], rule=1)
    # drop the virtual start parabola (empty range), convert to 0-based
    keep = [e for e in range(len(ks_p)) if js_p[e] < js_p[e + 1]]
    assert ks.tolist() == [ks_p[e] - 1 for e in keep]
    assert js.tolist() == [js_p[e] - 1 for e in keep]
    assert js_p[-1] == 10 + 1
    # smallest-index rule: the tie at j = 7 goes to column 5's site (index 14)
    ks0, js0 = oracle.row_envelope(Dv[0], R[0], rule=0)
    assert ks0.tolist() == [4, 7]
    assert js0.tolist() == [0, 7]


# -------------------------------------------------------- brute-force agreement

def _tie_heavy(rng, H, W):
    # masks symmetric under both reflections: many equidistant site pairs
    h2, w2 = (H + 1) // 2, (W + 1) // 2
    q = (rng.random((h2, w2)) < rng.uniform(0.02, 0.3)).astype(np.uint8)
    full = np.zeros((H, W), np.uint8)
    full[:h2, :w2] = q
    full[:, W - w2:] |= full[:, :w2][:, ::-1]
    full[H - h2:, :] |= full[:h2, :][::-1, :]
    return full


def _random_masks(n, seed):
    rng = np.random.default_rng(seed)
    for t in range(n):
        H = int(rng.integers(1, 15))
        W = int(rng.integers(1, 15))
        kind = t % 3
        if kind == 0:
            m = (rng.random((H, W)) < rng.uniform(0.0, 0.5)).astype(np.uint8)
        elif kind == 1:
            m = _tie_heavy(rng, H, W)
        else:
            m = np.zeros((H, W), np.uint8)
            for _ in range(int(rng.integers(0, 4))):
                m[rng.integers(0, H), rng.integers(0, W)] = 1
        yield m, int(rng.integers(0, 2))


def test_all_oracle_forms_agree_on_small_masks():
    for m, pol in _random_masks(1500, 11):
        D1, F1 = oracle.brute(m, pol, nthreads=1)
        D1c, F1c = oracle.brute(m, pol, contour_only=True, nthreads=1)
        D2, F2 = oracle.separable(m, pol, nthreads=1)
        D3, F3 = oracle.basic_rows(m, pol, nthreads=1)
        for D, F in ((D1c, F1c), (D2, F2), (D3, F3)):
            assert np.array_equal(D, D1), (m, pol)
            assert np.array_equal(F, F1), (m, pol)


def test_brute_at_matches_full_brute():
    rng = np.random.default_rng(5)
    m = (rng.random((40, 57)) < 0.05).astype(np.uint8)
    D, F = oracle.brute(m)
    lin = rng.choice(40 * 57, size=300, replace=False)
    Ds, Fs = oracle.brute_at(m, lin)
    assert np.array_equal(Ds, D.ravel()[lin])
    assert np.array_equal(Fs, F.ravel()[lin])


def test_tiny_brute_force_by_enumeration():
    # every 3 x 3 mask: the oracle's D and F against a direct enumeration of
    # the definition written with Python integers
    for bits in range(1 << 9):
        m = np.array([(bits >> b) & 1 for b in range(9)], np.uint8).reshape(3, 3)
        for pol in (0, 1):
            D, F = oracle.separable(m, pol, nthreads=1)
            sites = [(r, c) for r in range(3) for c in range(3)
                     if (m[r, c] != 0) != (pol == 1)]
            for i in range(3):
                for j in range(3):
                    if not sites:
                        assert D[i, j] == INF_SQ and F[i, j] == -1
                        continue
                    best = min(((i - r) ** 2 + (j - c) ** 2, r * 3 + c) for r, c in sites)
                    assert (D[i, j], F[i, j]) == best


# ------------------------------------------------------------------ closed forms

def test_no_site_gives_sentinel():
    for fn in (oracle.brute, oracle.separable, oracle.basic_rows):
        D, F = fn(np.zeros((7, 5), np.uint8))
        assert np.all(D == INF_SQ) and np.all(F == -1)
        D, F = fn(np.ones((7, 5), np.uint8), 1)
        assert np.all(D == INF_SQ) and np.all(F == -1)


def test_all_sites_zero_and_own_index():
    for fn in (oracle.brute, oracle.separable):
        D, F = fn(np.ones((6, 9), np.uint8))
        assert np.all(D == 0)
        assert np.array_equal(F, np.arange(54).reshape(6, 9))


def test_corner_site_closed_form():
    m = workloads.corner(37, 53)
    D, F = oracle.separable(m)
    i, j = np.mgrid[0:37, 0:53]
    assert np.array_equal(D, i * i + j * j)
    assert np.all(F == 0)


def test_single_site_anywhere_separable():
    rng = np.random.default_rng(3)
    for _ in range(50):
        H, W = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        r, c = int(rng.integers(0, H)), int(rng.integers(0, W))
        m = np.zeros((H, W), np.uint8)
        m[r, c] = 1
        D, F = oracle.separable(m)
        i, j = np.mgrid[0:H, 0:W]
        assert np.array_equal(D, (i - r) ** 2 + (j - c) ** 2)
        assert np.all(F == r * W + c)


def test_sites_in_one_row_reduce_to_1d():
    # All sites in row r0: D(i, j) = (i - r0)^2 + e(j)^2 where e(j) is the 1-D
    # distance along the row to the nearest site column, found by scanning.
    rng = np.random.default_rng(4)
    H, W, r0 = 23, 61, 9
    m = np.zeros((H, W), np.uint8)
    cols = np.sort(rng.choice(W, size=7, replace=False))
    m[r0, cols] = 1
    D, F = oracle.separable(m)
    for j in range(W):
        e = min(abs(j - c) for c in cols)
        c_best = min(c for c in cols if abs(j - c) == e)
        for i in range(H):
            assert D[i, j] == (i - r0) ** 2 + e * e
            assert F[i, j] == r0 * W + c_best


# -------------------------------------------------------------------- invariants

def _check_invariants(m, pol, D, F):
    H, W = m.shape
    site = (m != 0) != (pol == 1)
    if not site.any():
        assert np.all(D == INF_SQ) and np.all(F == -1)
        return
    assert np.array_equal(D == 0, site)
    r, c = F // W, F % W
    assert np.all(site[r, c])
    i, j = np.mgrid[0:H, 0:W]
    assert np.array_equal(D.astype(np.int64), (i - r) ** 2 + (j - c) ** 2)
    assert D.max() <= (H - 1) ** 2 + (W - 1) ** 2
    # local optimality: no 8-neighbour's site is better for this pixel
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            if di == 0 and dj == 0:
                continue
            ii = np.clip(i + di, 0, H - 1)
            jj = np.clip(j + dj, 0, W - 1)
            Fn = F[ii, jj]
            rn, cn = Fn // W, Fn % W
            Dn = (i - rn) ** 2 + (j - cn) ** 2
            worse = (Dn < D) | ((Dn == D) & (Fn < F))
            assert not worse.any()
    # the distance is 1-Lipschitz between 4-neighbours
    d = np.sqrt(D.astype(np.float64))
    assert np.all(np.abs(np.diff(d, axis=0)) <= 1 + 1e-9)
    assert np.all(np.abs(np.diff(d, axis=1)) <= 1 + 1e-9)


def test_invariants_on_generated_masks():
    masks = [
        workloads.bernoulli(64, 80, 0.01, seed=1),
        workloads.disks(96, 70, n_disks=6, rmin=2, rmax=20, p_points=1e-3, seed=2),
        workloads.points(50, 120, n=12, seed=3),
        workloads.ellipses(70, 90, 8, 3, 20, seed=4),
    ]
    for m in masks:
        for pol in (0, 1):
            D, F = oracle.separable(m, pol)
            _check_invariants(m, pol, D, F)


def test_padding_translation_invariance():
    rng = np.random.default_rng(8)
    m = (rng.random((30, 41)) < 0.03).astype(np.uint8)
    D, F = oracle.separable(m)
    top, left = 5, 9
    P = np.zeros((30 + top + 4, 41 + left + 7), np.uint8)
    P[top:top + 30, left:left + 41] = m
    DP, FP = oracle.separable(P)
    Wp = P.shape[1]
    assert np.array_equal(DP[top:top + 30, left:left + 41], D)
    r, c = F // 41, F % 41
    assert np.array_equal(FP[top:top + 30, left:left + 41], (r + top) * Wp + (c + left))


def test_flip_transpose_equivariance_of_D():
    rng = np.random.default_rng(9)
    m = (rng.random((33, 47)) < 0.02).astype(np.uint8)
    D, _ = oracle.separable(m)
    for f in (np.flipud, np.fliplr, np.transpose):
        Df, _ = oracle.separable(np.ascontiguousarray(f(m)))
        assert np.array_equal(Df, f(D))


def test_polarity_complement():
    rng = np.random.default_rng(10)
    m = (rng.random((40, 40)) < 0.3).astype(np.uint8)
    D0, _ = oracle.separable(m, 0)
    D1, _ = oracle.separable(m, 1)
    assert np.all((D0 == 0) ^ (D1 == 0))


# -------------------------------------------------------------------- sqrt

def _f32_sqrt_correctly_rounded(D: int) -> np.float32:
    """Nearest fp32 to the real square root of the integer D, decided with
    exact integer arithmetic (no library square root involved): on the fp32
    grid of spacing 2^(e-23) around sqrt(D), X = isqrt(D * 4^(23-e)) is the last
    grid point at or below sqrt(D), and the midpoint test compares squares."""
    if D == 0:
        return np.float32(0)
    e = math.isqrt(D).bit_length() - 1  # 2^e <= sqrt(D) < 2^(e+1)
    sc = 4 ** (23 - e)
    X = math.isqrt(D * sc)
    # sqrt(D) is nearer to (X+1) * ulp iff 4 * D * sc > (2X + 1)^2 (never equal)
    if 4 * D * sc > (2 * X + 1) ** 2:
        X += 1
    return np.float32(math.ldexp(X, e - 23))


def test_sqrt_epilogue():
    k = np.arange(0, 46341, 7, dtype=np.int64)
    sq = (k * k).astype(np.int32)
    assert np.array_equal(oracle.sqrt_f32(sq), k.astype(np.float32))
    D = np.array([INF_SQ, 0, 1, 2, 2**31 - 2], np.int32)
    d = oracle.sqrt_f32(D)
    assert np.isinf(d[0]) and d[1] == 0 and d[2] == 1
    rng = np.random.default_rng(12)
    D = np.concatenate([rng.integers(0, 2**31 - 2, size=20000, dtype=np.int64),
                        rng.integers(2**24, 2**26, size=5000, dtype=np.int64),
                        np.arange(0, 5000, dtype=np.int64)])
    d = oracle.sqrt_f32(D.astype(np.int32))
    for Dv, dv in zip(D.tolist(), d):
        assert dv == _f32_sqrt_correctly_rounded(Dv), Dv
    assert np.all(np.diff(oracle.sqrt_f32(np.sort(D).astype(np.int32))) >= 0)
