"""Pins of the oracle for the other exact metrics of the Minkowski family
(Eq. eq_Minkowski): city-block (e = 1) and chessboard (e = infinity).

The brute-force definition is pinned by the distance tables the paper prints
from a centre pixel, and the four-scan city-block transform of Section 2.1 by
the tables of its worked example; the two are then checked against each other
on random masks, where the scans share nothing with the definition."""
import numpy as np
import pytest

import oracle
import workloads
from tests.golden_io import INF, table

INF_SQ = oracle.INF_SQ


def _centre_site(polarity=0):
    m = np.zeros((9, 10), np.uint8)
    m[4, 4] = 1
    return m if polarity == 0 else 1 - m


@pytest.mark.parametrize("polarity", [0, 1])
def test_cityblock_definition_matches_figure(polarity):
    D, F = oracle.brute_metric(_centre_site(polarity), 1, polarity)
    assert np.array_equal(D, table("fig_cityblock_b.txt"))
    assert (F == 4 * 10 + 4).all()


@pytest.mark.parametrize("polarity", [0, 1])
def test_chessboard_definition_matches_figure(polarity):
    D, F = oracle.brute_metric(_centre_site(polarity), 2, polarity)
    assert np.array_equal(D, table("fig_chessboard_b.txt"))
    assert (F == 4 * 10 + 4).all()


def test_cityblock_scans_vertical_stage_matches_figure():
    D = oracle.cityblock_scans(workloads.paper_example(), stages=2).astype(np.int64)
    D[D == INF_SQ] = INF
    assert np.array_equal(D, table("fig_cityblockdt_parallel_b.txt"))


def test_cityblock_final_matches_figure_but_the_erratum():
    m = workloads.paper_example()
    want = table("fig_cityblockdt_c.txt")
    scans = oracle.cityblock_scans(m)
    brute, _ = oracle.brute_metric(m, 1)
    ok = np.ones(want.shape, bool)
    ok[5, 8] = False  # printed 3; the nearest object pixel is 2 steps away
    for D in (scans, brute):
        assert np.array_equal(D[ok], want[ok])
        assert D[5, 8] == 2


@pytest.mark.parametrize("seed", range(12))
def test_cityblock_scans_equal_definition(seed):
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(1, 40)), int(rng.integers(1, 40))
    m = (rng.random((H, W)) < rng.choice([0.0, 0.01, 0.1, 0.5, 1.0])).astype(np.uint8)
    for pol in (0, 1):
        brute, F = oracle.brute_metric(m, 1, pol)
        assert np.array_equal(oracle.cityblock_scans(m, pol), brute)


@pytest.mark.parametrize("metric", [1, 2])
def test_metric_closed_forms_and_invariants(metric):
    # one site in a corner: d = i + j (city-block) or max(i, j) (chessboard)
    m = np.zeros((13, 17), np.uint8)
    m[0, 0] = 1
    D, F = oracle.brute_metric(m, metric)
    i, j = np.mgrid[0:13, 0:17]
    assert np.array_equal(D, i + j if metric == 1 else np.maximum(i, j))
    assert (F == 0).all()
    # no site: infinity and no feature; every pixel a site: zero, own index
    D, F = oracle.brute_metric(np.zeros((5, 6), np.uint8), metric)
    assert (D == INF_SQ).all() and (F == -1).all()
    D, F = oracle.brute_metric(np.ones((5, 6), np.uint8), metric)
    assert (D == 0).all() and np.array_equal(F, np.arange(30).reshape(5, 6))
    # random masks: F is a site at distance D, no site is nearer, and of the
    # sites at distance D it has the smallest index; chessboard <= city-block
    rng = np.random.default_rng(5 + metric)
    m = (rng.random((19, 23)) < 0.05).astype(np.uint8)
    D, F = oracle.brute_metric(m, metric)
    r, c = np.nonzero(m)
    for p in range(m.size):
        pi, pj = divmod(p, 23)
        di, dj = np.abs(r - pi), np.abs(c - pj)
        d = di + dj if metric == 1 else np.maximum(di, dj)
        assert D.flat[p] == d.min()
        assert F.flat[p] == (r * 23 + c)[d == d.min()].min()
    D1, _ = oracle.brute_metric(m, 1)
    D2, _ = oracle.brute_metric(m, 2)
    assert (D2 <= D1).all() and (D1 <= 2 * D2).all()


@pytest.mark.parametrize("pol", [0, 1])
def test_chessboard_feature_is_the_squares_topmost_leftmost_site(pol):
    """Under the chessboard metric every site of the square of half-side D
    around a pixel lies at distance exactly D (D being the smallest distance),
    so the nearest site with the smallest index is the square's topmost site,
    leftmost among those: a characterisation by slicing, checked against the
    oracle's features (smallest index among the nearest)."""
    rng = np.random.default_rng(2106311 + pol)
    for H, W, p in [(17, 29, 0.03), (23, 11, 0.1), (31, 31, 0.01), (9, 40, 0.2)]:
        m = (rng.random((H, W)) < p).astype(np.uint8)
        site = (m != 0) if pol == 0 else (m == 0)
        if not site.any():
            continue
        D, F = oracle.brute_metric(m, 2, pol)
        for i in range(H):
            for j in range(W):
                d = int(D[i, j])
                box = site[max(0, i - d):i + d + 1, max(0, j - d):j + d + 1]
                rows = np.nonzero(box.any(axis=1))[0]
                r = rows[0]
                c = np.nonzero(box[r])[0][0]
                assert F[i, j] == (max(0, i - d) + r) * W + max(0, j - d) + c, (i, j)
                # and no site lies strictly inside the square
                inner = site[max(0, i - d + 1):i + d, max(0, j - d + 1):j + d]
                assert not inner.any()


# ---------------------------------------------------------------- chamfer 4-3

def _float_table(name):
    import os
    from tests.golden_io import GOLDEN
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                rows.append([float(v) for v in line])
    return np.array(rows)


@pytest.mark.parametrize("polarity", [0, 1])
def test_chamfer_definition_matches_figure(polarity):
    # Figure fig_chamfer(b) prints (d/3)^2 rounded to one decimal
    D, F = oracle.brute_metric(_centre_site(polarity), 3, polarity)
    assert np.array_equal(np.round(10 * (D / 3.0) ** 2) / 10, _float_table("fig_chamfer_b.txt"))
    assert (F == 4 * 10 + 4).all()


def test_chamfer_forward_scan_matches_figure_but_the_erratum():
    D = oracle.chamfer_scans(workloads.paper_example(), passes=1).astype(np.int64)
    D[D == INF_SQ] = INF
    want = table("fig_chamfer43dt_a.txt")
    ok = np.ones(want.shape, bool)
    ok[8, 1] = False  # printed 14; the upper neighbour's 9 + 3 is smaller
    assert np.array_equal(D[ok], want[ok])
    assert D[8, 1] == 12 and D[7, 1] == 9


def test_chamfer_final_matches_figure():
    m = workloads.paper_example()
    want = table("fig_chamfer43dt_b.txt")
    assert np.array_equal(oracle.chamfer_scans(m), want)
    assert np.array_equal(oracle.brute_metric(m, 3)[0], want)


@pytest.mark.parametrize("seed", range(12))
def test_chamfer_scans_equal_definition(seed):
    # the two raster scans reach, at every pixel, the shortest 3/4-step path
    # to the nearest site, which the definition takes as min(di,dj) diagonal
    # and |di-dj| straight steps
    rng = np.random.default_rng(100 + seed)
    H, W = int(rng.integers(1, 40)), int(rng.integers(1, 40))
    m = (rng.random((H, W)) < rng.choice([0.0, 0.005, 0.05, 0.3, 1.0])).astype(np.uint8)
    for pol in (0, 1):
        assert np.array_equal(oracle.chamfer_scans(m, pol), oracle.brute_metric(m, 3, pol)[0])


def test_chamfer_bounds_against_euclidean():
    # d/3 lies within [4/(3 sqrt 2), sqrt(10)/3] of the Euclidean distance
    # (offsets along a diagonal, and with |di| = 3 |dj|), and both ends are met
    rng = np.random.default_rng(7)
    m = (rng.random((60, 70)) < 0.003).astype(np.uint8)
    C, _ = oracle.brute_metric(m, 3)
    E, _ = oracle.brute(m)
    e = np.sqrt(E.astype(np.float64))
    c = C / 3.0
    nz = E > 0
    lo, hi = 4 / (3 * np.sqrt(2)), np.sqrt(10) / 3
    assert (c[nz] >= lo * e[nz] - 1e-12).all() and (c[nz] <= hi * e[nz] + 1e-12).all()
    one = np.zeros((31, 31), np.uint8)
    one[15, 15] = 1
    C1, _ = oracle.brute_metric(one, 3)
    assert C1[15 + 9, 15 + 9] == 36 and C1[15 + 9, 15 + 3] == 30  # diagonal; di = 3 dj


@pytest.mark.parametrize("metric", [1, 2, 3])
def test_sampled_definition_equals_full_definition(metric):
    """brute_metric_at (the definition at listed pixels, used where the full
    definition is too slow) gives the full definition's (D, F) at every pixel
    it is asked for, in any order, both polarities; and at the printed
    centre-pixel tables it reproduces the figures through that agreement."""
    rng = np.random.default_rng(4100 + metric)
    for _ in range(6):
        H, W = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        m = (rng.random((H, W)) < rng.choice([0.01, 0.1, 0.5])).astype(np.uint8)
        for pol in (0, 1):
            Db, Fb = oracle.brute_metric(m, metric, pol)
            lin = rng.permutation(H * W)
            D, F = oracle.brute_metric_at(m, metric, lin, pol)
            assert np.array_equal(D, Db.reshape(-1)[lin])
            assert np.array_equal(F, Fb.reshape(-1)[lin])
