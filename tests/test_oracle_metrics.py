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
