"""Pins of the oracle's region labels (Section 1.1: each region stands for one
object point or a cluster of connected points; Section 1.2: 4- and
8-neighbourhood).  Connected-component labelling is not spelled out in the
paper, so the pins are the cases its text fixes (the diagonal pair of Figure
fig_neighbourhoods(b): one object under 8-neighbourhood, two under
4-neighbourhood), closed forms (checkerboards, full and empty masks, isolated
points) and an independent computation by a different algorithm (iterated
minimum over neighbours until nothing changes) on random masks."""
import numpy as np
import pytest

import oracle
import workloads


def _labels(m, pol=0, conn=8):
    _, F = oracle.separable(m, pol)
    return oracle.regions(m, F, pol, conn), F


def _components_by_min_propagation(site, conn):
    """Each site starts with its own linear index; repeat 'take the minimum
    over yourself and your site neighbours' until nothing changes."""
    H, W = site.shape
    big = np.iinfo(np.int64).max
    lab = np.where(site, np.arange(H * W, dtype=np.int64).reshape(H, W), big)
    offs = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    if conn == 8:
        offs += [(-1, -1), (-1, 1), (1, -1), (1, 1)]
    while True:
        new = lab.copy()
        for di, dj in offs:
            sh = np.full((H, W), big, np.int64)
            src = lab[max(0, di):H + min(0, di), max(0, dj):W + min(0, dj)]
            sh[max(0, -di):H + min(0, -di), max(0, -dj):W + min(0, -dj)] = src
            new = np.where(site, np.minimum(new, sh), big)
        if np.array_equal(new, lab):
            return lab
        lab = new


def test_diagonal_pair_is_one_object_in_8_and_two_in_4():
    # Figure fig_neighbourhoods(b): two groups of object pixels that touch only
    # at a corner
    m = np.zeros((6, 6), np.uint8)
    m[1:3, 1:3] = 1
    m[3:5, 3:5] = 1
    L8, F = _labels(m, 0, 8)
    L4, _ = _labels(m, 0, 4)
    site = m != 0
    assert len(set(L8[site].tolist())) == 1 and set(L8[site].tolist()) == {1 * 6 + 1}
    assert set(L4[site].tolist()) == {1 * 6 + 1, 3 * 6 + 3}


def test_checkerboards():
    m = (np.add.outer(np.arange(7), np.arange(9)) % 2 == 0).astype(np.uint8)
    L4, F = _labels(m, 0, 4)
    L8, _ = _labels(m, 0, 8)
    site = m != 0
    idx = np.arange(m.size).reshape(m.shape)
    assert np.array_equal(L4[site], idx[site])  # every site alone
    assert np.array_equal(L4, F)                # so labels are the features
    assert (L8 == 0).all()                      # one object, first site (0, 0)


def test_full_empty_and_isolated_points():
    full = np.ones((5, 7), np.uint8)
    for conn in (4, 8):
        assert (_labels(full, 0, conn)[0] == 0).all()
        assert (_labels(full, 1, conn)[0] == -1).all()   # no background pixel
        assert (_labels(np.zeros((5, 7), np.uint8), 0, conn)[0] == -1).all()
    m = workloads.points(64, 80, 12, seed=3)
    for conn in (4, 8):
        L, F = _labels(m, 0, conn)
        assert np.array_equal(L, F)


def test_paper_example_components():
    m = workloads.paper_example()
    for conn in (4, 8):
        L, F = _labels(m, 0, conn)
        assert sorted(set(L.ravel().tolist())) == [14, 27, 41, 55, 67]
        # (2,7) and (3,7) are vertical neighbours: one region labelled 27
        assert L.ravel()[37] == 27 and F.ravel()[37] == 37


@pytest.mark.parametrize("seed", range(10))
def test_regions_against_min_propagation(seed):
    rng = np.random.default_rng(500 + seed)
    H, W = int(rng.integers(1, 30)), int(rng.integers(1, 30))
    m = (rng.random((H, W)) < rng.choice([0.05, 0.3, 0.5, 0.7])).astype(np.uint8)
    for pol in (0, 1):
        site = (m != 0) if pol == 0 else (m == 0)
        _, F = oracle.separable(m, pol)
        for conn in (4, 8):
            L = oracle.regions(m, F, pol, conn)
            comp = _components_by_min_propagation(site, conn)
            want = np.where(F >= 0, comp.ravel()[np.maximum(F, 0)], -1)
            assert np.array_equal(L, want), (seed, pol, conn)
