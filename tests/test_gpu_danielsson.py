"""Danielsson's approximate transform on the GPU (edt_danielsson): distances and
propagated relative positions bit-exact with the oracle's two scans of
Section 2.3 -- on the worked example (the printed positions), random masks of
both polarities and assorted shapes, 512 x 512 disks, and the three-site
configuration whose disconnected region the propagation misses."""
import numpy as np
import pytest

import oracle
import workloads
from tests.test_oracle_danielsson import MISSED_PIXEL, missed_mask, positions

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def edt():
    import torch
    import paper_2106_03503_amd as edt
    assert torch.cuda.is_available()
    return edt


def _run(edt, m, pol=0):
    import torch
    D, R = edt.danielsson(torch.from_numpy(m).to("cuda:0"), polarity=pol)
    torch.cuda.synchronize()
    return D.cpu().numpy(), R.cpu().numpy()


def test_paper_example(edt):
    m = workloads.paper_example()
    D, R = _run(edt, m)
    Do, Ro = oracle.danielsson(m)
    assert np.array_equal(D, Do) and np.array_equal(R, Ro)
    want = positions("fig_danielssondt_c.txt")
    ok = np.ones(want.shape, bool)
    ok[2, 2] = False  # erratum cell of the printed table
    assert np.array_equal(R[ok], want[ok])


@pytest.mark.parametrize("seed", range(12))
def test_random_masks(edt, seed):
    rng = np.random.default_rng(900 + seed)
    shapes = [(1, 1), (1, 50), (50, 1), (2, 2), (37, 65), (64, 64), (70, 129), (100, 300),
              (9, 1000), (200, 63), (33, 257), (120, 180)]
    H, W = shapes[seed]
    m = (rng.random((H, W)) < rng.choice([0.0, 0.002, 0.02, 0.1, 0.5])).astype(np.uint8)
    for pol in (0, 1):
        D, R = _run(edt, m, pol)
        Do, Ro = oracle.danielsson(m, pol)
        assert np.array_equal(D, Do), (H, W, pol)
        assert np.array_equal(R, Ro), (H, W, pol)


@pytest.mark.parametrize("shape", [(3, 8192), (5, 4160), (4, 127)])
def test_widest_rows(edt, shape):
    # rows of the largest width the call takes, and widths just past and
    # short of a multiple of 64: the sweeps walk a row 64 pixels at a time
    H, W = shape
    m = (np.random.default_rng(W).random((H, W)) < 0.001).astype(np.uint8)
    m[0, W // 3] = 1
    for pol in (0, 1):
        D, R = _run(edt, m, pol)
        Do, Ro = oracle.danielsson(m, pol)
        assert np.array_equal(D, Do) and np.array_equal(R, Ro), (H, W, pol)


def test_disks_512(edt):
    m = workloads.disks(512, 512, n_disks=30, rmin=3, rmax=40)
    for pol in (0, 1):
        D, R = _run(edt, m, pol)
        Do, Ro = oracle.danielsson(m, pol)
        assert np.array_equal(D, Do) and np.array_equal(R, Ro), pol
        assert (D >= oracle.separable(m, pol)[0]).all()


def test_missed_region(edt):
    m = missed_mask()
    D, _ = _run(edt, m)
    E, _ = oracle.separable(m)
    assert np.array_equal(D, oracle.danielsson(m)[0])
    assert D[MISSED_PIXEL] > E[MISSED_PIXEL]


def test_errors(edt):
    import torch
    for shape in ((4, 8193), (1025, 4096)):
        with pytest.raises(edt.EDTError) as e:
            edt.danielsson(torch.zeros(shape, dtype=torch.uint8, device="cuda:0"))
        assert e.value.status == -3
