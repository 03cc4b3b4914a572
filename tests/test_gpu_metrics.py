"""City-block and chessboard transforms on the GPU (edt_sq / edt_feature with
EDT_METRIC_CITYBLOCK and EDT_METRIC_CHESSBOARD): bit-exact with the oracle's
definition (O1) and, for city-block, with its four propagation scans."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def edt():
    import torch
    import paper_2106_03503_amd as edt
    assert torch.cuda.is_available()
    return edt


def _run(edt, m, pol, metric, feature):
    import torch
    mt = torch.from_numpy(m).to("cuda:0")
    if feature:
        D, F = edt.feature(mt, polarity=pol, metric=metric)
        return D.cpu().numpy(), F.cpu().numpy()
    return edt.sq(mt, polarity=pol, metric=metric).cpu().numpy(), None


def _masks():
    rng = np.random.default_rng(2106301)
    out = [("paper example", workloads.paper_example())]
    for H, W, p in [(1, 1, 1.0), (1, 300, 0.01), (300, 1, 0.01), (64, 64, 0.0), (64, 64, 1.0),
                    (97, 133, 0.002), (130, 257, 0.05), (200, 1100, 0.01), (33, 2050, 0.3),
                    (40, 4100, 0.001), (9, 9000, 0.01)]:
        out.append((f"{H}x{W} p={p}", (rng.random((H, W)) < p).astype(np.uint8)))
    out.append(("ellipses 160x300", workloads.ellipses(160, 300, 12, 3, 40, rng=rng)))
    m = np.zeros((90, 120), np.uint8)
    m[::7, ::5] = 1  # regular grid: many equidistant sites
    out.append(("grid 90x120", m))
    return out


MASKS = _masks()


@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("k", range(len(MASKS)), ids=[n for n, _ in MASKS])
def test_metric_matches_definition(edt, metric, k):
    name, m = MASKS[k]
    for pol in (0, 1):
        Db, Fb = oracle.brute_metric(m, metric, pol)
        D, F = _run(edt, m, pol, metric, feature=(metric == 1))
        assert np.array_equal(D, Db), (name, pol)
        if metric == 1:
            assert np.array_equal(F, Fb), (name, pol)
            assert np.array_equal(D, oracle.cityblock_scans(m, pol)), (name, pol)


def test_metric_errors(edt):
    import torch
    mt = torch.zeros((8, 8), dtype=torch.uint8, device="cuda:0")
    with pytest.raises(edt.EDTError) as e:
        edt.feature(mt, metric=2)  # chessboard features: not decided by the vertical pass
    assert e.value.status == -2
    with pytest.raises(edt.EDTError) as e:
        edt.sq(mt, metric=3)  # chamfer 4-3: reserved
    assert e.value.status == -2
    with pytest.raises(edt.EDTError) as e:
        edt.sq(mt, metric=4)
    assert e.value.status == -1


def test_wide_rows_chessboard_and_cityblock(edt):
    """Rows wider than the LDS forms take (the global-slot form)."""
    rng = np.random.default_rng(2106302)
    m = (rng.random((6, 20000)) < 0.002).astype(np.uint8)
    for metric in (1, 2):
        Db, Fb = oracle.brute_metric(m, metric, 0)
        D, F = _run(edt, m, 0, metric, feature=(metric == 1))
        assert np.array_equal(D, Db)
        if metric == 1:
            assert np.array_equal(F, Fb)
