"""Region labels on the GPU (edt_regions): bit-exact with the oracle's flood
fill over the same feature transform, for both neighbourhoods and both
polarities, on random, tie-heavy, blob and point masks, on pitched buffers,
on images without sites, and at 16384 x 16384 where 30 isolated points make
every pixel's label its feature."""
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


def _gpu_regions(edt, m, pol, conn, pad=0):
    import torch
    dev = torch.device("cuda:0")
    H, W = m.shape
    mask = torch.from_numpy(m).to(dev)
    Fb = torch.full((H, W + pad), -7, dtype=torch.int32, device=dev)
    Lb = torch.full((H, W + pad), -9, dtype=torch.int32, device=dev)
    _, F = edt.feature(mask, polarity=pol, want_dist=False, out_feat=Fb[:, :W])
    L = edt.regions(mask, F, polarity=pol, connectivity=conn, out=Lb[:, :W])
    torch.cuda.synchronize()
    if pad:
        assert bool((Lb[:, W:] == -9).all())  # padding never written
    return F.cpu().numpy(), L.cpu().numpy()


def _masks():
    rng = np.random.default_rng(2106401)
    out = [("paper example", workloads.paper_example())]
    for H, W, p in [(1, 1, 1.0), (1, 200, 0.3), (200, 1, 0.3), (50, 60, 0.0), (50, 60, 1.0),
                    (97, 133, 0.45), (64, 300, 0.6), (130, 257, 0.05), (33, 2050, 0.5)]:
        out.append((f"{H}x{W} p={p}", (rng.random((H, W)) < p).astype(np.uint8)))
    out.append(("checkerboard", (np.add.outer(np.arange(40), np.arange(57)) % 2).astype(np.uint8)))
    out.append(("ellipses 300x400", workloads.ellipses(300, 400, 25, 3, 60, rng=rng)))
    out.append(("disks 512", workloads.disks(512, 512, n_disks=40, rmin=3, rmax=60)))
    return out


MASKS = _masks()


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("k", range(len(MASKS)), ids=[n for n, _ in MASKS])
def test_regions_match_oracle(edt, k, conn):
    name, m = MASKS[k]
    for pol in (0, 1):
        F, L = _gpu_regions(edt, m, pol, conn, pad=3 if k % 2 else 0)
        _, Fo = oracle.separable(m, pol)
        assert np.array_equal(F, Fo), (name, pol)
        assert np.array_equal(L, oracle.regions(m, Fo, pol, conn)), (name, pol, conn)


def test_regions_of_isolated_points_are_the_features_16384(edt):
    import torch
    m = workloads.points(16384, 16384, 30)
    dev = torch.device("cuda:0")
    mask = torch.from_numpy(m).to(dev)
    _, F = edt.feature(mask, want_dist=False)
    for conn in (4, 8):
        L = edt.regions(mask, F, connectivity=conn)
        torch.cuda.synchronize()
        assert bool((L == F).all())
        del L
    # one 8-connected object spanning the whole image: a full-height diagonal
    m2 = np.zeros((16384, 16384), np.uint8)
    idx = np.arange(16384)
    m2[idx, idx] = 1
    mask2 = torch.from_numpy(m2).to(dev)
    _, F2 = edt.feature(mask2, want_dist=False)
    L8 = edt.regions(mask2, F2, connectivity=8)
    L4 = edt.regions(mask2, F2, connectivity=4)
    torch.cuda.synchronize()
    assert bool((L8 == 0).all())  # the whole diagonal is one object, first site (0, 0)
    assert bool((L4 == F2).all())  # under 4-neighbourhood every pixel is alone


def test_regions_errors(edt):
    import torch
    mt = torch.zeros((8, 8), dtype=torch.uint8, device="cuda:0")
    F = torch.zeros((8, 8), dtype=torch.int32, device="cuda:0")
    with pytest.raises(edt.EDTError) as e:
        edt.regions(mt, F, connectivity=6)
    assert e.value.status == -1
    with pytest.raises(edt.EDTError) as e:
        edt.regions(mt, F, out=F)  # labels may not overlap the feature transform
    assert e.value.status == -1
