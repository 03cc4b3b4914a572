"""fp32 Euclidean distances written by the row pass itself (edt_dist_f32):
bit-exact with the oracle's square root of its squared distances (fp64 root
rounded to fp32, +inf without a site) and with the library's two-pass path
(edt_sq, then edt_sqrt_f32), with features equal to edt_feature's, for each
row form: the one-wavefront form (few listed columns), the chunked form
(1024 < W, other metrics' path widths), the segment scan and search (W > 1024,
dense rows), in both polarities, plus ragged and site-free images."""
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


def _check(edt, m, pol, with_oracle=True):
    import torch
    mt = torch.from_numpy(m).to("cuda:0")
    Df, Ff = edt.dist_f32(mt, polarity=pol, want_feature=True)
    D2, F2 = edt.feature(mt, polarity=pol)
    two_pass = edt.sqrt_f32(D2)
    Dn, _ = edt.dist_f32(mt, polarity=pol)  # no feature output
    torch.cuda.synchronize()
    assert Df.dtype == torch.float32
    assert torch.equal(Df.view(torch.int32), two_pass.view(torch.int32))
    assert torch.equal(Dn.view(torch.int32), two_pass.view(torch.int32))
    assert torch.equal(Ff, F2)
    if with_oracle:
        Do, Fo = oracle.separable(m, pol)
        want = oracle.sqrt_f32(Do)
        assert np.array_equal(Df.cpu().numpy().view(np.int32), want.view(np.int32))
        assert np.array_equal(Ff.cpu().numpy(), Fo)


@pytest.mark.parametrize("shape,density", [((37, 65), 0.01), ((300, 500), 0.002),
                                           ((64, 1025), 0.3), ((129, 2048), 0.05),
                                           ((70, 3000), 0.5), ((33, 8193), 0.2)])
def test_random_masks_both_polarities(edt, shape, density):
    H, W = shape
    m = (np.random.default_rng(H * 7 + W).random((H, W)) < density).astype(np.uint8)
    for pol in (0, 1):
        _check(edt, m, pol)


def test_disks_dense_rows(edt):
    # dense rows of 2048 columns: the segment scan and search
    m = workloads.disks(1024, 2048, n_disks=60, rmin=5, rmax=80)
    for pol in (0, 1):
        _check(edt, m, pol)


def test_points_sparse_rows(edt):
    m = workloads.points(512, 4096, n=30)
    _check(edt, m, 0)


def test_site_free_and_full(edt):
    import torch
    for m in (np.zeros((5, 70), np.uint8), np.ones((6, 1030), np.uint8)):
        _check(edt, m, 0)
    D, _ = edt.dist_f32(torch.zeros((3, 9), dtype=torch.uint8, device="cuda:0"))
    torch.cuda.synchronize()
    assert torch.isinf(D).all() and (D > 0).all()


def test_dense_4096_against_the_two_pass_path(edt):
    # the 4096^2 disk image, every pixel against edt_sq + edt_sqrt_f32 and on
    # sampled pixels against the oracle's brute force
    import torch
    m = workloads.disks(4096, 4096)
    _check(edt, m, 0, with_oracle=False)
    Df, _ = edt.dist_f32(torch.from_numpy(m).to("cuda:0"))
    lin = np.random.default_rng(5).choice(m.size, 20000, replace=False)
    Db, _ = oracle.brute_at(m, lin)
    got = Df.cpu().numpy().reshape(-1)[lin]
    assert np.array_equal(got.view(np.int32), oracle.sqrt_f32(Db).view(np.int32))
