"""Parity at the full sizes of the measured workloads, in the launch
configuration bench.py times:

* 16384 x 16384 with 30 object points through edt_feature: every pixel against
  the definition (the oracle's brute force at all 268M pixels, in row chunks),
  plus the same shape with one object pixel in a corner (closed form
  D = i^2 + j^2, F = 0) and with none (sentinels);
* 4096 x 4096 disks, both polarities: every pixel against the oracle's
  separable transform, and a sample against its brute force;
* dense disks at 16384 x 16384 and 8192 x 8192 (segments of 512 and 256
  candidates), both polarities: the same;
* the 2048-image ragged batch through edt_batch_submit with the schedule the
  autotuner picks (lanes up to 1024 columns, largest first): every image
  against the oracle's separable transform."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

INF_SQ = oracle.INF_SQ


@pytest.fixture(scope="module")
def edt():
    import torch
    import paper_2106_03503_amd as edt
    assert torch.cuda.is_available()
    return edt


def _feature_full(edt, m, pol):
    import torch
    dev = torch.device("cuda:0")
    H, W = m.shape
    mask = torch.from_numpy(m).to(dev)
    D = torch.empty((H, W), dtype=torch.int32, device=dev)
    F = torch.empty((H, W), dtype=torch.int32, device=dev)
    ws = torch.empty(edt.workspace_bytes(H, W, True), dtype=torch.uint8, device=dev)
    for _ in range(2):  # the second call runs on a workspace the first one left dirty
        D.fill_(-7)
        F.fill_(-7)
        edt.feature(mask, polarity=pol, out_dist=D, out_feat=F, workspace=ws)
    torch.cuda.synchronize()
    del ws
    return D, F


def test_points_16384_every_pixel_against_the_definition(edt):
    import torch
    m = workloads.points(16384, 16384, 30)
    H, W = m.shape
    D, F = _feature_full(edt, m, 0)
    rows = 512
    for r0 in range(0, H, rows):
        lin = np.arange(r0 * W, (r0 + rows) * W, dtype=np.int64)
        Do, Fo = oracle.brute_at(m, lin)
        d = D[r0:r0 + rows].cpu().numpy().ravel()
        f = F[r0:r0 + rows].cpu().numpy().ravel()
        bad = np.flatnonzero((d != Do) | (f != Fo))
        assert bad.size == 0, (r0, lin[bad[:5]], d[bad[:5]], Do[bad[:5]], f[bad[:5]], Fo[bad[:5]])
    del D, F
    torch.cuda.empty_cache()


def test_corner_and_empty_16384_closed_forms(edt):
    import torch
    H = W = 16384
    m = workloads.corner(H, W)
    D, F = _feature_full(edt, m, 0)
    i = torch.arange(H, device=D.device, dtype=torch.int64)
    for r0 in range(0, H, 2048):
        ii = i[r0:r0 + 2048, None]
        want = ii * ii + i[None, :] * i[None, :]  # row^2 + column^2 to site (0, 0)
        assert bool((D[r0:r0 + 2048].to(torch.int64) == want).all()), r0
    assert bool((F == 0).all())
    del D, F
    m = np.zeros((H, W), np.uint8)
    D, F = _feature_full(edt, m, 0)
    assert bool((D == INF_SQ).all()) and bool((F == -1).all())
    del D, F
    torch.cuda.empty_cache()


@pytest.mark.parametrize("pol", [0, 1])
def test_disks_4096_every_pixel_against_the_oracle(edt, pol):
    m = workloads.disks(4096, 4096)
    D, F = _feature_full(edt, m, pol)
    Do, Fo = oracle.separable(m, pol)
    d, f = D.cpu().numpy(), F.cpu().numpy()
    assert np.array_equal(d, Do) and np.array_equal(f, Fo)
    rng = np.random.default_rng(pol)
    lin = rng.choice(m.size, 20000, replace=False)
    Db, Fb = oracle.brute_at(m, lin, pol)
    assert np.array_equal(d.ravel()[lin], Db) and np.array_equal(f.ravel()[lin], Fb)


@pytest.mark.parametrize("pol", [0, 1])
def test_dense_16384_every_pixel_against_the_oracle(edt, pol):
    # the dense 16384^2 disk image (3200 disks of radius 5-200 and isolated
    # points) in the configuration bench.py times: segments of 512 candidates,
    # the bounded search over them and the merge for the rows it leaves
    import torch
    m = workloads.disks(16384, 16384, n_disks=3200)
    D, F = _feature_full(edt, m, pol)
    d, f = D.cpu().numpy(), F.cpu().numpy()
    del D, F
    torch.cuda.empty_cache()
    Do, Fo = oracle.separable(m, pol)
    assert np.array_equal(d, Do) and np.array_equal(f, Fo)
    del Do, Fo
    rng = np.random.default_rng(10 + pol)
    lin = rng.choice(m.size, 2000, replace=False)
    Db, Fb = oracle.brute_at(m, lin, pol)
    assert np.array_equal(d.ravel()[lin], Db) and np.array_equal(f.ravel()[lin], Fb)


@pytest.mark.parametrize("pol", [0, 1])
def test_dense_8192_every_pixel_against_the_oracle(edt, pol):
    # 8192^2 disks at the density of the 16384^2 image: segments of 256
    # candidates (the longest length that still gives 4096 scan items here)
    import torch
    m = workloads.disks(8192, 8192, n_disks=800)
    D, F = _feature_full(edt, m, pol)
    d, f = D.cpu().numpy(), F.cpu().numpy()
    del D, F
    torch.cuda.empty_cache()
    Do, Fo = oracle.separable(m, pol)
    assert np.array_equal(d, Do) and np.array_equal(f, Fo)
    rng = np.random.default_rng(20 + pol)
    lin = rng.choice(m.size, 2000, replace=False)
    Db, Fb = oracle.brute_at(m, lin, pol)
    assert np.array_equal(d.ravel()[lin], Db) and np.array_equal(f.ravel()[lin], Fb)


def test_batch_2048_every_image_against_the_oracle(edt):
    import torch
    dev = torch.device("cuda:0")
    imgs = workloads.ragged_batch(2048)
    plan = edt.BatchPlan([(mm.shape[0], mm.shape[1], p, True) for mm, p in imgs])
    plan.set_schedule(1024, True)
    mask = plan.pack([mm for mm, _ in imgs], dev)
    D, F = plan.outputs(dev)
    D.fill_(-7)
    F.fill_(-7)
    ws = plan.submit(mask, D, F)
    ws = plan.submit(mask, D, F, workspace=ws)  # graph replay on the same buffers
    torch.cuda.synchronize()
    Dh, Fh = D.cpu(), F.cpu()
    for q, (mm, pol) in enumerate(imgs):
        Do, Fo = oracle.separable(mm, pol)
        assert np.array_equal(plan.image(Dh, q).numpy(), Do), (q, mm.shape, pol)
        assert np.array_equal(plan.image(Fh, q).numpy(), Fo), (q, mm.shape, pol)
    plan.close()
