"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Small and mid-size images are compared element by element with the oracle's
separable transform (itself pinned to brute force and to the paper's tables in
test_oracle.py) and, where cheap, with brute force directly.  Full-size
images are compared with the oracle in full where it finishes in seconds, and
always at sampled pixels by brute force plus invariants that hold at any size.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

INF_SQ = 2**31 - 1


@pytest.fixture(scope="module")
def edt():
    import torch
    import paper_2106_03503_amd as edt
    assert torch.cuda.is_available()
    return edt


def run(edt, m, pol, pitch_pad=0, out_pad=0, col_off=0):
    import torch
    dev = torch.device("cuda:0")
    H, W = m.shape
    big = torch.zeros((H, col_off + W + pitch_pad), dtype=torch.uint8, device=dev)
    big[:, col_off:col_off + W] = torch.from_numpy(m).to(dev)
    mask = big[:, col_off:col_off + W]
    Dbuf = torch.full((H, W + out_pad), -7, dtype=torch.int32, device=dev)
    Fbuf = torch.full((H, W + out_pad), -7, dtype=torch.int32, device=dev)
    D, F = edt.feature(mask, polarity=pol, out_dist=Dbuf[:, :W], out_feat=Fbuf[:, :W])
    Dsq = edt.sq(mask, polarity=pol)
    torch.cuda.synchronize()
    if out_pad:
        # the padding columns are never written
        assert bool((Dbuf[:, W:] == -7).all()) and bool((Fbuf[:, W:] == -7).all())
    return D.cpu().numpy(), F.cpu().numpy(), Dsq.cpu().numpy()


def check_exact(edt, m, pol, **kw):
    D, F, Dsq = run(edt, m, pol, **kw)
    Do, Fo = oracle.separable(m, pol)
    assert np.array_equal(D, Do), f"D differs on {m.shape} pol={pol}"
    assert np.array_equal(F, Fo), f"F differs on {m.shape} pol={pol}"
    assert np.array_equal(Dsq, Do), f"edt_sq differs on {m.shape} pol={pol}"
    return D, F


def test_paper_example_matches_printed_table(edt):
    from tests.golden_io import table
    m = workloads.paper_example()
    D, F = check_exact(edt, m, 0)
    assert np.array_equal(D, table("fig_eedt_c_final.txt"))


@pytest.mark.parametrize("pol", [0, 1])
def test_bernoulli_256_and_crop_against_brute_force(edt, pol):
    m = workloads.bernoulli(256, 256, 0.01)
    D, F = check_exact(edt, m, pol)
    Db, Fb = oracle.brute(m, pol, contour_only=True)
    assert np.array_equal(D, Db) and np.array_equal(F, Fb)
    crop = np.ascontiguousarray(m[:64, :64])
    Dc, Fc, _ = run(edt, crop, pol)
    Db, Fb = oracle.brute(crop, pol)
    assert np.array_equal(Dc, Db) and np.array_equal(Fc, Fb)


@pytest.mark.parametrize("shape", [(1, 1), (1, 300), (300, 1), (63, 65), (64, 64), (65, 63),
                                   (127, 129), (129, 257), (200, 513), (3, 1000)])
@pytest.mark.parametrize("pol", [0, 1])
def test_edge_shapes_random(edt, shape, pol):
    rng = np.random.default_rng(hash(shape) % 1000 + pol)
    m = (rng.random(shape) < 0.05).astype(np.uint8)
    check_exact(edt, m, pol)


@pytest.mark.parametrize("kind", ["empty", "full", "corner", "one_far", "one_row", "one_col"])
@pytest.mark.parametrize("pol", [0, 1])
def test_degenerate_masks(edt, kind, pol):
    H, W = 150, 170
    m = np.zeros((H, W), np.uint8)
    if kind == "full":
        m[:] = 1
    elif kind == "corner":
        m[0, 0] = 1
    elif kind == "one_far":
        m[H - 1, W - 1] = 1
    elif kind == "one_row":
        m[77, ::13] = 1
    elif kind == "one_col":
        m[::11, 91] = 1
    D, F = check_exact(edt, m, pol)
    site = (m != 0) != (pol == 1)
    if not site.any():
        assert np.all(D == INF_SQ) and np.all(F == -1)
    if site.all():
        assert np.all(D == 0)


def test_tie_heavy_symmetric_masks(edt):
    rng = np.random.default_rng(99)
    for t in range(20):
        H, W = int(rng.integers(20, 90)), int(rng.integers(20, 90))
        q = (rng.random(((H + 1) // 2, (W + 1) // 2)) < rng.uniform(0.01, 0.2)).astype(np.uint8)
        m = np.zeros((H, W), np.uint8)
        m[:q.shape[0], :q.shape[1]] = q
        m[:, W - q.shape[1]:] |= m[:, :q.shape[1]][:, ::-1]
        m[H - q.shape[0]:, :] |= m[:q.shape[0], :][::-1, :]
        check_exact(edt, m, t % 2)
        Db, Fb = oracle.brute(m, t % 2)
        D, F, _ = run(edt, m, t % 2)
        assert np.array_equal(D, Db) and np.array_equal(F, Fb)


def test_pitched_mask_and_outputs(edt):
    m = workloads.bernoulli(77, 301, 0.02, seed=5)
    check_exact(edt, m, 0, pitch_pad=37, out_pad=11)
    check_exact(edt, m, 1, pitch_pad=1, out_pad=3)


def test_wide_rows_use_the_global_row_slots(edt):
    # rows wider than what the row pass keeps in LDS
    for W, p in ((11000, 0.001), (16384, 0.0005), (20001, 0.3)):
        m = workloads.bernoulli(70, W, p, seed=W)
        check_exact(edt, m, 0)
    m = workloads.points(40, 16384, n=5, seed=1)
    check_exact(edt, m, 1)  # every column holds sites: dense wide rows


def test_disks_mid_size_both_polarities(edt):
    m = workloads.disks(1024, 1024, n_disks=40, rmin=3, rmax=60, p_points=1e-4, seed=3)
    for pol in (0, 1):
        check_exact(edt, m, pol)


def test_sqrt_epilogue_matches_oracle(edt):
    import torch
    m = workloads.bernoulli(300, 400, 0.001, seed=2)
    D, _, _ = run(edt, m, 0)
    d = edt.sqrt_f32(torch.from_numpy(D).cuda())
    big = torch.tensor([0, 1, 2, 3, 2**31 - 2, INF_SQ, 536805378], dtype=torch.int32).cuda()
    d2 = edt.sqrt_f32(big)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), oracle.sqrt_f32(D))
    assert np.array_equal(d2.cpu().numpy(), oracle.sqrt_f32(big.cpu().numpy()))


@pytest.mark.parametrize("W", [1025, 2048, 2049, 4096, 4097, 8192, 8193, 16384, 16385, 32767])
def test_dense_row_forms_by_width(edt, W):
    # every width class of the dense row pass (and the global-slot form)
    H = 33 if W > 16384 else 70
    m = workloads.bernoulli(H, W, 0.2, seed=W)
    check_exact(edt, m, 0)
    check_exact(edt, m, 1)


@pytest.mark.parametrize("ncols", [1, 2, 63, 64, 65, 1023, 1024, 1025, 1100])
def test_candidate_count_around_the_sparse_limit(edt, ncols):
    # exactly ncols columns hold sites: the sparse form takes up to 1024
    rng = np.random.default_rng(ncols)
    H, W = 90, 3000
    m = np.zeros((H, W), np.uint8)
    cols = rng.choice(W, size=ncols, replace=False)
    m[rng.integers(0, H, size=ncols), cols] = 1
    check_exact(edt, m, 0)


@pytest.mark.parametrize("W,pad", [(1029, 11), (1029, 3), (1029, 0), (1024, 0), (1040, 0),
                                   (1036, 0), (17, 15), (33, 0)])
def test_mask_load_paths(edt, W, pad):
    # mask row pitch = W + pad bytes: multiples of 16 and of 4 take the wide
    # and word loads, others the byte loads; widths not a multiple of the
    # lane's column count leave a ragged last lane
    m = workloads.bernoulli(131, W, 0.01, seed=W + pad)
    check_exact(edt, m, 0, pitch_pad=pad)
    check_exact(edt, m, 1, pitch_pad=pad)


@pytest.mark.parametrize("W,off,pad", [(1029, 1, 0), (300, 3, 1), (66, 2, 0), (5, 1, 0),
                                       (1024, 4, 0)])
def test_mask_base_off_word_boundary(edt, W, off, pad):
    # the mask starts `off` bytes into its buffer: rows then begin inside a
    # 4-byte word and the band-bit pass reads the words around each lane's bytes
    m = workloads.bernoulli(131, W, 0.02, seed=3 * W + off)
    check_exact(edt, m, 0, pitch_pad=pad, col_off=off)
    check_exact(edt, m, 1, pitch_pad=pad, col_off=off)


@pytest.mark.parametrize("pol", [0, 1])
def test_tallest_image_rows_next_to_the_no_site_marker(edt, pol):
    # H = 32767, the largest side: site rows up to 32766 travel as int16 next to
    # the "no site below" marker (INT16_MAX), squared distances reach ~2^30,
    # and the band carries of a single image span 512 bands
    H, W = 32767, 64
    m = np.zeros((H, W), np.uint8)
    m[0, 3] = m[H - 1, 60] = 1          # opposite corners of the column range
    m[H - 1, 0] = m[0, W - 1] = 1
    m[H // 2, 20] = 1
    m[:, 41] = 0                         # column 41 holds no object pixel
    m[17000:17010, 50] = 1               # a short vertical run mid-image
    D, F = check_exact(edt, m, pol)
    if pol == 0:
        assert D.max() <= (H - 1) ** 2 + (W - 1) ** 2
        assert D[H // 4, 41] > 0
    else:
        # inverted: the sites are everything but these pixels and column 41
        # is all sites
        assert (D[:, 41] == 0).all()


@pytest.mark.parametrize("pol", [0, 1])
def test_tall_single_image_more_than_256_bands(edt, pol):
    # 20000 rows = 313 bands: the single-image band carries of images with more
    # than the 256 bands whose masks the column slices keep in registers (the
    # form that reads them again for each sweep)
    H, W = 20000, 300
    rng = np.random.default_rng(2106111 + pol)
    m = (rng.random((H, W)) < 2e-4).astype(np.uint8)
    m[:, 7] = 0
    m[:, 150] = 0
    m[rng.integers(0, H, 40), 150] = 1   # a column with a few far-apart sites
    m[12345:12400, 200:203] = 1
    check_exact(edt, m, pol)


@pytest.mark.parametrize("kind", ["diagonal", "top_row", "two_rows", "sparse_top"])
def test_dense_rows_with_far_sites(edt, kind):
    # every column holds a site (the segment path), but many pixels lie far from
    # all of them: their bounded search over segment envelopes gives up and the
    # row is merged instead; rows near the sites keep the bounded search
    H, W = 600, 3000
    m = np.zeros((H, W), np.uint8)
    cols = np.arange(W)
    if kind == "diagonal":
        m[(cols * (H - 1)) // (W - 1), cols] = 1
    elif kind == "top_row":
        m[0, :] = 1
    elif kind == "two_rows":
        m[0, ::2] = 1
        m[H - 1, 1::2] = 1
    else:
        m[0, :] = 1
        m[1:, :] = (np.random.default_rng(5).random((H - 1, W)) < 2e-5)
    check_exact(edt, m, 0)
    check_exact(edt, m, 1)


@pytest.mark.parametrize("W", [2100, 4097, 9000])
def test_segment_path_with_ties(edt, W):
    # more than 1024 listed columns (the segment scan and the bounded search
    # over segments) on tie-heavy masks: a regular grid of sites, where many
    # pixels are equidistant from several sites, and a mirror-symmetric mask
    H = 150
    g = np.zeros((H, W), np.uint8)
    g[::5, ::2] = 1
    check_exact(edt, g, 0)
    check_exact(edt, g, 1)
    rng = np.random.default_rng(W)
    half = (rng.random((H, W // 2)) < 0.01).astype(np.uint8)
    half[:, ::3] |= (rng.random((H, (W // 2 + 2) // 3)) < 0.05).astype(np.uint8)
    m = np.concatenate([half, half[:, ::-1]], axis=1)
    m = np.concatenate([m, np.zeros((H, W - m.shape[1]), np.uint8)], axis=1)
    m[: H // 2] |= m[H // 2:][: H // 2][::-1]
    check_exact(edt, m, 0)
    check_exact(edt, m, 1)
