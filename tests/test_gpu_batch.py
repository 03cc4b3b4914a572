"""Batched transform of images of uneven size: bit-exact with the oracle and
with the single-image path, on first submission and on graph replays."""
import os

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


def _images(seed, n, extra=()):
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n):
        H, W = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        kind = q % 4
        if kind == 0:
            m = (rng.random((H, W)) < rng.uniform(0, 0.2)).astype(np.uint8)
        elif kind == 1:
            m = workloads.ellipses(H, W, int(rng.integers(1, 8)), 2, 30, rng=rng)
        elif kind == 2:
            m = np.zeros((H, W), np.uint8)
            m[rng.integers(0, H, 3), rng.integers(0, W, 3)] = 1
        else:
            m = np.zeros((H, W), np.uint8)  # no object at all
        out.append((m, int(rng.integers(0, 2)), bool(rng.integers(0, 2))))
    for (H, W, p) in extra:
        out.append(((rng.random((H, W)) < p).astype(np.uint8), int(rng.integers(0, 2)), True))
    return out


def _check_batch(edt, imgs, want_dist=True, submits=2, fresh_buffers=False, schedule=None):
    import torch
    dev = torch.device("cuda:0")
    plan = edt.BatchPlan([(m.shape[0], m.shape[1], p, f) for m, p, f in imgs], want_dist=want_dist)
    if schedule is not None:
        plan.set_schedule(*schedule)
    mask = plan.pack([m for m, _, _ in imgs], dev)
    D, F = plan.outputs(dev)
    ws = None
    for rep in range(submits):
        if fresh_buffers and rep > 0:
            D, F = plan.outputs(dev)
            ws = None
        if D is not None:
            D.fill_(-9)
        if F is not None:
            F.fill_(-9)
        ws = plan.submit(mask, D, F, workspace=ws)
        torch.cuda.synchronize()
        for q, (m, pol, wf) in enumerate(imgs):
            Do, Fo = oracle.separable(m, pol)
            if want_dist:
                assert np.array_equal(plan.image(D, q).cpu().numpy(), Do), (rep, q, m.shape, pol)
            if wf:
                assert np.array_equal(plan.image(F, q).cpu().numpy(), Fo), (rep, q, m.shape, pol)
    plan.close()


def test_ragged_batch_matches_oracle_with_graph_replay(edt):
    imgs = _images(1, 40, extra=[(64, 1025, 0.3), (70, 2049, 0.2), (33, 4100, 0.2),
                                 (20, 9000, 0.1), (5, 16384, 0.05), (9, 3000, 0.0005)])
    _check_batch(edt, imgs, submits=3)


def test_ragged_batch_without_graphs(edt, monkeypatch):
    monkeypatch.setenv("EDT_NO_GRAPH", "1")
    _check_batch(edt, _images(2, 25, extra=[(40, 1500, 0.3)]), submits=2)


def test_new_buffers_recapture(edt):
    _check_batch(edt, _images(3, 12), submits=3, fresh_buffers=True)


def test_unpadded_rows_and_offsets(edt, monkeypatch):
    # rows packed with no padding: mask rows and image offsets fall anywhere
    # inside 4-byte words, output rows anywhere inside 16-byte lines
    import paper_2106_03503_amd._lib as lib
    monkeypatch.setattr(lib, "_round_up", lambda v, a: v)
    imgs = _images(6, 30, extra=[(131, 1029, 0.02), (67, 301, 0.3), (3, 5, 0.5)])
    _check_batch(edt, imgs, submits=2)


def test_features_only_batch(edt):
    imgs = [(m, p, True) for m, p, _ in _images(4, 15)]
    _check_batch(edt, imgs, want_dist=False, submits=1)


def test_batch_equals_single_image_calls(edt):
    import torch
    dev = torch.device("cuda:0")
    imgs = [(m, p, True) for m, p in workloads.ragged_batch(24, 64, 400, seed=7)]
    plan = edt.BatchPlan([(m.shape[0], m.shape[1], p, True) for m, p, _ in imgs])
    mask = plan.pack([m for m, _, _ in imgs], dev)
    D, F = plan.outputs(dev)
    plan.submit(mask, D, F)
    for q, (m, pol, _) in enumerate(imgs):
        Ds, Fs = edt.feature(torch.from_numpy(m).to(dev), polarity=pol)
        assert torch.equal(plan.image(D, q), Ds)
        assert torch.equal(plan.image(F, q), Fs)
    plan.close()


def _deep_pop_mask(H, W, seed):
    """Rows whose envelopes grow long and are then mostly popped at once: in
    each row band the site rows drift away slowly from left to right (every
    parabola survives), then a column with a site in the band itself hides
    dozens of them, more than the 16 stack entries a lane keeps in LDS."""
    rng = np.random.default_rng(seed)
    m = np.zeros((H, W), np.uint8)
    for c in range(W):
        if c % 97 == 96:
            m[rng.integers(0, H, 8), c] = 1  # near sites: deep pops
        else:
            m[min(H - 1, (c % 97) // 2), c] = 1  # slowly drifting sites
    return m


def test_lane_rows_deep_pops_and_ties(edt):
    """The one-lane-per-row pass: stacks deeper than its LDS ring, pops that
    reach below it, tie-heavy regular grids, and sizes that leave partial
    row groups and partial 4-pixel stores."""
    rng = np.random.default_rng(11)
    imgs = []
    for k, (H, W) in enumerate([(130, 700), (64, 1000), (65, 333), (200, 257), (7, 4096)]):
        imgs.append((_deep_pop_mask(H, W, k), k % 2, True))
    for k, (H, W, step) in enumerate([(96, 301, 6), (129, 513, 4), (70, 998, 10)]):
        m = np.zeros((H, W), np.uint8)
        m[::step, ::step] = 1  # equidistant sites everywhere: ties
        imgs.append((m, 0, True))
        imgs.append((1 - m, 1, True))
    for (H, W) in [(1, 1), (1, 4096), (4096, 1), (3, 5), (64, 64)]:
        imgs.append(((rng.random((H, W)) < 0.3).astype(np.uint8), 0, True))
    _check_batch(edt, imgs, submits=2)


def test_lane_rows_at_the_packed_height_limit(edt):
    """The one-lane-per-row pass packs a stack entry's site row into 12 bits:
    images 4096 rows tall take it with sites on their last row (row 4095) and
    deep stacks; one row taller goes to the one-workgroup-per-row pass.  Both
    polarities, against the oracle."""
    rng = np.random.default_rng(12)
    imgs = []
    for H in (4096, 4097):
        m = np.zeros((H, 300), np.uint8)
        m[H - 1, ::7] = 1                                   # sites on the last row
        m[rng.integers(0, H, 40), rng.integers(0, 300, 40)] = 1
        m[(np.arange(300) * 13) % H, np.arange(300)] = 1    # a site in every column
        imgs.append((m, 0, True))
        imgs.append((m, 1, True))
    _check_batch(edt, imgs, submits=2)


def test_autotune_keeps_results_and_picks_the_fastest(edt):
    import torch
    dev = torch.device("cuda:0")
    imgs = _images(12, 30, extra=[(70, 700, 0.3), (40, 1500, 0.05), (9, 200, 0.5)])
    plan = edt.BatchPlan([(m.shape[0], m.shape[1], p, f) for m, p, f in imgs])
    mask = plan.pack([m for m, _, _ in imgs], dev)
    D, F = plan.outputs(dev)
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device=dev)
    cands, chosen = plan.autotune(mask, D, F, workspace=ws)
    # every combination of lane width, order, branches, the single path for the
    # 1500-wide image and the transposed order (not without the lane pass)
    assert len(cands) == 40 and 0 <= chosen < len(cands)
    assert {c["lane_w"] for c in cands} >= {0, 256, 1024}
    assert {c["branches"] for c in cands} == {1, 2}
    assert {c["wide_single"] for c in cands} == {False, True}
    assert {c["transpose"] for c in cands} == {False, True}
    assert cands[chosen]["ms"] == min(c["ms"] for c in cands)
    for rep in range(2):  # the tuned schedule, replayed
        D.fill_(-9)
        F.fill_(-9)
        plan.submit(mask, D, F, workspace=ws)
        torch.cuda.synchronize()
        for q, (m, pol, wf) in enumerate(imgs):
            Do, Fo = oracle.separable(m, pol)
            assert np.array_equal(plan.image(D, q).cpu().numpy(), Do), (rep, q)
            if wf:
                assert np.array_equal(plan.image(F, q).cpu().numpy(), Fo), (rep, q)
    for lane_w, lf, br, wsg, tr in ((0, True, 1, False, False), (256, False, 2, False, True),
                                    (1024, True, 2, True, True), (1024, False, 1, True, False)):
        plan.set_schedule(lane_w, lf, br, wsg, tr)  # schedules set by hand
        D.fill_(-9)
        F.fill_(-9)
        plan.submit(mask, D, F, workspace=ws)
        torch.cuda.synchronize()
        for q, (m, pol, wf) in enumerate(imgs):
            Do, Fo = oracle.separable(m, pol)
            assert np.array_equal(plan.image(D, q).cpu().numpy(), Do), (lane_w, q)
            if wf:
                assert np.array_equal(plan.image(F, q).cpu().numpy(), Fo), (lane_w, q)
    with pytest.raises(edt.EDTError):
        plan.set_schedule(2048, False)
    with pytest.raises(edt.EDTError):
        plan.set_schedule(1024, False, branches=3)
    plan.close()


def _wide_images(seed):
    """Images wider than tall (and some taller, left as they are), with tie-heavy
    grids: the transposed order breaks ties by the smaller original row first."""
    rng = np.random.default_rng(seed)
    out = []
    for (H, W) in [(1, 2), (1, 700), (3, 1024), (63, 64), (64, 65), (65, 1000), (100, 3000),
                   (7, 4096), (300, 301), (1024, 1100), (200, 90), (40, 40)]:
        for kind in range(3):
            if kind == 0:
                m = (rng.random((H, W)) < rng.uniform(0.001, 0.2)).astype(np.uint8)
            elif kind == 1:
                m = np.zeros((H, W), np.uint8)
                m[::max(1, H // 5), ::3] = 1  # a grid: many equidistant sites
            else:
                m = workloads.ellipses(H, W, 6, 2, 40, rng=rng)
            out.append((m, int(rng.integers(0, 2)), bool(rng.integers(0, 2)) or kind == 1))
    return out


@pytest.mark.parametrize("lane_w,branches", [(1024, 1), (256, 2)])
def test_transposed_order_matches_oracle(edt, lane_w, branches):
    # images wider than tall run as their transposes (Section 3.2.1), with
    # graph replays; features are original indices with the smallest-index rule
    _check_batch(edt, _wide_images(2106401), submits=2,
                 schedule=(lane_w, True, branches, False, True))


def test_transposed_order_features_only(edt):
    imgs = [(m, pol, True) for m, pol, _ in _wide_images(2106402)[:18]]
    _check_batch(edt, imgs, want_dist=False, submits=1, schedule=(1024, False, 1, False, True))


def test_plan_reserves_the_lane_envelopes(edt):
    """The one-lane-per-row pass keeps each row's envelope in the image's
    workspace (4 bytes per row per 32-rounded column): a plan reserves that
    beside the single-image workspace for every image the pass can take, and
    for the transposed sides of an image that may run as its transpose."""
    def cp(w):
        return (w + 31) // 32 * 32

    for H, W in [(1, 1), (33, 70), (300, 1000), (4096, 1024), (700, 64)]:
        ws = edt.BatchPlan([(H, W, 0, True)]).workspace_bytes
        assert ws >= edt.workspace_bytes(H, W) + 4 * H * cp(W), (H, W)
    # wider than tall, at most 1024 tall and 4096 wide: may run transposed
    H, W = 200, 3000
    ws = edt.BatchPlan([(H, W, 1, True)]).workspace_bytes
    assert ws >= edt.workspace_bytes(W, H) + 4 * W * cp(H)
