"""edt_feature_noalloc (the static per-device workspace) against edt_feature
(a caller workspace), through the C ABI: two calls in a row, the second on a
smaller image, so the second runs over what the first left in the array."""
import numpy as np
import pytest

import workloads

SCRATCH = 128 << 20


def _run_both(edt, lib, m, pol, metric=0):
    import torch
    dev = torch.device("cuda:0")
    H, W = m.shape
    mask = torch.from_numpy(m).to(dev)
    stream = torch.cuda.current_stream().cuda_stream
    D0 = torch.full((H, W), -5, dtype=torch.int32, device=dev)
    F0 = torch.full((H, W), -5, dtype=torch.int32, device=dev)
    ws = torch.empty(edt.workspace_bytes(H, W), dtype=torch.uint8, device=dev)
    assert ws.numel() <= SCRATCH
    assert lib.edt_feature(mask.data_ptr(), H, W, W, pol, metric, D0.data_ptr(), F0.data_ptr(),
                           W, ws.data_ptr(), ws.numel(), stream) == 0
    D1 = torch.full((H, W), -7, dtype=torch.int32, device=dev)
    F1 = torch.full((H, W), -7, dtype=torch.int32, device=dev)
    print(f"noalloc: {H}x{W} polarity {pol} metric {metric}", flush=True)
    assert lib.edt_feature_noalloc(mask.data_ptr(), H, W, W, pol, metric, D1.data_ptr(),
                                   F1.data_ptr(), W, stream) == 0
    torch.cuda.synchronize()
    return D0.cpu().numpy(), F0.cpu().numpy(), D1.cpu().numpy(), F1.cpu().numpy()


@pytest.mark.gpu
def test_noalloc_equals_workspace_entry_point_on_two_calls():
    import oracle
    import paper_2106_03503_amd as edt
    from paper_2106_03503_amd import _lib
    lib = _lib.lib
    # a large image first (dense rows: the segment scan and its sizes in the
    # workspace), then a smaller one over what it left behind
    cases = [(workloads.disks(2048, 3000, n_disks=60, seed=11), 0),
             (workloads.bernoulli(300, 517, 0.03, seed=12), 1)]
    for m, pol in cases:
        D0, F0, D1, F1 = _run_both(edt, lib, m, pol)
        np.testing.assert_array_equal(D1, D0)
        np.testing.assert_array_equal(F1, F0)
    # the smaller image also against the oracle
    Do, Fo = oracle.separable(*cases[1])
    np.testing.assert_array_equal(D1, Do)
    np.testing.assert_array_equal(F1, Fo)


@pytest.mark.gpu
def test_noalloc_features_only_and_the_size_limit():
    import torch
    import paper_2106_03503_amd as edt
    from paper_2106_03503_amd import _lib
    m = workloads.bernoulli(129, 70, 0.05, seed=13)
    dev = torch.device("cuda:0")
    mask = torch.from_numpy(m).to(dev)
    F = torch.empty((129, 70), dtype=torch.int32, device=dev)
    edt.feature_noalloc(mask, None, F, polarity=0)
    _, F0 = edt.feature(mask, polarity=0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(F.cpu().numpy(), F0.cpu().numpy())
    # an image whose workspace exceeds the static array is refused before any launch
    big = 8192
    assert edt.workspace_bytes(big, big) > SCRATCH
    st = _lib.lib.edt_feature_noalloc(mask.data_ptr(), big, big, big, 0, 0, F.data_ptr(),
                                      F.data_ptr(), big, None)
    assert st == -3
