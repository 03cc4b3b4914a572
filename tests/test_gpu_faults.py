"""Error paths under a launch failure forced from the host
(edt_debug_fail_launch): the call whose launch fails reports EDT_ERR_DEVICE,
later launches of that call are not enqueued, and the calls, batch
submissions and served requests that follow are unaffected.  No kernel runs
with bad arguments and nothing faults on the device."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

EDT_ERR_DEVICE = -7


@pytest.fixture(scope="module")
def edt():
    import torch
    import paper_2106_03503_amd as edt
    assert torch.cuda.is_available()
    yield edt
    edt._lib.lib.edt_debug_fail_launch(0)


def _arm(edt, k):
    assert edt._lib.lib.edt_debug_fail_launch(k) == 0


def test_arming_checks_its_argument(edt):
    assert edt._lib.lib.edt_debug_fail_launch(-1) == -1
    _arm(edt, 0)


@pytest.mark.parametrize("k", [1, 2, 4, 5, 6, 7, 8])
def test_single_call_fails_at_any_launch_then_recovers(edt, k):
    # a dense image takes eight launches: band bits, carries, column list,
    # nearest rows, the sparse form (exits), segment scan, bounded search, merge
    import torch
    dev = torch.device("cuda:0")
    m = workloads.bernoulli(300, 2000, 0.05, seed=k)
    mask = torch.from_numpy(m).to(dev)
    D = torch.empty((300, 2000), dtype=torch.int32, device=dev)
    F = torch.empty_like(D)
    ws = torch.empty(edt.workspace_bytes(300, 2000), dtype=torch.uint8, device=dev)
    print(f"faults: single call, launch {k}", flush=True)
    _arm(edt, k)
    with pytest.raises(edt.EDTError) as e:
        edt.feature(mask, out_dist=D, out_feat=F, workspace=ws)
    assert e.value.status == EDT_ERR_DEVICE
    torch.cuda.synchronize()
    edt.feature(mask, out_dist=D, out_feat=F, workspace=ws)  # nothing armed now
    torch.cuda.synchronize()
    Do, Fo = oracle.separable(m, 0)
    assert np.array_equal(D.cpu().numpy(), Do) and np.array_equal(F.cpu().numpy(), Fo)


def test_batch_capture_failure_then_recapture(edt):
    import torch
    dev = torch.device("cuda:0")
    imgs = [(workloads.bernoulli(70 + 9 * q, 90 + 31 * q, 0.03, seed=q), q % 2) for q in range(12)]
    plan = edt.BatchPlan([(m.shape[0], m.shape[1], p, True) for m, p in imgs])
    mask = plan.pack([m for m, _ in imgs], dev)
    D, F = plan.outputs(dev)
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device=dev)
    for branches in (1, 2):
        plan.set_schedule(1024, True, branches)
        print(f"faults: batch, {branches} branch(es)", flush=True)
        _arm(edt, 3)  # fails while the graph is captured
        with pytest.raises(edt.EDTError) as e:
            plan.submit(mask, D, F, workspace=ws)
        assert e.value.status == EDT_ERR_DEVICE
        torch.cuda.synchronize()
        for rep in range(2):  # captured again, then replayed
            D.fill_(-9)
            F.fill_(-9)
            plan.submit(mask, D, F, workspace=ws)
            torch.cuda.synchronize()
            for q, (m, pol) in enumerate(imgs):
                Do, Fo = oracle.separable(m, pol)
                assert np.array_equal(plan.image(D, q).cpu().numpy(), Do), (branches, rep, q)
                assert np.array_equal(plan.image(F, q).cpu().numpy(), Fo), (branches, rep, q)
    plan.close()


def test_served_request_failure_is_its_own(edt):
    import torch
    dev = torch.device("cuda:0")
    a = torch.from_numpy(workloads.bernoulli(200, 300, 0.02, seed=1)).to(dev)
    b = torch.from_numpy(workloads.bernoulli(150, 170, 0.02, seed=2)).to(dev)
    torch.cuda.synchronize()
    srv = edt.Server(64 << 20, n_streams=2)
    print("faults: served request", flush=True)
    _arm(edt, 1)  # the scheduler's first launch
    t1 = srv.submit(a, want_feature=True)
    with pytest.raises(edt.EDTError) as e:
        srv.wait(t1, timeout=60)
    assert e.value.status == EDT_ERR_DEVICE
    t2 = srv.submit(b, want_feature=True)
    D2, F2 = srv.wait(t2, timeout=60)
    Da, Fa = edt.feature(b)
    torch.cuda.synchronize()
    assert torch.equal(D2, Da) and torch.equal(F2, Fa)
    st = srv.stats()
    assert st["failed"] == 1 and st["done"] == 2
    with pytest.raises(edt.EDTError) as e:  # destroy reports the failed request
        srv.close()
    assert e.value.status == EDT_ERR_DEVICE
