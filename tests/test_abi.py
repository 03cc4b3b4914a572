"""The C ABI on the CPU: the library loads, exports every entry point that
include/edt.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "edt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(edt_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def edt():
    import paper_2106_03503_amd as edt
    return edt


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("edt_sq", "edt_feature", "edt_sqrt_f32", "edt_workspace_bytes",
                 "edt_status_string", "edt_abi_version"):
        assert must in names


def test_library_exports_every_declared_symbol(edt):
    lib = ctypes.CDLL(edt.library_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_abi_version_and_status_strings(edt):
    from paper_2106_03503_amd import _lib
    assert edt.abi_version() == 2
    for code, text in ((0, "ok"), (-1, "invalid argument"), (-2, "unsupported metric"),
                       (-3, "image too large"), (-7, "device error")):
        assert _lib.status_string(code) == text
    assert _lib.status_string(12345) == "unknown status"


def test_workspace_bytes(edt):
    assert edt.workspace_bytes(0, 10) == 0
    assert edt.workspace_bytes(10, 0) == 0
    assert edt.workspace_bytes(32768, 10) == 0
    assert edt.workspace_bytes(10, 32768) == 0
    a = edt.workspace_bytes(100, 100)
    b = edt.workspace_bytes(200, 100)
    assert 0 < a < b
    # at least the int16 intermediate of 2 bytes per pixel
    assert edt.workspace_bytes(16384, 16384) >= 2 * 16384 * 16384


def test_argument_validation_returns_before_any_launch(edt):
    from paper_2106_03503_amd import _lib
    lib = _lib.lib
    fake = 0x1000  # never dereferenced: every call below fails validation
    ws = edt.workspace_bytes(10, 10)
    # sizes
    assert lib.edt_sq(fake, 0, 10, 10, 0, 0, fake, 10, fake, ws, None) == -3
    assert lib.edt_sq(fake, 10, 40000, 40000, 0, 0, fake, 40000, fake, ws, None) == -3
    # null pointers and pitches
    assert lib.edt_sq(None, 10, 10, 10, 0, 0, fake, 10, fake, ws, None) == -1
    assert lib.edt_sq(fake, 10, 10, 10, 0, 0, None, 10, fake, ws, None) == -1
    assert lib.edt_sq(fake, 10, 10, 9, 0, 0, fake, 10, fake, ws, None) == -1
    assert lib.edt_sq(fake, 10, 10, 10, 0, 0, fake, 9, fake, ws, None) == -1
    assert lib.edt_feature(fake, 10, 10, 10, 0, 0, fake, None, 10, fake, ws, None) == -1
    # enums
    assert lib.edt_sq(fake, 10, 10, 10, 2, 0, fake, 10, fake, ws, None) == -1
    assert lib.edt_sq(fake, 10, 10, 10, 0, 4, fake, 10, fake, ws, None) == -1  # past chamfer 4-3
    assert lib.edt_sq(fake, 10, 10, 10, 0, -1, fake, 10, fake, ws, None) == -1
    assert lib.edt_sq(fake, 10, 10, 10, 0, 9, fake, 10, fake, ws, None) == -1
    # workspace: short, missing, misaligned
    assert lib.edt_sq(fake, 10, 10, 10, 0, 0, fake, 10, fake, ws - 1, None) == -1
    assert lib.edt_sq(fake, 10, 10, 10, 0, 0, fake, 10, None, ws, None) == -1
    assert lib.edt_sq(fake, 10, 10, 10, 0, 0, fake, 10, fake + 8, ws, None) == -1
    # fp32 distances: a distance output is required; sizes, pitches and the
    # workspace as for edt_sq
    assert lib.edt_dist_f32(fake, 10, 10, 10, 0, None, fake, 10, fake, ws, None) == -1
    assert lib.edt_dist_f32(fake, 0, 10, 10, 0, fake, None, 10, fake, ws, None) == -3
    assert lib.edt_dist_f32(fake, 10, 10, 10, 0, fake, None, 9, fake, ws, None) == -1
    assert lib.edt_dist_f32(fake, 10, 10, 10, 2, fake, None, 10, fake, ws, None) == -1
    assert lib.edt_dist_f32(fake, 10, 10, 10, 0, fake, None, 10, fake, ws - 1, None) == -1
    # region labels: sizes, pointers, pitches, enums, overlap of labels with the inputs
    big = 0x10000000
    assert lib.edt_regions(fake, 0, 10, 10, 0, 8, fake, big, 10, None) == -3
    assert lib.edt_regions(fake, 10, 40000, 40000, 0, 8, fake, big, 40000, None) == -3
    assert lib.edt_regions(fake, 30000, 30000, 30000, 0, 8, fake, big, 80000, None) == -3
    assert lib.edt_regions(None, 10, 10, 10, 0, 8, fake, big, 10, None) == -1
    assert lib.edt_regions(fake, 10, 10, 10, 0, 8, None, big, 10, None) == -1
    assert lib.edt_regions(fake, 10, 10, 10, 0, 8, fake, None, 10, None) == -1
    assert lib.edt_regions(fake, 10, 10, 9, 0, 8, fake, big, 10, None) == -1
    assert lib.edt_regions(fake, 10, 10, 10, 0, 8, fake, big, 9, None) == -1
    assert lib.edt_regions(fake, 10, 10, 10, 2, 8, fake, big, 10, None) == -1
    assert lib.edt_regions(fake, 10, 10, 10, 0, 6, fake, big, 10, None) == -1
    assert lib.edt_regions(fake, 10, 10, 10, 0, 8, big + 40, big, 10, None) == -1  # labels over feature
    assert lib.edt_regions(big + 4, 10, 10, 10, 0, 8, fake, big, 10, None) == -1   # labels over mask
    # Danielsson: sizes, pointers, pitches, polarity, dist over rel
    assert lib.edt_danielsson(fake, 10, 8193, 8193, 0, big, big + 400000, 8193, None) == -3
    assert lib.edt_danielsson(fake, 0, 10, 10, 0, big, big + 4000, 10, None) == -3
    assert lib.edt_danielsson(None, 10, 10, 10, 0, big, big + 4000, 10, None) == -1
    assert lib.edt_danielsson(fake, 10, 10, 10, 0, None, big + 4000, 10, None) == -1
    assert lib.edt_danielsson(fake, 10, 10, 10, 0, big, None, 10, None) == -1
    assert lib.edt_danielsson(fake, 10, 10, 9, 0, big, big + 4000, 10, None) == -1
    assert lib.edt_danielsson(fake, 10, 10, 10, 3, big, big + 4000, 10, None) == -1
    assert lib.edt_danielsson(fake, 10, 10, 10, 0, big, big + 40, 10, None) == -1  # overlap
    # the static-workspace variant: the size limit, then edt_feature's checks
    assert lib.edt_feature_noalloc(fake, 8192, 8192, 8192, 0, 0, fake, fake, 8192, None) == -3
    assert lib.edt_feature_noalloc(fake, 0, 10, 10, 0, 0, fake, fake, 10, None) == -3
    assert lib.edt_feature_noalloc(fake, 10, 10, 10, 0, 0, fake, None, 10, None) == -1
    assert lib.edt_feature_noalloc(None, 10, 10, 10, 0, 0, fake, fake, 10, None) == -1
    assert lib.edt_feature_noalloc(fake, 10, 10, 9, 0, 0, fake, fake, 10, None) == -1
    assert lib.edt_feature_noalloc(fake, 10, 10, 10, 3, 0, fake, fake, 10, None) == -1
    assert lib.edt_feature_noalloc(fake, 10, 10, 10, 0, 4, fake, fake, 10, None) == -1
    # sqrt
    assert lib.edt_sqrt_f32(fake, fake, -1, None) == -1
    assert lib.edt_sqrt_f32(None, fake, 5, None) == -1
    assert lib.edt_sqrt_f32(None, None, 0, None) == 0  # empty: nothing to do


def test_python_binding_rejects_cpu_tensors(edt):
    import torch
    with pytest.raises(ValueError):
        edt.sq(torch.zeros((4, 4), dtype=torch.uint8))
    with pytest.raises(ValueError):
        edt.feature(torch.zeros((4, 4, 4), dtype=torch.uint8))


def test_batch_plan_validation_before_any_device_call(edt):
    import ctypes
    from paper_2106_03503_amd import _lib
    D = _lib.ImageDesc

    def plan(descs, n=None, want_dist=1):
        arr = (D * max(1, len(descs)))(*descs)
        p = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        return _lib.lib.edt_batch_plan(ctypes.cast(arr, ctypes.c_void_p),
                                       len(descs) if n is None else n, want_dist,
                                       ctypes.byref(p), ctypes.byref(ws))

    ok = D(0, 16, 0, 16, 8, 16, 0, 1)
    assert plan([ok], n=0) == -1
    assert plan([D(0, 16, 0, 16, 0, 16, 0, 1)]) == -3          # H = 0
    assert plan([D(0, 20000, 0, 20000, 4, 20000, 0, 1)]) == -3  # wider than a batch allows
    assert plan([D(0, 8, 0, 16, 8, 16, 0, 1)]) == -1           # mask pitch < W
    assert plan([D(0, 16, 0, 8, 8, 16, 0, 1)]) == -1           # out pitch < W
    assert plan([D(0, 16, 0, 16, 8, 16, 5, 1)]) == -1          # polarity
    assert plan([D(-16, 16, 0, 16, 8, 16, 0, 1)]) == -1        # negative offset
    # an image that writes neither distances nor features is refused (with
    # want_dist = 0 every image must want its features)
    assert plan([D(0, 16, 0, 16, 8, 16, 0, 0)], want_dist=0) == -1
    assert plan([D(0, 16, 0, 16, 8, 16, 0, 1), D(256, 16, 256, 16, 8, 16, 1, 0)],
                want_dist=0) == -1
    assert _lib.lib.edt_plan_destroy(None) == -1


def test_serve_validation_before_any_device_call(edt):
    import ctypes
    from paper_2106_03503_amd import _lib
    lib = _lib.lib
    C = _lib.ServeConfig
    fake = 0x100000  # 256-byte aligned, never dereferenced
    srv = ctypes.c_void_p()

    def create(cfg, arena=fake, nbytes=1 << 30):
        return lib.edt_serve_create(ctypes.byref(cfg) if cfg is not None else None, arena,
                                    nbytes, ctypes.byref(srv))

    assert create(None) == -1
    assert create(C(0, 0, 1, 0)) == -1                  # max_inflight
    assert create(C(0, 8, 0, 0)) == -1                  # n_streams
    assert create(C(0, 8, 17, 0)) == -1                 # n_streams above the limit
    assert create(C(0, 8, 1, 1025)) == -1               # max_group above the limit
    assert create(C(0, 8, 1, 0), arena=fake + 64) == -1  # misaligned arena
    assert create(C(0, 8, 1, 0), arena=None) == -1
    assert create(C(2 << 30, 8, 1, 0)) == -1            # budget above the arena
    assert create(C(4096, 8, 1, 0)) == -1               # budget below the launch tables
    assert srv.value is None
    # reserved bytes: 2 * n_streams tables
    r1 = _lib.Server.reserved_bytes(1, 16)
    assert r1 > 0 and r1 % 256 == 0
    assert _lib.Server.reserved_bytes(2, 16) == 2 * r1
    assert _lib.Server.reserved_bytes(1, 1024) > r1
    assert _lib.Server.reserved_bytes(0, 16) == 0
    # null server handles
    t = ctypes.c_uint64()
    done = ctypes.c_int32()
    assert lib.edt_serve_submit(None, None, ctypes.byref(t)) == -1
    assert lib.edt_serve_poll(None, 1, ctypes.byref(done)) == -1
    assert lib.edt_serve_wait(None, 1, 0) == -1
    assert lib.edt_serve_stats(None, None) == -1
    assert lib.edt_serve_destroy(None) == -1
