"""ctypes marshalling for libedt.so (argument checks and pointers only)."""
from __future__ import annotations

import ctypes
import os

# torch first: its HIP runtime must be the one libedt.so binds to, so that the
# streams and device pointers torch hands over are valid in the library.
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libedt.so")

EDT_OK = 0
EDT_TO_OBJECT = 0
EDT_TO_BACKGROUND = 1
EDT_METRIC_EUCLIDEAN_SQ = 0
EDT_METRIC_CITYBLOCK = 1
EDT_METRIC_CHESSBOARD = 2
EDT_METRIC_CHAMFER34 = 3
EDT_INF_SQ = 2**31 - 1
EDT_NO_SITE = -1


class EDTError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


def library_path() -> str:
    return _LIB_PATH


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"{_LIB_PATH} is not built; run __graft_entry__.build() "
            "(or python paper_2106_03503_amd/build.py)")
    lib = ctypes.CDLL(_LIB_PATH)
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.edt_abi_version.argtypes = []
    lib.edt_abi_version.restype = i32
    lib.edt_status_string.argtypes = [i32]
    lib.edt_status_string.restype = ctypes.c_char_p
    lib.edt_workspace_bytes.argtypes = [i32, i32, i32]
    lib.edt_workspace_bytes.restype = sz
    lib.edt_sq.argtypes = [P, i32, i32, i64, i32, i32, P, i64, P, sz, P]
    lib.edt_sq.restype = i32
    lib.edt_feature.argtypes = [P, i32, i32, i64, i32, i32, P, P, i64, P, sz, P]
    lib.edt_feature.restype = i32
    lib.edt_feature_noalloc.argtypes = [P, i32, i32, i64, i32, i32, P, P, i64, P]
    lib.edt_feature_noalloc.restype = i32
    lib.edt_sqrt_f32.argtypes = [P, P, i64, P]
    lib.edt_sqrt_f32.restype = i32
    lib.edt_dist_f32.argtypes = [P, i32, i32, i64, i32, P, P, i64, P, sz, P]
    lib.edt_dist_f32.restype = i32
    lib.edt_regions.argtypes = [P, i32, i32, i64, i32, i32, P, P, i64, P]
    lib.edt_regions.restype = i32
    lib.edt_danielsson.argtypes = [P, i32, i32, i64, i32, P, P, i64, P]
    lib.edt_danielsson.restype = i32
    lib.edt_debug_fail_launch.argtypes = [i32]
    lib.edt_debug_fail_launch.restype = i32
    lib.edt_profile_begin.argtypes = []
    lib.edt_profile_begin.restype = i32
    lib.edt_profile_end.argtypes = [P, i32, P]
    lib.edt_profile_end.restype = i32
    return lib


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


_lib = _load()
lib = _lib  # exported for tests of the raw ABI


def abi_version() -> int:
    return _lib.edt_abi_version()


def status_string(status: int) -> str:
    return _lib.edt_status_string(status).decode()


def workspace_bytes(H: int, W: int, want_feature: bool = True) -> int:
    return int(_lib.edt_workspace_bytes(H, W, int(want_feature)))


def _check(status: int, what: str) -> None:
    if status != EDT_OK:
        raise EDTError(status, what)


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _check_mask(mask: torch.Tensor):
    if not isinstance(mask, torch.Tensor) or mask.dim() != 2:
        raise ValueError("mask must be a 2-D torch tensor")
    if mask.dtype not in (torch.uint8, torch.bool):
        raise ValueError("mask must be uint8 (0 = background, nonzero = object)")
    if not mask.is_cuda:
        raise ValueError("mask must be on a GPU device")
    if mask.dtype == torch.bool:
        mask = mask.view(torch.uint8)
    if mask.stride(1) != 1:
        mask = mask.contiguous()
    return mask


def _check_out(t, H, W, device, name):
    if t is None:
        return torch.empty((H, W), dtype=torch.int32, device=device)
    if t.dtype != torch.int32 or t.shape != (H, W) or t.device != device or t.stride(1) != 1:
        raise ValueError(f"{name} must be an int32 {H}x{W} tensor on {device} with unit column stride")
    return t


def _workspace(H, W, want_feature, device, workspace):
    need = workspace_bytes(H, W, want_feature)
    if need == 0:
        raise EDTError(-3, "workspace")
    if workspace is None:
        return torch.empty(need, dtype=torch.uint8, device=device)
    if workspace.numel() * workspace.element_size() < need or workspace.device != device:
        raise ValueError(f"workspace needs {need} bytes on {device}")
    return workspace


def sq(mask: torch.Tensor, polarity: int = EDT_TO_OBJECT, metric: int = EDT_METRIC_EUCLIDEAN_SQ,
       out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
       stream=None) -> torch.Tensor:
    """Distance of every pixel to the nearest site (int32): squared Euclidean
    (metric 0), city-block (1), chessboard (2) or chamfer 4-3 (3: three times
    the approximate distance)."""
    mask = _check_mask(mask)
    H, W = mask.shape
    out = _check_out(out, H, W, mask.device, "out")
    if out.stride(0) < W:
        raise ValueError("out row pitch must be >= W")
    ws = _workspace(H, W, False, mask.device, workspace)
    _check(_lib.edt_sq(mask.data_ptr(), H, W, mask.stride(0), polarity, metric,
                       out.data_ptr(), out.stride(0), ws.data_ptr(),
                       ws.numel() * ws.element_size(), _stream_ptr(stream)), "edt_sq")
    return out


def feature(mask: torch.Tensor, polarity: int = EDT_TO_OBJECT,
            metric: int = EDT_METRIC_EUCLIDEAN_SQ, want_dist: bool = True,
            out_dist: torch.Tensor | None = None, out_feat: torch.Tensor | None = None,
            workspace: torch.Tensor | None = None, stream=None):
    """(squared distance, nearest-site linear index r*W + c); the distance is
    None when want_dist is False."""
    mask = _check_mask(mask)
    H, W = mask.shape
    F = _check_out(out_feat, H, W, mask.device, "out_feat")
    D = _check_out(out_dist, H, W, mask.device, "out_dist") if want_dist else None
    if D is not None and D.stride(0) != F.stride(0):
        raise ValueError("out_dist and out_feat must share one row pitch")
    ws = _workspace(H, W, True, mask.device, workspace)
    _check(_lib.edt_feature(mask.data_ptr(), H, W, mask.stride(0), polarity, metric,
                            D.data_ptr() if D is not None else None, F.data_ptr(),
                            F.stride(0), ws.data_ptr(), ws.numel() * ws.element_size(),
                            _stream_ptr(stream)), "edt_feature")
    return D, F


def feature_noalloc(mask: torch.Tensor, out_dist: torch.Tensor | None, out_feat: torch.Tensor,
                    polarity: int = EDT_TO_OBJECT, metric: int = EDT_METRIC_EUCLIDEAN_SQ,
                    stream=None):
    """edt.feature into caller-given outputs, with the library's static
    per-device workspace instead of a workspace tensor (nothing is allocated;
    calls that overlap on one device race).  out_dist may be None."""
    mask = _check_mask(mask)
    H, W = mask.shape
    F = _check_out(out_feat, H, W, mask.device, "out_feat")
    D = _check_out(out_dist, H, W, mask.device, "out_dist") if out_dist is not None else None
    if D is not None and D.stride(0) != F.stride(0):
        raise ValueError("out_dist and out_feat must share one row pitch")
    _check(_lib.edt_feature_noalloc(mask.data_ptr(), H, W, mask.stride(0), polarity, metric,
                                    D.data_ptr() if D is not None else None, F.data_ptr(),
                                    F.stride(0), _stream_ptr(stream)), "edt_feature_noalloc")
    return D, F


def sqrt_f32(dist_sq: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """float32 sqrt of int32 squared distances (EDT_INF_SQ -> +inf)."""
    if dist_sq.dtype != torch.int32 or not dist_sq.is_cuda or not dist_sq.is_contiguous():
        raise ValueError("dist_sq must be a contiguous int32 GPU tensor")
    if out is None:
        out = torch.empty(dist_sq.shape, dtype=torch.float32, device=dist_sq.device)
    elif out.dtype != torch.float32 or out.shape != dist_sq.shape or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor of the same shape")
    _check(_lib.edt_sqrt_f32(dist_sq.data_ptr(), out.data_ptr(), dist_sq.numel(),
                             _stream_ptr(stream)), "edt_sqrt_f32")
    return out


def dist_f32(mask: torch.Tensor, polarity: int = EDT_TO_OBJECT, want_feature: bool = False,
             out_dist: torch.Tensor | None = None, out_feat: torch.Tensor | None = None,
             workspace: torch.Tensor | None = None, stream=None):
    """(float32 Euclidean distance, nearest-site index or None), the distance
    written by the row pass itself: equal to sqrt_f32 of edt.sq's result."""
    mask = _check_mask(mask)
    H, W = mask.shape
    if out_dist is None:
        D = torch.empty((H, W), dtype=torch.float32, device=mask.device)
    elif (out_dist.dtype != torch.float32 or out_dist.shape != (H, W)
          or out_dist.device != mask.device or out_dist.stride(1) != 1):
        raise ValueError(f"out_dist must be a float32 {H}x{W} tensor on {mask.device} "
                         "with unit column stride")
    else:
        D = out_dist
    F = _check_out(out_feat, H, W, mask.device, "out_feat") if want_feature else None
    if F is not None and D.stride(0) != F.stride(0):
        raise ValueError("out_dist and out_feat must share one row pitch")
    ws = _workspace(H, W, want_feature, mask.device, workspace)
    _check(_lib.edt_dist_f32(mask.data_ptr(), H, W, mask.stride(0), polarity, D.data_ptr(),
                             F.data_ptr() if F is not None else None, D.stride(0),
                             ws.data_ptr(), ws.numel() * ws.element_size(),
                             _stream_ptr(stream)), "edt_dist_f32")
    return D, F


def regions(mask: torch.Tensor, feature: torch.Tensor, polarity: int = EDT_TO_OBJECT,
            connectivity: int = 8, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Voronoi region of every pixel (int32): the smallest linear index of the
    connected component (4- or 8-neighbourhood) of sites that holds its
    nearest site; ``feature`` is edt.feature's output for the same mask and
    polarity."""
    mask = _check_mask(mask)
    H, W = mask.shape
    if feature.dtype != torch.int32 or feature.shape != (H, W) or feature.stride(1) != 1 \
            or feature.device != mask.device:
        raise ValueError(f"feature must be an int32 {H}x{W} tensor on {mask.device}")
    if out is None:
        out = torch.empty_strided((H, W), (feature.stride(0), 1), dtype=torch.int32,
                                  device=mask.device)
    else:
        out = _check_out(out, H, W, mask.device, "out")
        if out.stride(0) != feature.stride(0):
            raise ValueError("out and feature must share one row pitch")
    _check(_lib.edt_regions(mask.data_ptr(), H, W, mask.stride(0), polarity, connectivity,
                            feature.data_ptr(), out.data_ptr(), feature.stride(0),
                            _stream_ptr(stream)), "edt_regions")
    return out


def danielsson(mask: torch.Tensor, polarity: int = EDT_TO_OBJECT,
               out_dist: torch.Tensor | None = None, out_rel: torch.Tensor | None = None,
               stream=None):
    """Danielsson's approximate transform (comparison only): (dist_sq, rel)
    with rel = (dy << 16) | dx the propagated relative position."""
    mask = _check_mask(mask)
    H, W = mask.shape
    D = _check_out(out_dist, H, W, mask.device, "out_dist")
    R = _check_out(out_rel, H, W, mask.device, "out_rel")
    if D.stride(0) != R.stride(0):
        raise ValueError("out_dist and out_rel must share one row pitch")
    _check(_lib.edt_danielsson(mask.data_ptr(), H, W, mask.stride(0), polarity, D.data_ptr(),
                               R.data_ptr(), D.stride(0), _stream_ptr(stream)), "edt_danielsson")
    return D, R


def profile_begin() -> None:
    """Start per-kernel event timing inside the library."""
    _check(_lib.edt_profile_begin(), "edt_profile_begin")


def profile_end() -> dict:
    """Stop timing; {kernel name: (launches, total milliseconds)}."""
    cap = 64
    arr = (KernelTime * cap)()
    n = ctypes.c_int32(0)
    _check(_lib.edt_profile_end(ctypes.cast(arr, ctypes.c_void_p), cap,
                                ctypes.cast(ctypes.pointer(n), ctypes.c_void_p)),
           "edt_profile_end")
    return {arr[q].name.decode(): (int(arr[q].launches), float(arr[q].total_ms))
            for q in range(min(n.value, cap))}


# ---------------------------------------------------------------- batches

class ImageDesc(ctypes.Structure):
    _fields_ = [("mask_offset", ctypes.c_int64), ("mask_pitch", ctypes.c_int64),
                ("out_offset", ctypes.c_int64), ("out_pitch", ctypes.c_int64),
                ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("polarity", ctypes.c_int32), ("want_feature", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("lane_w", ctypes.c_int32), ("largest_first", ctypes.c_int32),
                ("branches", ctypes.c_int32), ("wide_single", ctypes.c_int32),
                ("transpose", ctypes.c_int32)]


EDT_TUNE_MAX = 48


class TuneReport(ctypes.Structure):
    _fields_ = [("tried", ctypes.c_int32), ("chosen", ctypes.c_int32),
                ("cand", Schedule * EDT_TUNE_MAX), ("ms", ctypes.c_float * EDT_TUNE_MAX)]


def _bind_batch():
    P, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    _lib.edt_batch_autotune.argtypes = [P, P, P, P, P, sz, P, P]
    _lib.edt_batch_autotune.restype = i32
    _lib.edt_batch_set_schedule.argtypes = [P, P]
    _lib.edt_batch_set_schedule.restype = i32
    _lib.edt_batch_plan.argtypes = [P, i32, i32, P, P]
    _lib.edt_batch_plan.restype = i32
    _lib.edt_batch_submit.argtypes = [P, P, P, P, P, sz, P]
    _lib.edt_batch_submit.restype = i32
    _lib.edt_plan_destroy.argtypes = [P]
    _lib.edt_plan_destroy.restype = i32


_bind_batch()


def _round_up(v: int, a: int) -> int:
    return (v + a - 1) // a * a


class BatchPlan:
    """A batch of images of uneven size laid out back to back in one mask
    buffer (rows padded to 16 bytes) and one buffer per output (rows padded to
    4 elements).  ``images`` is a list of (H, W, polarity, want_feature)."""

    def __init__(self, images, want_dist: bool = True):
        self.images = [(int(h), int(w), int(p), bool(f)) for h, w, p, f in images]
        n = len(self.images)
        descs = (ImageDesc * max(n, 1))()
        moff = ooff = 0
        self.mask_off, self.out_off, self.mask_pitch, self.out_pitch = [], [], [], []
        for q, (h, w, p, f) in enumerate(self.images):
            mp, op = _round_up(w, 16), _round_up(w, 4)
            descs[q] = ImageDesc(moff, mp, ooff, op, h, w, p, int(f))
            self.mask_off.append(moff)
            self.out_off.append(ooff)
            self.mask_pitch.append(mp)
            self.out_pitch.append(op)
            moff += h * mp
            ooff += h * op
        self.mask_bytes, self.out_elems = moff, ooff
        self.want_dist = bool(want_dist)
        self.any_feat = any(f for _, _, _, f in self.images)
        self._plan = ctypes.c_void_p()
        ws = ctypes.c_size_t(0)
        _check(_lib.edt_batch_plan(ctypes.cast(descs, ctypes.c_void_p), n, int(want_dist),
                                   ctypes.byref(self._plan), ctypes.byref(ws)), "edt_batch_plan")
        self.workspace_bytes = int(ws.value)

    def pack(self, masks, device) -> torch.Tensor:
        """Copy a list of 2-D uint8 numpy masks into one device buffer."""
        import numpy as np
        flat = np.zeros(self.mask_bytes, np.uint8)
        for q, m in enumerate(masks):
            h, w = self.images[q][:2]
            if m.shape != (h, w):
                raise ValueError(f"mask {q} has shape {m.shape}, planned {(h, w)}")
            view = flat[self.mask_off[q]:self.mask_off[q] + h * self.mask_pitch[q]]
            view.reshape(h, self.mask_pitch[q])[:, :w] = m
        return torch.from_numpy(flat).to(device)

    def outputs(self, device):
        d = torch.empty(self.out_elems, dtype=torch.int32, device=device) if self.want_dist else None
        f = torch.empty(self.out_elems, dtype=torch.int32, device=device) if self.any_feat else None
        return d, f

    def image(self, flat: torch.Tensor, q: int) -> torch.Tensor:
        """(H, W) view of image q inside a flat output buffer."""
        h, w = self.images[q][:2]
        o, p = self.out_off[q], self.out_pitch[q]
        return flat[o:o + h * p].view(h, p)[:, :w]

    def submit(self, mask_flat, dist_flat=None, feat_flat=None, workspace=None, stream=None):
        if workspace is None:
            workspace = torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8,
                                    device=mask_flat.device)
        _check(_lib.edt_batch_submit(self._plan, mask_flat.data_ptr(),
                                     dist_flat.data_ptr() if dist_flat is not None else None,
                                     feat_flat.data_ptr() if feat_flat is not None else None,
                                     workspace.data_ptr(),
                                     workspace.numel() * workspace.element_size(),
                                     _stream_ptr(stream)), "edt_batch_submit")
        return workspace

    def autotune(self, mask_flat, dist_flat=None, feat_flat=None, workspace=None, stream=None):
        """Time the candidate schedules on these buffers and keep the fastest;
        returns [{lane_w, largest_first, ms}, ...] and the chosen index."""
        if workspace is None:
            workspace = torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8,
                                    device=mask_flat.device)
        rep = TuneReport()
        _check(_lib.edt_batch_autotune(self._plan, mask_flat.data_ptr(),
                                       dist_flat.data_ptr() if dist_flat is not None else None,
                                       feat_flat.data_ptr() if feat_flat is not None else None,
                                       workspace.data_ptr(),
                                       workspace.numel() * workspace.element_size(),
                                       _stream_ptr(stream), ctypes.byref(rep)),
               "edt_batch_autotune")
        cands = [{"lane_w": rep.cand[q].lane_w, "largest_first": bool(rep.cand[q].largest_first),
                  "branches": rep.cand[q].branches, "wide_single": bool(rep.cand[q].wide_single),
                  "transpose": bool(rep.cand[q].transpose),
                  "ms": round(float(rep.ms[q]), 4)} for q in range(rep.tried)]
        return cands, int(rep.chosen)

    def set_schedule(self, lane_w: int, largest_first: bool, branches: int = 1,
                     wide_single: bool = False, transpose: bool = False):
        """Use a known schedule (e.g. one autotune picked) for later submissions."""
        sc = Schedule(int(lane_w), int(largest_first), int(branches), int(wide_single),
                      int(transpose))
        _check(_lib.edt_batch_set_schedule(self._plan, ctypes.byref(sc)),
               "edt_batch_set_schedule")

    def close(self):
        if self._plan:
            _check(_lib.edt_plan_destroy(self._plan), "edt_plan_destroy")
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- serving

EDT_ERR_BUSY = -5
EDT_ERR_NOT_READY = -6


class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_inflight", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("max_group", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("mask", ctypes.c_void_p), ("mask_pitch", ctypes.c_int64),
                ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("polarity", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("dist_sq", ctypes.c_void_p), ("feature", ctypes.c_void_p),
                ("out_pitch", ctypes.c_int64), ("stream", ctypes.c_void_p)]


class ServeCounters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("rejected_busy", ctypes.c_uint64),
                ("rejected_too_large", ctypes.c_uint64), ("done", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("pixels_done", ctypes.c_uint64), ("p50_ns", ctypes.c_double),
                ("p99_ns", ctypes.c_double), ("mean_ns", ctypes.c_double),
                ("max_ns", ctypes.c_double), ("gpix_per_s", ctypes.c_double),
                ("hbm_in_use", ctypes.c_size_t), ("hbm_high_water", ctypes.c_size_t)]


def _bind_serve():
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    _lib.edt_serve_create.argtypes = [P, P, sz, P]
    _lib.edt_serve_create.restype = i32
    _lib.edt_serve_submit.argtypes = [P, P, P]
    _lib.edt_serve_submit.restype = i32
    _lib.edt_serve_poll.argtypes = [P, ctypes.c_uint64, P]
    _lib.edt_serve_poll.restype = i32
    _lib.edt_serve_wait.argtypes = [P, ctypes.c_uint64, i64]
    _lib.edt_serve_wait.restype = i32
    _lib.edt_serve_stats.argtypes = [P, P]
    _lib.edt_serve_stats.restype = i32
    _lib.edt_serve_destroy.argtypes = [P]
    _lib.edt_serve_destroy.restype = i32
    _lib.edt_serve_reserved_bytes.argtypes = [P]
    _lib.edt_serve_reserved_bytes.restype = sz


_bind_serve()


class Server:
    """Request server over the library's scheduler (edt_serve_*).

    The arena (``arena_bytes`` of device memory, allocated here with torch)
    holds the workspaces of admitted requests; ``hbm_budget`` (default: the
    arena) caps what admitted work may hold at once.  ``submit`` returns a
    ticket; the tensors of a request are kept alive here until its ticket has
    been waited for."""

    def __init__(self, arena_bytes: int, hbm_budget: int = 0, max_inflight: int = 1024,
                 n_streams: int = 4, max_group: int = 0, device=None):
        device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        self.device = device
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        cfg = ServeConfig(int(hbm_budget), int(max_inflight), int(n_streams), int(max_group))
        self._srv = ctypes.c_void_p()
        _check(_lib.edt_serve_create(ctypes.byref(cfg), self.arena.data_ptr(),
                                     self.arena.numel(), ctypes.byref(self._srv)),
               "edt_serve_create")
        self._held = {}

    @staticmethod
    def reserved_bytes(n_streams: int = 4, max_group: int = 0) -> int:
        """Arena bytes a server keeps for its launch tables."""
        cfg = ServeConfig(0, 1, int(n_streams), int(max_group))
        return int(_lib.edt_serve_reserved_bytes(ctypes.byref(cfg)))

    def submit_raw(self, mask: torch.Tensor, dist, feat, polarity: int = EDT_TO_OBJECT,
                   stream=None) -> int:
        """Queue a request with caller-made outputs (int32 (H, W) tensors, one
        of them may be None).  Returns the ticket; raises EDTError (status
        EDT_ERR_BUSY when the server is full)."""
        mask = _check_mask(mask)
        H, W = mask.shape
        pitch = None
        for t in (dist, feat):
            if t is not None:
                _check_out(t, H, W, mask.device, "output")
                if pitch is not None and t.stride(0) != pitch:
                    raise ValueError("outputs must share one row pitch")
                pitch = t.stride(0)
        if pitch is None:
            raise ValueError("at least one output is needed")
        req = Request(mask.data_ptr(), mask.stride(0), H, W, int(polarity), 0,
                      dist.data_ptr() if dist is not None else None,
                      feat.data_ptr() if feat is not None else None, pitch,
                      _stream_ptr(stream))
        ticket = ctypes.c_uint64(0)
        _check(_lib.edt_serve_submit(self._srv, ctypes.byref(req), ctypes.byref(ticket)),
               "edt_serve_submit")
        self._held[ticket.value] = (mask, dist, feat)
        return ticket.value

    def submit(self, mask: torch.Tensor, polarity: int = EDT_TO_OBJECT,
               want_dist: bool = True, want_feature: bool = False, stream=None) -> int:
        """Queue a request; outputs are allocated here and returned by wait()."""
        H, W = mask.shape
        dist = torch.empty((H, W), dtype=torch.int32, device=mask.device) if want_dist else None
        feat = torch.empty((H, W), dtype=torch.int32, device=mask.device) if want_feature else None
        return self.submit_raw(mask, dist, feat, polarity, stream)

    def poll(self, ticket: int) -> bool:
        done = ctypes.c_int32(0)
        _check(_lib.edt_serve_poll(self._srv, ticket, ctypes.byref(done)), "edt_serve_poll")
        return bool(done.value)

    def wait(self, ticket: int, timeout: float | None = None):
        """Wait for a ticket; returns its (dist, feature) tensors (None where
        not requested).  Raises EDTError with EDT_ERR_NOT_READY on timeout."""
        ns = -1 if timeout is None else int(timeout * 1e9)
        st = _lib.edt_serve_wait(self._srv, ticket, ns)
        if st == EDT_ERR_NOT_READY:
            raise EDTError(st, "edt_serve_wait")
        held = self._held.pop(ticket, (None, None, None))
        _check(st, "edt_serve_wait")
        return held[1], held[2]

    def stats(self) -> dict:
        c = ServeCounters()
        _check(_lib.edt_serve_stats(self._srv, ctypes.byref(c)), "edt_serve_stats")
        return {name: getattr(c, name) for name, _ in ServeCounters._fields_}

    def close(self):
        if self._srv:
            st = _lib.edt_serve_destroy(self._srv)
            self._srv = ctypes.c_void_p()
            self._held.clear()
            _check(st, "edt_serve_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
