"""Exact Euclidean distance transform and feature transform on MI355X.

Thin Python binding of libedt (the C ABI in include/edt.h): it checks torch
tensors, allocates outputs and workspace with torch, and passes raw device
pointers and torch's current HIP stream to the library.  Every step of the
transform runs in the library's HIP kernels; there is no fallback.

    import paper_2106_03503_amd as edt
    D = edt.sq(mask)                 # int32 squared distances
    D, F = edt.feature(mask)         # + nearest-site linear index
    d = edt.sqrt_f32(D)              # float32 distances
    L = edt.regions(mask, F)         # Voronoi regions of the connected objects
    srv = edt.Server(1 << 30)        # request server: submit / wait / stats
"""
from ._lib import (  # noqa: F401
    EDT_INF_SQ,
    EDT_METRIC_CHAMFER34,
    EDT_METRIC_CHESSBOARD,
    EDT_METRIC_CITYBLOCK,
    EDT_METRIC_EUCLIDEAN_SQ,
    EDT_NO_SITE,
    EDT_TO_BACKGROUND,
    EDT_TO_OBJECT,
    BatchPlan,
    Server,
    EDTError,
    abi_version,
    danielsson,
    feature,
    feature_noalloc,
    library_path,
    profile_begin,
    profile_end,
    regions,
    sq,
    sqrt_f32,
    dist_f32,
    workspace_bytes,
)
