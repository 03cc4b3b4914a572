"""Seeded synthetic binary masks shaped like the paper's examples.

The paper's figures show scattered object points with their Voronoi diagram
(Figure fig_voronoi, 30 points), blob-like objects (Figure fig_blobs) and
overlapping cells (Figure fig_cellSeparation); their images are not part of the
paper's text, so these generators draw masks of the same kind from fixed seeds.
Both the HIP path and the CPU oracle are fed from here.  Nothing in this module
computes a distance: it only draws masks.

Every generator returns a C-contiguous ``numpy.uint8`` array (1 = object pixel,
0 = background) and is deterministic for a given seed (numpy PCG64).
"""
from __future__ import annotations

import math
import os

import numpy as np

SEED_BERNOULLI = 2106001
SEED_DISKS = 2106002
SEED_POINTS = 2106003
SEED_BATCH = 2106004
SEED_SERVE = 2106005

_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden")


def paper_example() -> np.ndarray:
    """The 9 x 10 worked example of Section 3.1 (six object pixels), read from
    tests/golden/example_sites.txt (1-based positions as printed)."""
    rows = cols = None
    xs = ys = None
    with open(os.path.join(_GOLDEN, "example_sites.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            if line[0] == "rows":
                rows = int(line[1])
            elif line[0] == "cols":
                cols = int(line[1])
            elif line[0] == "x":
                xs = [int(v) for v in line[1:]]
            elif line[0] == "y":
                ys = [int(v) for v in line[1:]]
    m = np.zeros((rows, cols), np.uint8)
    for x, y in zip(xs, ys):
        m[y - 1, x - 1] = 1
    return m


def bernoulli(H: int, W: int, p: float, seed: int = SEED_BERNOULLI) -> np.ndarray:
    """Object pixels i.i.d. Bernoulli(p)."""
    rng = np.random.default_rng(seed)
    return (rng.random((H, W)) < p).astype(np.uint8)


def disks(H: int, W: int, n_disks: int = 200, rmin: float = 5.0, rmax: float = 200.0,
          p_points: float = 1e-4, seed: int = SEED_DISKS) -> np.ndarray:
    """Filled disks (real radius uniform in [rmin, rmax], real centre uniform
    over the image) OR'ed with isolated Bernoulli(p_points) points.  A pixel
    (y, x) is inside a disk when (y-cy)^2 + (x-cx)^2 <= r^2."""
    rng = np.random.default_rng(seed)
    m = (rng.random((H, W)) < p_points).astype(np.uint8)
    for _ in range(n_disks):
        r = rng.uniform(rmin, rmax)
        cy = rng.uniform(0, H)
        cx = rng.uniform(0, W)
        y0, y1 = max(0, int(math.floor(cy - r))), min(H, int(math.ceil(cy + r)) + 1)
        x0, x1 = max(0, int(math.floor(cx - r))), min(W, int(math.ceil(cx + r)) + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        yy = np.arange(y0, y1, dtype=np.float64)[:, None] - cy
        xx = np.arange(x0, x1, dtype=np.float64)[None, :] - cx
        m[y0:y1, x0:x1] |= (yy * yy + xx * xx <= r * r).astype(np.uint8)
    return m


def points(H: int, W: int, n: int = 30, seed: int = SEED_POINTS) -> np.ndarray:
    """n distinct object points, uniform over the image (Figure fig_voronoi)."""
    rng = np.random.default_rng(seed)
    lin = rng.choice(H * W, size=n, replace=False)
    m = np.zeros(H * W, np.uint8)
    m[lin] = 1
    return m.reshape(H, W)


def corner(H: int, W: int) -> np.ndarray:
    """A single object pixel at (0, 0)."""
    m = np.zeros((H, W), np.uint8)
    m[0, 0] = 1
    return m


def empty(H: int, W: int) -> np.ndarray:
    """All background."""
    return np.zeros((H, W), np.uint8)


def ellipses(H: int, W: int, n: int, amin: float = 4.0, amax: float = 80.0,
             rng: np.random.Generator | None = None, seed: int = SEED_BATCH) -> np.ndarray:
    """n overlapping filled ellipses (cell-like objects, Figure
    fig_cellSeparation): centre uniform over the image, semi-axes a, b uniform
    in [amin, amax], orientation theta uniform in [0, pi).  Pixel (y, x) is
    inside when ((dx cos t + dy sin t)/a)^2 + ((-dx sin t + dy cos t)/b)^2 <= 1."""
    if rng is None:
        rng = np.random.default_rng(seed)
    m = np.zeros((H, W), np.uint8)
    for _ in range(n):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        a, b = rng.uniform(amin, amax), rng.uniform(amin, amax)
        t = rng.uniform(0.0, math.pi)
        r = max(a, b)
        y0, y1 = max(0, int(math.floor(cy - r))), min(H, int(math.ceil(cy + r)) + 1)
        x0, x1 = max(0, int(math.floor(cx - r))), min(W, int(math.ceil(cx + r)) + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        dy = np.arange(y0, y1, dtype=np.float64)[:, None] - cy
        dx = np.arange(x0, x1, dtype=np.float64)[None, :] - cx
        c, s = math.cos(t), math.sin(t)
        u = (dx * c + dy * s) / a
        v = (-dx * s + dy * c) / b
        m[y0:y1, x0:x1] |= (u * u + v * v <= 1.0).astype(np.uint8)
    return m


def ragged_batch(n_images: int = 2048, smin: int = 64, smax: int = 1024,
                 nmin: int = 5, nmax: int = 60, seed: int = SEED_BATCH):
    """Batch of images of uneven size: H and W independently uniform in
    [smin, smax], each with nmin..nmax ellipses, polarity Bernoulli(0.5).
    Returns a list of (mask, polarity)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_images):
        H = int(rng.integers(smin, smax + 1))
        W = int(rng.integers(smin, smax + 1))
        n = int(rng.integers(nmin, nmax + 1))
        pol = int(rng.integers(0, 2))
        out.append((ellipses(H, W, n, rng=rng), pol))
    return out


def serving_requests(n: int, rate: float, smin: int = 128, smax: int = 8192,
                     seed: int = SEED_SERVE):
    """Request stream: Poisson arrivals at ``rate`` per second, square masks of
    side round(exp(U(ln smin, ln smax))), Bernoulli or ellipse masks (50/50) at
    log-uniform density in [1e-4, 0.3], half distance-only and half
    distance+feature.  Returns a list of dicts with keys t (arrival time, s),
    side, kind, density, want_feature, polarity and seed (the mask itself is
    drawn on demand by ``request_mask``)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for q in range(n):
        t += rng.exponential(1.0 / rate)
        side = int(round(math.exp(rng.uniform(math.log(smin), math.log(smax)))))
        kind = "bernoulli" if rng.random() < 0.5 else "ellipses"
        dens = math.exp(rng.uniform(math.log(1e-4), math.log(0.3)))
        reqs.append(dict(t=t, side=side, kind=kind, density=dens,
                         want_feature=bool(rng.random() < 0.5),
                         polarity=0, seed=seed * 1000003 + q))
    return reqs


def request_mask(req) -> np.ndarray:
    """Mask of one serving request (see ``serving_requests``)."""
    s = req["side"]
    rng = np.random.default_rng(req["seed"])
    if req["kind"] == "bernoulli":
        return (rng.random((s, s)) < req["density"]).astype(np.uint8)
    # ellipses whose expected total area is about density * s^2
    amean = 0.5 * (4.0 + min(80.0, max(8.0, s / 8.0)))
    n = max(1, int(req["density"] * s * s / (math.pi * amean * amean)))
    n = min(n, 4000)
    return ellipses(s, s, n, 4.0, min(80.0, max(8.0, s / 8.0)), rng=rng)
