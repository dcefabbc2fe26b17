"""Seeded synthetic images for the all-pairs geodesic distance workloads.

This module only draws pixel values; it holds none of the method's arithmetic
(no weights, no distances).  Both the CPU oracle's tests and the GPU library's
tests and benchmark take their inputs from here, so that the two sides see the
same bytes.

The paper's own test images ("bumps", "hairpin bend", "random", 25x25, grey
levels 1..255, Section 3) are not available.  The generators below stand in
for them: iid uniform images play the role of "random", sums of Gaussian blobs
play the role of "bumps", and a piecewise-constant Voronoi image with 8 bands
plays the role of the multivariate images the paper says the method extends to
(Sections 2 and 5).

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64), whose stream
is stable across platforms, and returns a C-contiguous uint8 array in HWC
order (HW for one channel).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "uniform_image",
    "blob_image",
    "voronoi_image",
    "hairpin_image",
    "deltar_images",
    "spiral_draws",
    "geometric_graph",
    "config1",
    "config2",
    "config3",
    "config4",
    "serving_trace",
    "sha256",
    "Request",
]


def sha256(a: np.ndarray) -> str:
    """SHA-256 of the raw bytes of ``a`` (records which image a result is for)."""
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def uniform_image(rng: np.random.Generator, h: int, w: int, lo: int = 1, hi: int = 255) -> np.ndarray:
    """iid uniform grey levels in [lo, hi], shape (h, w), uint8."""
    return np.ascontiguousarray(rng.integers(lo, hi + 1, size=(h, w), dtype=np.uint8))


def blob_image(rng: np.random.Generator, h: int, w: int, n_blobs: int = 20,
               sigma=(4.0, 20.0), amp=(30.0, 150.0), noise: int = 10) -> np.ndarray:
    """Sum of ``n_blobs`` isotropic Gaussian bumps plus integer noise, clipped to [1, 255].

    Blob centres are uniform over the pixel plane, widths uniform in ``sigma``
    and heights uniform in ``amp``.  The float image is rounded, integer noise
    uniform in {-noise..noise} is added, and the result is clipped to [1, 255].
    """
    yy, xx = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64), indexing="ij")
    img = np.zeros((h, w), dtype=np.float64)
    cy = rng.uniform(0.0, h, size=n_blobs)
    cx = rng.uniform(0.0, w, size=n_blobs)
    sg = rng.uniform(sigma[0], sigma[1], size=n_blobs)
    am = rng.uniform(amp[0], amp[1], size=n_blobs)
    for i in range(n_blobs):
        img += am[i] * np.exp(-((yy - cy[i]) ** 2 + (xx - cx[i]) ** 2) / (2.0 * sg[i] ** 2))
    img = np.rint(img).astype(np.int64)
    img += rng.integers(-noise, noise + 1, size=(h, w))
    return np.ascontiguousarray(np.clip(img, 1, 255).astype(np.uint8))


def hairpin_image(rng: np.random.Generator, h: int = 25, w: int = 25, half_width: float = 1.2,
                  channel=(10, 30), background=(150, 250)) -> np.ndarray:
    """A dark hairpin-shaped channel on a bright noisy background, uint8 (h, w).

    The channel's centre line runs up the left leg (x = 0.3 w, from y = 0.9 h
    to y = 0.4 h), over a half circle of radius 0.2 w centred at (0.4 h, 0.5 w),
    and down the right leg (x = 0.7 w) to y = 0.9 h.  Pixels within
    ``half_width`` of the centre line draw iid values in ``channel``, the others
    in ``background`` (both inclusive).  With the sum-of-grey-levels metric the
    cheap paths follow the bend.
    """
    yy, xx = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64), indexing="ij")
    cy, cx, r = 0.4 * h, 0.5 * w, 0.2 * w
    y0, y1 = 0.4 * h, 0.9 * h
    def leg(x0):
        dy = np.where(yy < y0, y0 - yy, np.where(yy > y1, yy - y1, 0.0))
        return np.hypot(xx - x0, dy)
    ring = np.abs(np.hypot(yy - cy, xx - cx) - r)
    ring = np.where(yy <= cy, ring, np.inf)  # the upper half circle only
    dist = np.minimum(np.minimum(leg(cx - r), leg(cx + r)), ring)
    lo = rng.integers(channel[0], channel[1] + 1, size=(h, w))
    hi = rng.integers(background[0], background[1] + 1, size=(h, w))
    return np.ascontiguousarray(np.where(dist <= half_width, lo, hi).astype(np.uint8))


def deltar_images(seed: int = 7, side: int = 25) -> dict:
    """Stand-ins for the paper's three side x side comparison images (Section 3):
    "random" (iid 1..255), "bumps" (6 Gaussian blobs of width 2..6 px on the
    blob generator) and "hairpin" (hairpin_image)."""
    rng = np.random.default_rng(seed)
    return {"random": uniform_image(rng, side, side),
            "bumps": blob_image(rng, side, side, n_blobs=6, sigma=(2.0, 6.0), amp=(60.0, 200.0), noise=5),
            "hairpin": hairpin_image(rng, side, side)}


def spiral_draws(seed: int, n: int) -> np.ndarray:
    """n uniform 32-bit draws for the spiral methods' random selections."""
    return np.random.default_rng(seed).integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)


def geometric_graph(rng: np.random.Generator, n: int, k: int = 6, wmax: int = 100):
    """A connected undirected graph in CSR form (row_ptr int64, col int32,
    weight int32), rows sorted by neighbour id.

    n points uniform in the unit square; every point is joined to its k
    nearest points, and consecutive points in x order are joined as well (a
    chain that makes the graph connected).  An edge's weight is
    1 + floor(wmax * sqrt(n) * |p - q|), the same in both directions, so it is
    at least 1 and about wmax for a typical neighbour spacing.
    """
    from scipy.spatial import cKDTree
    pts = rng.uniform(0.0, 1.0, size=(n, 2))
    edges = set()
    if n > 1:
        kk = min(k + 1, n)
        _, nn = cKDTree(pts).query(pts, k=kk)
        nn = np.asarray(nn).reshape(n, kk)
        for u in range(n):
            for v in nn[u, 1:]:
                v = int(v)
                if v != u:
                    edges.add((min(u, v), max(u, v)))
        order = np.argsort(pts[:, 0], kind="stable")
        for a, b in zip(order[:-1], order[1:]):
            a, b = int(a), int(b)
            edges.add((min(a, b), max(a, b)))
    e = np.array(sorted(edges), dtype=np.int64).reshape(-1, 2)
    w = 1 + np.floor(wmax * np.sqrt(n) * np.linalg.norm(pts[e[:, 0]] - pts[e[:, 1]], axis=1)).astype(np.int64)
    src = np.concatenate([e[:, 0], e[:, 1]])
    dst = np.concatenate([e[:, 1], e[:, 0]])
    ww = np.concatenate([w, w])
    o = np.lexsort((dst, src))
    src, dst, ww = src[o], dst[o], ww[o]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, src + 1, 1)
    rp = np.cumsum(rp)
    return rp, dst.astype(np.int32), ww.astype(np.int32)


def voronoi_image(rng: np.random.Generator, h: int, w: int, bands: int = 8, n_seeds: int = 50,
                  noise_sigma: float = 6.0) -> np.ndarray:
    """Piecewise-constant multiband image on the Voronoi cells of random seed pixels.

    ``n_seeds`` distinct seed pixels are drawn uniformly; each pixel belongs to
    its nearest seed (Euclidean, ties to the lower seed id).  Each region gets a
    per-band mean uniform in [0, 255]; Gaussian noise of std ``noise_sigma`` is
    added, then values are rounded and clipped to [0, 255].  Shape (h, w, bands).
    """
    flat = rng.choice(h * w, size=n_seeds, replace=False)
    sy, sx = (flat // w).astype(np.float64), (flat % w).astype(np.float64)
    yy, xx = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64), indexing="ij")
    d2 = (yy[None] - sy[:, None, None]) ** 2 + (xx[None] - sx[:, None, None]) ** 2
    region = np.argmin(d2, axis=0)  # argmin returns the first (lowest id) on ties
    means = rng.uniform(0.0, 255.0, size=(n_seeds, bands))
    img = means[region] + rng.normal(0.0, noise_sigma, size=(h, w, bands))
    return np.ascontiguousarray(np.clip(np.rint(img), 0, 255).astype(np.uint8))


# --- the five workload recipes -------------------------------------------------------------

def config1() -> np.ndarray:
    """32x32 single-channel, iid uniform in [1, 255], seed 0."""
    return uniform_image(np.random.default_rng(0), 32, 32)


def config2() -> np.ndarray:
    """128x128 single-channel blob image, seed 1."""
    return blob_image(np.random.default_rng(1), 128, 128)


def config3() -> np.ndarray:
    """192x192x8 Voronoi image (50 regions), seed 2."""
    return voronoi_image(np.random.default_rng(2), 192, 192)


def config4(n_images: int = 256, lo: int = 24, hi: int = 96, seed: int = 3):
    """A batch of ``n_images`` single-channel iid images with sides uniform in {lo..hi}.

    Returns a list of (h, w) uint8 arrays; heights and widths are drawn
    independently, so images are generally not square.
    """
    rng = np.random.default_rng(seed)
    hs = rng.integers(lo, hi + 1, size=n_images)
    ws = rng.integers(lo, hi + 1, size=n_images)
    return [uniform_image(rng, int(h), int(w)) for h, w in zip(hs, ws)]


@dataclass
class Request:
    """One request of the serving workload."""
    t_arrival: float                 # seconds after the start of the trace
    kind: str                        # "all_pairs" or "multi_source"
    image_id: int                    # index into the trace's image table
    sources: np.ndarray = field(default=None)  # int32 pixel ids for multi-source jobs


def serving_trace(rate: float, n_requests: int, seed: int = 4, p_all_pairs: float = 0.7,
                  side=(64, 192), big_side: int = 512, n_big: int = 8, max_k: int = 512):
    """Poisson request stream mixing all-pairs jobs and multi-source jobs.

    All-pairs jobs run on their own square blob image of side uniform in
    ``side``; multi-source jobs pick one of ``n_big`` pre-generated
    ``big_side``-square blob images and 1..``max_k`` distinct random sources.
    Returns ``(requests, images)`` where ``images`` is the image table.
    """
    rng = np.random.default_rng(seed)
    images = [blob_image(rng, big_side, big_side) for _ in range(n_big)]
    reqs = []
    t = 0.0
    for _ in range(n_requests):
        t += rng.exponential(1.0 / rate)
        if rng.uniform() < p_all_pairs:
            s = int(rng.integers(side[0], side[1] + 1))
            images.append(blob_image(rng, s, s))
            reqs.append(Request(t, "all_pairs", len(images) - 1))
        else:
            b = int(rng.integers(0, n_big))
            k = int(rng.integers(1, max_k + 1))
            src = rng.choice(big_side * big_side, size=k, replace=False).astype(np.int32)
            reqs.append(Request(t, "multi_source", b, np.sort(src)))
    return reqs, images
