"""Seeded synthetic scenes standing in for the paper's aerial images.

The paper evaluates on five Google Maps RGB images (Table II) that are not
available here; these generators produce scenes of the same kind -- flat
background, rectangular roofs, long road strips, a runway -- with per-band
means and Gaussian noise, at the sizes the workloads call for.  Nothing in
this module computes any part of the level set method: it only draws inputs,
so both the GPU library's tests and the CPU oracle consume the same arrays.

Layout of every image: H x W x B, row-major, band fastest, float64 (cast per
path).  Masks are uint8 H x W, nonzero = inside the initial curve (eq. (13)).

All randomness comes from ``numpy.random.default_rng`` seeded with a tuple
(workload id, image id, seed); ``array_digest`` gives a SHA-256 of an array so
that tests can pin the streams.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

TINY, LARGE, BATCH, PRECISION, SERVING = 1, 2, 3, 4, 5


@dataclass
class Scene:
    image: np.ndarray          # H x W x B float64
    init_region: np.ndarray    # uint8 H x W, initial curve for the region term
    init_edge: np.ndarray      # uint8 H x W, seeds inside objects for the edge term
    truth: np.ndarray          # uint8 H x W, union of painted objects
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.image.shape


def array_digest(a: np.ndarray) -> str:
    a = np.ascontiguousarray(a)
    h = hashlib.sha256()
    h.update(str(a.dtype).encode())
    h.update(str(a.shape).encode())
    h.update(a.tobytes())
    return h.hexdigest()


def _rng(workload: int, image_id: int, seed: int) -> np.random.Generator:
    return np.random.default_rng([workload, image_id, seed])


def centred_square(h: int, w: int, side_h: int, side_w: int) -> np.ndarray:
    m = np.zeros((h, w), np.uint8)
    y0 = (h - side_h) // 2
    x0 = (w - side_w) // 2
    m[y0:y0 + side_h, x0:x0 + side_w] = 1
    return m


def _paint_rects(img, truth, rng, n, side_lo, side_hi, value_fn):
    h, w, _ = img.shape
    rects = []
    for _ in range(n):
        rh = int(rng.integers(side_lo, side_hi + 1))
        rw = int(rng.integers(side_lo, side_hi + 1))
        rh, rw = min(rh, h), min(rw, w)
        y0 = int(rng.integers(0, h - rh + 1))
        x0 = int(rng.integers(0, w - rw + 1))
        img[y0:y0 + rh, x0:x0 + rw, :] = value_fn()
        truth[y0:y0 + rh, x0:x0 + rw] = 1
        rects.append((y0, x0, rh, rw))
    return rects


def scene_tiny(seed: int = 0, size: int = 256, n_rects: int = 3, noise: float = 0.05,
               bands: int = 1, workload: int = TINY, image_id: int = 0) -> Scene:
    """Flat background 0.3, `n_rects` rectangles of 0.7 (sides 20-80 px, random
    positions, overlaps allowed), i.i.d. Gaussian noise, no clipping.  Initial
    curve: a centred square of half the side (128 x 128 at 256 x 256)."""
    rng = _rng(workload, image_id, seed)
    h = w = size
    img = np.full((h, w, bands), 0.3)
    truth = np.zeros((h, w), np.uint8)
    rects = _paint_rects(img, truth, rng, n_rects, 20, 80, lambda: 0.7)
    img += rng.normal(0.0, noise, size=img.shape)
    init = centred_square(h, w, h // 2, w // 2)
    seeds = _edge_seeds_rects(h, w, rects)
    return Scene(img, init, seeds, truth, {"rects": rects, "seed": seed})


def scene_batch_image(seed: int, image_id: int, h: int, w: int, bands: int = 4) -> Scene:
    """The tiny workload's scene model scaled to an uneven H x W image: rectangle
    count round(3 * H * W / 256^2), same geometry in every band, independent
    noise per band (sigma 0.05).  Initial curve: centred half-size rectangle."""
    rng = _rng(BATCH, image_id, seed)
    img = np.full((h, w, bands), 0.3)
    truth = np.zeros((h, w), np.uint8)
    n = int(round(3 * h * w / 256 ** 2))
    rects = _paint_rects(img, truth, rng, n, 20, 80, lambda: 0.7)
    img += rng.normal(0.0, 0.05, size=img.shape)
    init = centred_square(h, w, h // 2, w // 2)
    return Scene(img, init, _edge_seeds_rects(h, w, rects), truth, {"rects": rects})


def batch_shapes(seed: int = 0, n: int = 64, lo: int = 512, hi: int = 2048):
    rng = _rng(BATCH, 10_000, seed)
    return [(int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))) for _ in range(n)]


def _edge_seeds_rects(h, w, rects, half=2):
    m = np.zeros((h, w), np.uint8)
    for (y0, x0, rh, rw) in rects:
        cy, cx = y0 + rh // 2, x0 + rw // 2
        m[max(cy - half, 0):cy + half + 1, max(cx - half, 0):cx + half + 1] = 1
    return m


def _strip(img, truth, seeds, rng, cy, cx, theta, width, length, means, seed_every=128):
    """Paint a strip of `width` px centred on the line through (cy, cx) with
    direction theta; `length` None = across the whole image."""
    h, w, _ = img.shape
    dy, dx = math.sin(theta), math.cos(theta)
    if length is None:
        y_lo, y_hi, x_lo, x_hi = 0, h, 0, w
    else:
        ext = length / 2 + width
        y_lo, y_hi = max(int(cy - abs(dy) * ext - width), 0), min(int(cy + abs(dy) * ext + width) + 1, h)
        x_lo, x_hi = max(int(cx - abs(dx) * ext - width), 0), min(int(cx + abs(dx) * ext + width) + 1, w)
    yy = np.arange(y_lo, y_hi, dtype=np.float64)[:, None]
    xx = np.arange(x_lo, x_hi, dtype=np.float64)[None, :]
    rel_y, rel_x = yy - cy, xx - cx
    across = np.abs(rel_x * dy - rel_y * dx)
    inside = across <= width / 2.0
    if length is not None:
        along = rel_x * dx + rel_y * dy
        inside &= np.abs(along) <= length / 2.0
    sub = img[y_lo:y_hi, x_lo:x_hi, :]
    sub[inside] = means
    truth[y_lo:y_hi, x_lo:x_hi][inside] = 1
    # seeds (5 x 5) every `seed_every` px along the centre line, inside the
    # image and, for a finite strip, at least 5 px inside its ends
    half_len = (length / 2.0 - 5.0) if length is not None else float(h + w)
    t = -half_len
    while t <= half_len:
        py, px = int(round(cy + t * dy)), int(round(cx + t * dx))
        if 2 <= py < h - 2 and 2 <= px < w - 2:
            seeds[py - 2:py + 3, px - 2:px + 3] = 1
        t += seed_every


def scene_multiband(seed: int = 0, size: int = 4096, bands: int = 4, n_roofs: int = 40,
                    n_roads: int = 6, runway: bool = False, noise: float = 0.03,
                    workload: int = LARGE, image_id: int = 0, height: int | None = None,
                    width: int | None = None) -> Scene:
    """Multiband aerial-like scene in [0, 1] (B, G, R, NIR): per-band background
    ~ U(0.2, 0.4); `n_roads` full-length strips (width 8-20 px, random angle,
    through a uniform point, band means ~ U(0.45, 0.6)); optionally one runway
    (width 60-120 px, length 2000-4000 px, fully inside); then `n_roofs`
    rectangles (sides 10-120 px, band means ~ U(0.5, 0.8)) painted over roads;
    Gaussian noise per pixel and band; clipped to [0, 1].

    Initial curves: region term -- centred square of half the side; edge term --
    5 x 5 seeds at roof centres and every 128 px along road/runway centre lines.
    Sizes are those of a 4096 px side (roads, roofs) and of an 8192 px side
    (runway), scaled down for smaller scenes, never up."""
    rng = _rng(workload, image_id, seed)
    h = height or size
    w = width or size
    runway_geom = None
    img = np.empty((h, w, bands))
    img[:] = rng.uniform(0.2, 0.4, size=bands)
    truth = np.zeros((h, w), np.uint8)
    seeds = np.zeros((h, w), np.uint8)
    scale = min(1.0, min(h, w) / 4096.0)   # roads and roofs: sizes given at a 4096 px side
    rscale = min(1.0, min(h, w) / 8192.0)  # runway: sizes given at an 8192 px side
    for _ in range(n_roads):
        width_px = rng.uniform(8, 20)
        theta = rng.uniform(0, math.pi)
        cy, cx = rng.uniform(0, h), rng.uniform(0, w)
        means = rng.uniform(0.45, 0.6, size=bands)
        _strip(img, truth, seeds, rng, cy, cx, theta, width_px, None, means)
    if runway:
        width_px = rng.uniform(60, 120) * max(rscale, 1.0 / 64)
        length = rng.uniform(2000, 4000) * max(rscale, 1.0 / 64)
        theta = rng.uniform(0, math.pi)
        ext_y = abs(math.sin(theta)) * length / 2 + width_px
        ext_x = abs(math.cos(theta)) * length / 2 + width_px
        cy = rng.uniform(min(ext_y, h / 2), max(h - ext_y, h / 2))
        cx = rng.uniform(min(ext_x, w / 2), max(w - ext_x, w / 2))
        means = rng.uniform(0.45, 0.6, size=bands)
        _strip(img, truth, seeds, rng, cy, cx, theta, width_px, length, means)
        runway_geom = (cy, cx, theta, width_px, length)
    side_hi = max(12, int(round(120 * max(scale, 0.125))))
    side_lo = min(10, side_hi)
    rects = _paint_rects(img, truth, rng, n_roofs, side_lo, side_hi,
                         lambda: rng.uniform(0.5, 0.8, size=bands))
    seeds |= _edge_seeds_rects(h, w, rects)
    img += rng.normal(0.0, noise, size=img.shape)
    np.clip(img, 0.0, 1.0, out=img)
    init = centred_square(h, w, h // 2, w // 2)
    return Scene(img, init, seeds, truth, {"rects": rects, "seed": seed, "runway": runway_geom})


def crop_scene(sc: Scene, y0: int, x0: int, h: int, w: int) -> Scene:
    """An H x W window of a scene, with its own initial curve (centred square
    of half the window side) and the window's edge seeds and truth."""
    img = np.ascontiguousarray(sc.image[y0:y0 + h, x0:x0 + w])
    truth = np.ascontiguousarray(sc.truth[y0:y0 + h, x0:x0 + w])
    seeds = np.ascontiguousarray(sc.init_edge[y0:y0 + h, x0:x0 + w])
    return Scene(img, centred_square(h, w, h // 2, w // 2), seeds, truth, {"crop": (y0, x0, h, w)})


def scene_large(seed: int = 0, size: int = 4096) -> Scene:
    """4096 x 4096 x 4 multiband scene: 40 roofs, 6 roads, noise 0.03."""
    return scene_multiband(seed, size=size, n_roofs=40, n_roads=6, workload=LARGE)


def scene_precision(seed: int = 0, size: int = 8192) -> Scene:
    """8192 x 8192 x 4: one runway (60-120 px wide, 2-4 km long at ~1 m/px)
    and 200 roofs, noise 0.03."""
    return scene_multiband(seed, size=size, n_roofs=200, n_roads=0, runway=True,
                           workload=PRECISION)


@dataclass
class Job:
    job_id: int
    arrival_s: float
    side: int
    bands: int
    term: str
    iters: int


def serving_trace(seed: int = 0, n_jobs: int = 2000, qps: float = 10.0):
    """Poisson arrivals at `qps`; side log-uniform in [256, 4096]; 1 or 4 bands;
    region or edge term 50/50; 100-300 iterations."""
    rng = _rng(SERVING, 0, seed)
    gaps = rng.exponential(1.0 / qps, size=n_jobs)
    t = np.cumsum(gaps)
    jobs = []
    for i in range(n_jobs):
        side = int(round(math.exp(rng.uniform(math.log(256), math.log(4096)))))
        bands = 1 if rng.random() < 0.5 else 4
        term = "region" if rng.random() < 0.5 else "edge"
        iters = int(rng.integers(100, 301))
        jobs.append(Job(i, float(t[i]), side, bands, term, iters))
    return jobs


def serving_pool(seed: int = 0, size: int = 4096) -> Scene:
    """Resident source of serving inputs: one multiband scene of the large
    workload's model (roads, roofs) at `size`; every job takes a window of it
    (serving_window), so jobs of side s see object counts scaled by area."""
    return scene_multiband(seed, size=size, n_roofs=max(1, int(round(40 * (size / 4096.0) ** 2))),
                           n_roads=max(1, int(round(6 * size / 4096.0))), workload=SERVING, image_id=0)


def serving_window(job: Job, pool_size: int = 4096, seed: int = 0):
    """Top-left corner of job's side x side window in the serving pool."""
    rng = _rng(SERVING, job.job_id + 1, seed)
    side = min(job.side, pool_size)
    return int(rng.integers(0, pool_size - side + 1)), int(rng.integers(0, pool_size - side + 1))


def serving_scene(job: Job, seed: int = 0) -> Scene:
    """Scene for one serving job: the multiband generator with counts scaled
    by area; single-band jobs take the band mean."""
    area = job.side * job.side / 4096.0 ** 2
    sc = scene_multiband(seed, size=job.side, bands=4, n_roofs=max(1, int(round(40 * area))),
                         n_roads=max(1, int(round(6 * math.sqrt(area)))), workload=SERVING,
                         image_id=job.job_id + 1)
    if job.bands == 1:
        sc.image = sc.image.mean(axis=2, keepdims=True)
    return sc


def rectangle_scene(h: int = 256, w: int = 256, rect=(98, 93, 60, 70), inside: float = 0.7,
                    outside: float = 0.3, noise: float = 0.0, seed: int = 0, bands: int = 1):
    """Noise-free (or noisy) single rectangle: returns (image, truth mask)."""
    rng = _rng(99, 0, seed)
    img = np.full((h, w, bands), outside)
    y0, x0, rh, rw = rect
    img[y0:y0 + rh, x0:x0 + rw, :] = inside
    truth = np.zeros((h, w), np.uint8)
    truth[y0:y0 + rh, x0:x0 + rw] = 1
    if noise > 0:
        img += rng.normal(0.0, noise, size=img.shape)
    return img, truth
