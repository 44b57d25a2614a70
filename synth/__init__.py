"""Seeded synthetic inputs for the hierarchical Russian-roulette hot path.

This module only draws random numbers: positions, dither tiles, range-query
triples, request streams.  It holds none of the method's arithmetic (no radical
inverse, no Morton code, no acceptance test, no shift lookup), so both the
oracle and the HIP path can consume the same arrays without sharing any of the
computation that is being checked.

The paper has no datasets or experiments (it is an algorithmic note), so every
workload here is a synthetic stand-in with the shapes of the paper's setting:
two large vertex sets (eye vertices e_j, light vertices l_i, Section 1) and a
per-eye Cranley-Patterson shift drawn from a 64x64 dither tile (Section 1 and
the teaser figure).  All generators use numpy's PCG64 (``default_rng(seed)``)
and return fresh arrays; nothing is cached.

Workload recipes (sizes, seeds and distributions):

* ``tiny``      1024 lights, 4096 eyes (64x64 pixels), uniform in [0,1)^3,
                tile seed 100, lights seed 101, eyes seed 102, s = 1e-3, leaf 1;
                plus 100k range queries (seed 103) with b - a <= 4096.
* ``rangemin``  2^28 queries with a < b uniform u32 and a uniform u32 shift
                (seed 200); check subset of 2^16 queries with b - a <= 2^16
                (seed 201).
* ``frame``     1920x1080 eyes and 2^20 lights from one 64-component isotropic
                Gaussian mixture (sigma 0.02) in the unit cube (seed 300 for
                the centres, 301 lights, 302 eyes), s = 1e-4, leaf 1.
* ``batched``   256 caches, cache c uses seed 400 + c: its own mixture,
                2^U[10,20] lights and 2^U[10,16] eyes, s = 1e-4.
* ``served``    16 resident hierarchies (seed 500 + h) of 2^(16 + 6h/15)
                lights; a Poisson request stream (seed 600) of eye tiles of
                2^U[8,18] eyes against a uniformly chosen hierarchy, each with
                its own random 32-bit shift offset.
"""

from __future__ import annotations

import numpy as np

TILE_SIDE = 64
TILE_SIZE = TILE_SIDE * TILE_SIDE
SIGMA = 0.02
N_CENTERS = 64


def dither_tile(seed: int = 100) -> np.ndarray:
    """64x64 tile of 32-bit shifts: a seeded permutation of k * 2^20, k < 4096.

    Row-major: element ``u * 64 + v``.  A true blue-noise tile is not
    available offline; a permutation of equally spaced values keeps the
    marginal distribution of the shifts stratified, which is what the
    traversal depends on.
    """
    rng = np.random.default_rng(seed)
    perm = rng.permutation(TILE_SIZE).astype(np.uint32)
    return (perm << np.uint32(20)).astype(np.uint32)


def uniform_points(n: int, seed: int) -> np.ndarray:
    """``n`` fp32 points uniform in [0,1)^3, shape (n, 3), C-contiguous."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.random((n, 3), dtype=np.float32))


def mixture_centers(seed: int, k: int = N_CENTERS) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((k, 3))


def mixture_points(n: int, centers: np.ndarray, seed: int,
                   sigma: float = SIGMA) -> np.ndarray:
    """``n`` fp32 points from an isotropic Gaussian mixture, clamped to [0,1]^3.

    Each point picks a component uniformly, adds N(0, sigma^2 I) in float64,
    clamps to the unit cube and is cast to fp32.
    """
    rng = np.random.default_rng(seed)
    comp = rng.integers(0, centers.shape[0], size=n)
    pts = centers[comp] + rng.normal(0.0, sigma, size=(n, 3))
    np.clip(pts, 0.0, 1.0, out=pts)
    return np.ascontiguousarray(pts.astype(np.float32))


def range_queries(n: int, seed: int, max_len: int | None = None):
    """Range-minimum queries (a, b, r) as three u32 arrays with a < b.

    With ``max_len`` None, a and b are two independent uniform u32 draws
    (equal pairs redrawn) ordered so that a < b.  Otherwise a is uniform in
    [0, 2^32 - 1 - max_len] and b = a + L with L uniform in [1, max_len].
    The shift r is uniform over all 32-bit values.
    """
    rng = np.random.default_rng(seed)
    if max_len is None:
        x = rng.integers(0, 1 << 32, size=n, dtype=np.uint64)
        y = rng.integers(0, 1 << 32, size=n, dtype=np.uint64)
        eq = np.nonzero(x == y)[0]
        while eq.size:
            y[eq] = rng.integers(0, 1 << 32, size=eq.size, dtype=np.uint64)
            eq = eq[x[eq] == y[eq]]
        a = np.minimum(x, y).astype(np.uint32)
        b = np.maximum(x, y).astype(np.uint32)
        del x, y
    else:
        a64 = rng.integers(0, (1 << 32) - 1 - max_len + 1, size=n,
                           dtype=np.uint64)
        ln = rng.integers(1, max_len + 1, size=n, dtype=np.uint64)
        a = a64.astype(np.uint32)
        b = (a64 + ln).astype(np.uint32)
    r = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    return a, b, r


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def tiny():
    """Uniform 1024 lights x 4096 eyes; 64 px wide; s = 1e-3; leaf size 1."""
    return dict(tile=dither_tile(100), lights=uniform_points(1024, 101),
                eyes=uniform_points(4096, 102), width=64, s=1e-3, leaf=1)


def tiny_queries():
    return range_queries(100_000, 103, max_len=4096)


def rangemin_queries(n: int = 1 << 28):
    return range_queries(n, 200)


def rangemin_check_queries():
    return range_queries(1 << 16, 201, max_len=1 << 16)


def frame(n_lights: int = 1 << 20, width: int = 1920, height: int = 1080):
    """Frame-scale scene: one shared 64-Gaussian mixture for lights and eyes."""
    c = mixture_centers(300)
    return dict(tile=dither_tile(100), lights=mixture_points(n_lights, c, 301),
                eyes=mixture_points(width * height, c, 302), width=width,
                s=1e-4, leaf=1)


def batched_cache(c: int):
    """Cache ``c`` of the 256-cache batch: own mixture and log-uniform sizes."""
    rng = np.random.default_rng(400 + c)
    n_l = int(np.floor(2.0 ** rng.uniform(10.0, 20.0)))
    n_e = int(np.floor(2.0 ** rng.uniform(10.0, 16.0)))
    centers = rng.random((N_CENTERS, 3))
    seeds = rng.integers(0, 1 << 31, size=2)
    return dict(lights=mixture_points(n_l, centers, int(seeds[0])),
                eyes=mixture_points(n_e, centers, int(seeds[1])), width=64,
                s=1e-4)


def served_hierarchy(h: int):
    n_l = int(np.floor(2.0 ** (16.0 + 6.0 * h / 15.0)))
    rng = np.random.default_rng(500 + h)
    centers = rng.random((N_CENTERS, 3))
    seed_l = int(rng.integers(0, 1 << 31))
    return dict(lights=mixture_points(n_l, centers, seed_l), centers=centers,
                seed=500 + h)


def served_requests(n_req: int, rate_hz: float, n_hier: int = 16,
                    seed: int = 600, lo: float = 8.0, hi: float = 18.0):
    """Poisson request stream: arrival times (s), hierarchy id, size, offset,
    and a per-request seed for its eye positions."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_req)
    t = np.cumsum(gaps) - gaps[0]
    hid = rng.integers(0, n_hier, size=n_req)
    size = np.floor(2.0 ** rng.uniform(lo, hi, size=n_req)).astype(np.int64)
    offset = rng.integers(0, 1 << 32, size=n_req,
                          dtype=np.uint64).astype(np.uint32)
    eseed = rng.integers(0, 1 << 31, size=n_req)
    return dict(t=t, hier=hid, size=size, offset=offset, eye_seed=eseed)


def request_eyes(centers: np.ndarray, n: int, seed: int) -> np.ndarray:
    return mixture_points(n, centers, int(seed))
