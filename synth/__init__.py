"""Seeded synthetic inputs for hierarchical agglomerative clustering.

This module only draws points. It holds none of the clustering arithmetic, so
both the FP64 oracle (``oracle/``) and the GPU library's callers (tests,
``bench.py``) can use it without sharing any part of the method.

Every generator draws in float64 with numpy's PCG64 ``default_rng(seed)``,
rounds to float32 once, and redraws rows that collide exactly after rounding
(duplicate points would give exact distance ties, and the dendrogram of an
input with ties is not unique).

Workload shapes (they stand in for the paper's synthetic UniformFill and
GaussianDisc sets and for its real data sets, none of which are reproduced):

* ``uniform``   i.i.d. uniform in [0,1]^d.
* ``blobs``     mixture of ``k`` isotropic Gaussians, centres uniform in
                [0,1]^d, equal weights, standard deviation ``sigma``.
* ``sphere_blobs``  unit-norm vectors around ``k`` random unit centres
                (Gaussian noise of std ``sigma``, then renormalised).
* ``uniform_fill``  the paper's UniformFill law (Sec. 6 data sets): uniform
                in a hypergrid of side sqrt(n).
* ``gaussian_disc`` the paper's GaussianDisc law: a hypergrid of side
                5 sqrt(n); 90% of the points split equally among five
                Gaussians with means uniform in the hypergrid and standard
                deviation sqrt(n)/6 (so that the stated diameter sqrt(n) is six
                standard deviations), the other 10% uniform in the hypergrid.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform",
    "blobs",
    "sphere_blobs",
    "uniform_fill",
    "gaussian_disc",
    "dedup_rows",
    "workload",
    "WORKLOADS",
    "serving_trace",
]


def _redraw_duplicates(x32: np.ndarray, redraw) -> np.ndarray:
    """Replace exact duplicate float32 rows (keeping the first copy)."""
    for _ in range(64):
        dup = dedup_rows(x32)
        if dup.size == 0:
            return x32
        x32[dup] = redraw(dup.size).astype(np.float32)
    raise RuntimeError("could not remove duplicate rows")


def dedup_rows(x32: np.ndarray) -> np.ndarray:
    """Indices of rows that repeat an earlier row exactly (bitwise)."""
    if x32.shape[0] < 2:
        return np.zeros(0, dtype=np.int64)
    v = np.ascontiguousarray(x32).view(np.dtype((np.void, x32.dtype.itemsize * x32.shape[1])))[:, 0]
    _, first = np.unique(v, return_index=True)
    keep = np.zeros(x32.shape[0], dtype=bool)
    keep[first] = True
    return np.nonzero(~keep)[0]


def uniform(n: int, d: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = rng.random((n, d)).astype(np.float32)
    return _redraw_duplicates(x, lambda m: rng.random((m, d)))


def blobs(n: int, d: int, k: int, sigma: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    centres = rng.random((k, d))
    lab = rng.integers(0, k, size=n)
    x = (centres[lab] + rng.normal(0.0, sigma, size=(n, d))).astype(np.float32)

    def redraw(m):
        lab2 = rng.integers(0, k, size=m)
        return centres[lab2] + rng.normal(0.0, sigma, size=(m, d))

    return _redraw_duplicates(x, redraw)


def sphere_blobs(n: int, d: int, k: int, sigma: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    c = rng.normal(size=(k, d))
    c /= np.linalg.norm(c, axis=1, keepdims=True)

    def draw(m):
        lab = rng.integers(0, k, size=m)
        y = c[lab] + rng.normal(0.0, sigma, size=(m, d))
        return y / np.linalg.norm(y, axis=1, keepdims=True)

    x = draw(n).astype(np.float32)
    return _redraw_duplicates(x, draw)


def uniform_fill(n: int, d: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    side = float(np.sqrt(n))
    x = (rng.random((n, d)) * side).astype(np.float32)
    return _redraw_duplicates(x, lambda m: rng.random((m, d)) * side)


def gaussian_disc(n: int, d: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    side = 5.0 * float(np.sqrt(n))
    sigma = float(np.sqrt(n)) / 6.0
    means = rng.random((5, d)) * side
    ng = int(round(0.9 * n))
    lab = np.arange(ng) % 5
    x = np.empty((n, d))
    x[:ng] = means[lab] + rng.normal(0.0, sigma, size=(ng, d))
    x[ng:] = rng.random((n - ng, d)) * side
    x = x[rng.permutation(n)].astype(np.float32)

    def redraw(m):
        # a duplicate is redrawn from the uniform part of the law
        return rng.random((m, d)) * side

    return _redraw_duplicates(x, redraw)


# Named workloads. Sizes follow the clustering configurations this library is
# measured on: a small parity case, 1M and 10M two-dimensional Gaussian
# mixtures (Ward and complete), 1M ten-dimensional sets (average) and 200K
# unit vectors in 128 dimensions.
WORKLOADS = {
    "u2k_d2": lambda seed=0: uniform(2_000, 2, seed),
    "blob50_1m_d2": lambda seed=11: blobs(1_000_000, 2, 50, 0.01, seed),
    "blob50_10m_d2": lambda seed=12: blobs(10_000_000, 2, 50, 0.01, seed),
    "u1m_d10": lambda seed=21: uniform(1_000_000, 10, seed),
    "blob100_1m_d10": lambda seed=22: blobs(1_000_000, 10, 100, 0.02, seed),
    "vmf1000_200k_d128": lambda seed=31: sphere_blobs(200_000, 128, 1000, 0.1, seed),
    # the paper's synthetic sets (Sec. 6), named as in its running-time table
    "2U1M": lambda seed=61: uniform_fill(1_000_000, 2, seed),
    "2G1M": lambda seed=62: gaussian_disc(1_000_000, 2, seed),
    "5U1M": lambda seed=63: uniform_fill(1_000_000, 5, seed),
    "5G1M": lambda seed=64: gaussian_disc(1_000_000, 5, seed),
    "2U10M": lambda seed=65: uniform_fill(10_000_000, 2, seed),
    "2G10M": lambda seed=66: gaussian_disc(10_000_000, 2, seed),
}


def workload(name: str, n: int | None = None, seed: int | None = None) -> np.ndarray:
    """Draw a named workload; ``n`` overrides the size with the same law."""
    base = {
        "u2k_d2": ("uniform", 2, None, None, 0),
        "blob50_1m_d2": ("blobs", 2, 50, 0.01, 11),
        "blob50_10m_d2": ("blobs", 2, 50, 0.01, 12),
        "u1m_d10": ("uniform", 10, None, None, 21),
        "blob100_1m_d10": ("blobs", 10, 100, 0.02, 22),
        "vmf1000_200k_d128": ("sphere", 128, 1000, 0.1, 31),
    }[name]
    kind, d, k, sigma, s0 = base
    seed = s0 if seed is None else seed
    if n is None:
        return WORKLOADS[name](seed)
    if kind == "uniform":
        return uniform(n, d, seed)
    if kind == "blobs":
        return blobs(n, d, k, sigma, seed)
    return sphere_blobs(n, d, k, sigma, seed)


def serving_trace(num: int, rate_hz: float, seed: int = 41, n_max: int = 200_000):
    """Poisson arrival trace of clustering requests of uneven shape.

    Each request: n log-uniform in [256, n_max], d uniform over {2,3,10,64},
    linkage uniform over {complete, average, ward}, a Gaussian mixture of
    5..100 blobs with sigma uniform in [0.01, 0.05]; request i's points are
    drawn from seed 50000+i (see ``request_points``).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=num)
    t = np.cumsum(gaps) - gaps[0]
    ns = np.floor(np.exp(rng.uniform(np.log(256), np.log(n_max), size=num))).astype(np.int64)
    ds = rng.choice(np.array([2, 3, 10, 64]), size=num)
    links = rng.choice(np.array(["complete", "average", "ward"]), size=num)
    ks = rng.integers(5, 101, size=num)
    sig = rng.uniform(0.01, 0.05, size=num)
    return [
        dict(idx=i, t=float(t[i]), n=int(ns[i]), d=int(ds[i]), linkage=str(links[i]),
             k=int(ks[i]), sigma=float(sig[i]), seed=50_000 + i)
        for i in range(num)
    ]


def request_points(req: dict) -> np.ndarray:
    return blobs(req["n"], req["d"], req["k"], req["sigma"], req["seed"])
