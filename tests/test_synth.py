"""The seeded generators (shared by the oracle tests and the GPU tests):
determinism, no duplicate rows, and the laws of the paper's synthetic sets
(Sec. 6: UniformFill in a hypergrid of side sqrt(n); GaussianDisc in one of
side 5 sqrt(n) with 90% of the points in five Gaussians)."""
import numpy as np

import synth


def test_deterministic_and_duplicate_free():
    for f in (lambda s: synth.uniform(5000, 3, s), lambda s: synth.blobs(5000, 2, 7, 0.01, s),
              lambda s: synth.uniform_fill(5000, 2, s), lambda s: synth.gaussian_disc(5000, 5, s)):
        a, b = f(3), f(3)
        assert a.dtype == np.float32 and np.array_equal(a, b)
        assert synth.dedup_rows(a).size == 0
        assert not np.array_equal(a, f(4))


def test_uniform_fill_law():
    n = 40_000
    x = synth.uniform_fill(n, 2, 1).astype(np.float64)
    side = np.sqrt(n)
    assert x.min() >= 0.0 and x.max() <= side
    # each quarter of the square holds about a quarter of the points
    q = ((x[:, 0] < side / 2).astype(int) + 2 * (x[:, 1] < side / 2)).astype(int)
    assert np.all(np.abs(np.bincount(q, minlength=4) / n - 0.25) < 0.02)


def test_gaussian_disc_law():
    n = 60_000
    x = synth.gaussian_disc(n, 2, 2).astype(np.float64)
    side = 5 * np.sqrt(n)
    sigma = np.sqrt(n) / 6
    # points far (> 5 sigma) from every dense centre are the uniform 10%; the
    # centres are found as the five densest cells of a coarse histogram
    h, ex, ey = np.histogram2d(x[:, 0], x[:, 1], bins=50, range=[[-side, 2 * side], [-side, 2 * side]])
    idx = np.argsort(h.ravel())[::-1][:5]
    cx = (ex[idx // 50] + ex[idx // 50 + 1]) / 2
    cy = (ey[idx % 50] + ey[idx % 50 + 1]) / 2
    d = np.sqrt((x[:, :1] - cx[None]) ** 2 + (x[:, 1:] - cy[None]) ** 2).min(1)
    far = (d > 5 * sigma).mean()
    assert 0.05 < far < 0.11
    inside = (x >= 0).all(1) & (x <= side).all(1)
    assert inside[d > 5 * sigma].mean() > 0.99
