"""Pins for the oracle's accelerated mode and its helpers.

* accelerated mode (grid-pruned queries) gives plain mode's rows bit for
  bit, the same query count and zero-distance count, and plain mode's tie
  certificate capped at ``oracle.GAP_CAP``, on every linkage, on uniform and
  clustered inputs, in one to ten dimensions, with duplicated points;
* ``tree_sums`` on a hand-built three-leaf tree;
* the tie certificate (``min_gap``) on inputs whose every query is worked
  out by hand, including an exact tie;
* ``canonical_fast`` is ``canonical``; ``merge_keys`` identifies the same
  merges as the tree helpers;
* the validity check used for inputs with ties accepts the oracle's own
  dendrograms and rejects a dendrogram with a wrong merge.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import _trees

LINKS = ["complete", "average", "ward", "avgsq"]


def _accel_matches_plain(x, link):
    Zp, cp = oracle.nnchain(x, link, threads=8)
    Za, ca = oracle.nnchain(x, link, accel=True)
    assert np.array_equal(Zp, Za), link
    assert ca["queries"] == cp["queries"] and ca["zero_best"] == cp["zero_best"]
    # with fewer than three clusters no query has a runner-up: both report 1
    want = cp["min_gap"] if x.shape[0] <= 2 else min(cp["min_gap"], oracle.GAP_CAP)
    assert ca["min_gap"] == want


@pytest.mark.parametrize("link", LINKS)
@pytest.mark.parametrize("n,d,kind,seed", [
    (2, 2, "u", 1), (3, 1, "u", 2), (500, 1, "u", 3), (2000, 2, "u", 4), (3000, 2, "b", 5),
    (1500, 3, "b", 6), (800, 5, "u", 7), (600, 10, "b", 8), (1000, 2, "g", 9), (700, 4, "f", 10),
])
def test_accel_equals_plain(link, n, d, kind, seed):
    if kind == "u":
        x = synth.uniform(n, d, seed)
    elif kind == "b":
        x = synth.blobs(n, d, 20, 0.02, seed)
    elif kind == "g":
        x = synth.gaussian_disc(n, d, seed)
    else:
        x = synth.uniform_fill(n, d, seed)
    _accel_matches_plain(x, link)


@pytest.mark.parametrize("link", LINKS)
def test_accel_equals_plain_with_ties(link):
    x = synth.blobs(1200, 2, 10, 0.02, 31)
    x[600:700] = x[:100]        # duplicated points: zero distances, cluster-ID ties
    x[900:] = np.float32(0.5)   # a block of identical points
    _accel_matches_plain(x, link)


@pytest.mark.parametrize("link", ["ward", "avgsq"])
def test_accel_equals_plain_20k(link):
    """The 50-Gaussian law of the 1M workload at 20,000 points (grid rebuilds,
    many rings, the two-level blocks)."""
    _accel_matches_plain(synth.blobs(20_000, 2, 50, 0.01, 11), link)


@pytest.mark.parametrize("link", ["complete", "average"])
def test_accel_equals_plain_5k(link):
    _accel_matches_plain(synth.blobs(5_000, 2, 50, 0.01, 11), link)


def test_tree_sums_hand_built():
    # leaves (1,2), (3,5), (10,-1); row 0 joins leaves 0 and 1 (node 3), row 1
    # joins leaf 2 with node 3 (node 4)
    x = np.array([[1, 2], [3, 5], [10, -1]], np.float32)
    Z = np.array([[0, 1, 1.0, 2], [2, 3, 2.0, 3]], np.float64)
    sums, sizes = oracle.tree_sums(x, Z)
    assert sizes.tolist() == [1, 1, 1, 2, 3]
    assert sums.tolist() == [[1, 2], [3, 5], [10, -1], [4, 7], [14, 6]]
    with pytest.raises(ValueError):
        oracle.tree_sums(x, np.array([[0, 4, 1.0, 2], [2, 3, 2.0, 3]], np.float64))


def test_min_gap_hand_worked():
    # points 0, 1, 3, 7 on a line, complete linkage; the chain's queries:
    #   from {0}:   1 (1),   3 (3), 7 (7)  gap (3-1)/3 = 2/3, push {1}
    #   from {1}:   0 (1),   3 (2), 7 (6)  gap (2-1)/2 = 1/2, merge {0,1} at 1
    #   from {0,1}: 3 (3),   7 (7)         gap 4/7,           push {3}
    #   from {3}:   {0,1} (3), 7 (4)       gap 1/4,           merge at 3
    #   from {0,1,3}: 7 (7) only, push {7}; from {7}: the rest only, merge at 7
    x = np.array([[0], [1], [3], [7]], np.float32)
    Z, cert = oracle.nnchain(x, "complete")
    assert cert["min_gap"] == 0.25 and cert["queries"] == 6 and cert["zero_best"] == 0
    assert Z[:, 2].tolist() == [1.0, 3.0, 7.0]
    _, ca = oracle.nnchain(x, "complete", accel=True)
    assert ca["min_gap"] == min(0.25, oracle.GAP_CAP) and ca["queries"] == 6
    # 0, 1, 2: the query from {1} sees 0 and 2 at the same distance (an exact
    # tie, decided by the lower cluster ID), so the certificate is 0
    x = np.array([[0], [1], [2]], np.float32)
    Z, cert = oracle.nnchain(x, "complete")
    assert cert["min_gap"] == 0.0
    assert Z[0, :2].tolist() == [0.0, 1.0]
    # a duplicated point: its query's best distance is exactly 0
    x = np.array([[0], [5], [0.5], [5]], np.float32)
    _, cert = oracle.nnchain(x, "ward")
    assert cert["zero_best"] >= 1


@pytest.mark.parametrize("link", LINKS)
def test_canonical_fast_equals_canonical(link):
    for seed in range(3):
        x = synth.blobs(1500, 2, 15, 0.02, 40 + seed)
        if seed == 2:
            x[10] = x[20]
            x[30:40] = x[50:60]
        Z, _ = oracle.nnchain(x, link)
        assert np.array_equal(oracle.canonical(Z, 1500), oracle.canonical_fast(Z, 1500))


def test_merge_keys_match_tree_helper():
    x = synth.blobs(800, 3, 10, 0.05, 44)
    Z, _ = oracle.nnchain(x, "average")
    k = oracle.merge_keys(Z, 800)
    ref = _trees.merge_set(Z, 800)
    assert [((a, b), (c, d)) for a, b, c, d in k.tolist()] == ref


@pytest.mark.parametrize("link", LINKS)
def test_validity_check_on_ties(link):
    x = synth.uniform(40, 2, 45)
    x[20:30] = x[:10]
    Z, _ = oracle.nnchain(x, link)
    _trees.assert_valid_hac(x, oracle.canonical(Z, 40), link)
    # the same rows with one merge's height raised are rejected
    C = oracle.canonical(Z, 40)
    C[-1, 2] *= 1.5
    with pytest.raises(AssertionError):
        _trees.assert_valid_hac(x, C, link)
