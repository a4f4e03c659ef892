"""Helpers that compare dendrograms as trees (no clustering arithmetic).

A cluster inside one dendrogram is identified by (lowest point index, size):
two different clusters of one dendrogram that share their lowest point are
nested, so their sizes differ. A merge is the unordered pair of its children's
identities; two dendrograms over the same points are the same tree iff their
merge sets are equal.
"""
import numpy as np


def merge_set(Z, n):
    Z = np.asarray(Z)
    m = Z.shape[0]
    lo = list(range(n)) + [0] * m
    sz = [1] * n + [0] * m
    out = []
    for r in range(m):
        a, b = int(Z[r, 0]), int(Z[r, 1])
        ka, kb = (lo[a], sz[a]), (lo[b], sz[b])
        out.append((min(ka, kb), max(ka, kb)))
        lo[n + r] = min(lo[a], lo[b])
        sz[n + r] = sz[a] + sz[b]
    return out


def heights_by_merge(Z, n):
    return dict(zip(merge_set(Z, n), np.asarray(Z)[:, 2].tolist()))


def assert_valid(Z, n):
    """scipy-style validity: each node used once, children created earlier,
    sizes add up."""
    Z = np.asarray(Z)
    assert Z.shape == (n - 1, 4)
    used = np.zeros(2 * n - 1, bool)
    size = np.ones(2 * n - 1, np.int64)
    for r in range(n - 1):
        a, b = int(Z[r, 0]), int(Z[r, 1])
        assert 0 <= a < n + r and 0 <= b < n + r and a != b, (r, a, b)
        assert not used[a] and not used[b], (r, a, b)
        used[a] = used[b] = True
        size[n + r] = size[a] + size[b]
        assert int(Z[r, 3]) == size[n + r], (r, Z[r, 3], size[n + r])
    assert n == 1 or not used[2 * n - 2]


def same_tree(Z1, Z2, n, rtol=0.0):
    m1, m2 = heights_by_merge(Z1, n), heights_by_merge(Z2, n)
    if set(m1) != set(m2):
        return False
    for k, h in m1.items():
        h2 = m2[k]
        if abs(h - h2) > rtol * max(abs(h), abs(h2)):
            return False
    return True


def max_rel_height_err(Z1, Z2, n):
    m1, m2 = heights_by_merge(Z1, n), heights_by_merge(Z2, n)
    err = 0.0
    for k, h in m1.items():
        h2 = m2[k]
        den = max(abs(h), abs(h2))
        if den > 0:
            err = max(err, abs(h - h2) / den)
    return err


def assert_valid_hac(x, Z, link, rtol=1e-12):
    """Validity of a dendrogram on inputs with ties (several dendrograms are
    then correct): in the row order given (a creation order), each merge's
    height is the linkage distance of its two children, and no cluster alive
    at that time is closer to either child than that height, i.e. the two
    were reciprocal nearest neighbours when they merged. Distances come from
    the oracle's definitions over explicit member sets (tiny inputs only)."""
    import oracle

    Z = np.asarray(Z)
    n = Z.shape[0] + 1
    assert_valid(Z, n)
    mem = {i: np.array([i], np.int64) for i in range(n)}
    alive = set(range(n))
    for r in range(n - 1):
        a, b, h = int(Z[r, 0]), int(Z[r, 1]), float(Z[r, 2])
        d_ab = oracle.linkage_dist(x, link, mem[a], mem[b])
        assert abs(d_ab - h) <= rtol * max(abs(h), abs(d_ab)), (r, h, d_ab)
        for c in alive:
            if c in (a, b):
                continue
            for v in (a, b):
                d = oracle.linkage_dist(x, link, mem[v], mem[c])
                assert d >= h * (1.0 - rtol), (r, v, c, d, h)
        alive -= {a, b}
        alive.add(n + r)
        mem[n + r] = np.concatenate([mem[a], mem[b]])
