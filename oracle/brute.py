"""Generic HAC by brute force, for tiny inputs (n up to a few dozen).

TEST INFRASTRUCTURE ONLY (see the package docstring).

At every step this evaluates the linkage distance of every pair of active
clusters straight from its definition and merges the pair with the smallest
key (distance, lower cluster ID, higher cluster ID); a cluster's ID is its
lowest point index. This is the "generic" algorithm the paper contrasts with
the nearest-neighbour chain (Sec. 2, Sec. 7); for reducible linkages and
inputs without ties both give the same dendrogram, which is what the chain
oracle is pinned against.

Ward's distance is taken here from the variance form of Table 1,
sqrt(2 (Var(A u B) - Var(A) - Var(B))) with Var(S) the sum of squared
deviations from the mean of S, so it shares no formula with the chain
oracle's closed form. Complete and average are the max and the mean of the
explicit pairwise distance matrix, avg-2 the mean of its squares.
"""
from __future__ import annotations

import numpy as np


def _var(P: np.ndarray) -> float:
    c = P.mean(axis=0)
    return float(((P - c) ** 2).sum())


def delta(x: np.ndarray, A, B, linkage: str) -> float:
    PA = x[np.asarray(A)].astype(np.float64)
    PB = x[np.asarray(B)].astype(np.float64)
    if linkage == "ward":
        v = 2.0 * (_var(np.vstack([PA, PB])) - _var(PA) - _var(PB))
        return float(np.sqrt(max(v, 0.0)))
    D2 = ((PA[:, None, :] - PB[None, :, :]) ** 2).sum(axis=2)
    if linkage == "avgsq":
        return float(D2.mean())
    D = np.sqrt(D2)
    if linkage == "complete":
        return float(D.max())
    if linkage == "average":
        return float(D.mean())
    raise ValueError(linkage)


def generic_hac(x: np.ndarray, linkage: str) -> np.ndarray:
    """Rows (node_a, node_b, height, size) in merge order, scipy node ids."""
    x = np.asarray(x)
    n = x.shape[0]
    clusters = {i: [i] for i in range(n)}  # ID -> members
    node = {i: i for i in range(n)}
    rows = []
    while len(clusters) > 1:
        ids = sorted(clusters)
        best = None
        for ia in range(len(ids)):
            for ib in range(ia + 1, len(ids)):
                a, b = ids[ia], ids[ib]
                key = (delta(x, clusters[a], clusters[b], linkage), a, b)
                if best is None or key < best:
                    best = key
        h, a, b = best
        na, nb = node[a], node[b]
        rows.append((min(na, nb), max(na, nb), h, len(clusters[a]) + len(clusters[b])))
        clusters[a] = clusters[a] + clusters.pop(b)
        node[a] = n + len(rows) - 1
        del node[b]
    return np.array(rows, dtype=np.float64).reshape(-1, 4)
