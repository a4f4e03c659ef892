"""Whole-tree digests of the FP64 oracle's dendrograms at full size.

TEST INFRASTRUCTURE. ``python tests/golden/digests.py [name ...]`` writes
``tests/golden/digest_<name>.txt``; it calls only ``oracle`` and ``synth``.
Each named input is clustered by the oracle in its accelerated mode (grid-
pruned queries, rows bit for bit those of the plain sequential chain), put in
the library's row convention (``oracle.canonical_fast``) and summarised as

* ``tree``    SHA-256 of the merge set: every merge's children as (lowest
              point index, size), sorted, int64 little-endian; independent of
              row order and heights, so two dendrograms are the same tree iff
              these digests agree;
* ``chunk``   SHA-256 of each block of CHUNK consecutive canonical rows, as
              float64 little-endian (a, b, height, size): equal chunks mean
              bit-identical rows (Ward and complete keys are exact, so the
              library's rows must match these);
* ``height``  a seeded sample of merges with their heights (repr of the
              double), for linkages whose heights are compared with a
              tolerance;
* the oracle's tie certificate (``min_gap`` is capped at 2^-23 in this mode).

The GPU tests recompute the same digests from the library's rows.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CHUNK = 1 << 16
HEIGHT_SAMPLES = 2000

# name -> (generator call as text, linkage)
CASES = {
    "blob50_1m_d2_ward": ("synth.blobs(1_000_000, 2, 50, 0.01, 11)", "ward"),
    "blob50_1m_d2_complete": ("synth.blobs(1_000_000, 2, 50, 0.01, 11)", "complete"),
    "blob50_1m_d2_avgsq": ("synth.blobs(1_000_000, 2, 50, 0.01, 11)", "avgsq"),
    "blob50_10m_d2_ward": ("synth.blobs(10_000_000, 2, 50, 0.01, 12)", "ward"),
}


def points(name):
    import synth

    return eval(CASES[name][0], {"synth": synth})


def tree_digest(keys: np.ndarray) -> str:
    k = np.ascontiguousarray(keys, dtype="<i8")
    order = np.lexsort((k[:, 3], k[:, 2], k[:, 1], k[:, 0]))
    return hashlib.sha256(np.ascontiguousarray(k[order]).tobytes()).hexdigest()


def chunk_digests(rows: np.ndarray) -> list:
    r = np.ascontiguousarray(rows, dtype="<f8")
    return [hashlib.sha256(r[i : i + CHUNK].tobytes()).hexdigest() for i in range(0, r.shape[0], CHUNK)]


def summarise(rows: np.ndarray, n: int):
    """tree digest, chunk digests and merge keys of canonical rows"""
    import oracle

    keys = oracle.merge_keys(rows, n)
    return tree_digest(keys), chunk_digests(rows), keys


def write(name: str) -> str:
    import oracle

    expr, link = CASES[name]
    x = points(name)
    n, d = x.shape
    t0 = time.perf_counter()
    Z, cert = oracle.nnchain(x, link, accel=True)
    secs = time.perf_counter() - t0
    rows = oracle.canonical_fast(Z, n)
    tree, chunks, keys = summarise(rows, n)
    rng = np.random.default_rng(1234)
    pick = np.sort(rng.choice(n - 1, size=min(HEIGHT_SAMPLES, n - 1), replace=False))
    path = os.path.join(HERE, "digest_%s.txt" % name)
    with open(path, "w") as f:
        f.write("# Whole-tree digest of the FP64 oracle (accelerated mode), written by\n")
        f.write("# tests/golden/digests.py; see its docstring for the format.\n")
        f.write("name %s\ninput %s\nn %d\nd %d\nlinkage %s\n" % (name, expr, n, d, link))
        f.write("min_gap %r\nzero_best %d\nqueries %d\n" % (float(cert["min_gap"]), cert["zero_best"],
                                                         cert["queries"]))
        f.write("oracle_seconds %.1f\nchunk_rows %d\n" % (secs, CHUNK))
        f.write("tree %s\n" % tree)
        for i, c in enumerate(chunks):
            f.write("chunk %d %s\n" % (i, c))
        for r in pick:
            k = keys[r]
            f.write("height %d %d %d %d %r\n" % (k[0], k[1], k[2], k[3], float(rows[r, 2])))
    print("%s: n=%d %s oracle %.1f s, min_gap %.3g, %d chunks" % (name, n, link, secs, cert["min_gap"],
                                                               len(chunks)), flush=True)
    return path


def read(name: str) -> dict:
    path = os.path.join(HERE, "digest_%s.txt" % name)
    out = {"chunks": [], "heights": {}}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split(None, 1)
            v = v.strip()
            if k == "chunk":
                i, h = v.split()
                assert int(i) == len(out["chunks"])
                out["chunks"].append(h)
            elif k == "height":
                a, sa, b, sb, h = v.split()
                out["heights"][(int(a), int(sa), int(b), int(sb))] = float(h)
            elif k in ("n", "d", "zero_best", "queries", "chunk_rows"):
                out[k] = int(v)
            elif k in ("min_gap", "oracle_seconds"):
                out[k] = float(v)
            else:
                out[k] = v
    return out


if __name__ == "__main__":
    for nm in sys.argv[1:] or list(CASES):
        write(nm)
