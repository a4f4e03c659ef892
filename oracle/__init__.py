"""FP64 oracle for ParChain-style hierarchical agglomerative clustering.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this package to check and time the GPU library. The GPU
library never imports, loads or calls anything here, and this package imports
nothing from the library.

Contents
  * ``nnchain``       sequential nearest-neighbour chain in FP64 (C, ``nnchain.c``);
                      ``accel=True`` answers its queries through a centroid grid
                      with exact pruning (same rows, bit for bit)
  * ``linkage_dist``  linkage distance of two explicit member sets (Table 1)
  * ``canonical``     the dendrogram row convention (sorted rows, scipy ids);
                      ``canonical_fast`` is the same rule in C for large n
  * ``brute``         generic HAC by brute force, for tiny inputs (``brute.py``)

Linkage codes: 0 complete, 1 average (mean Euclidean, avg-1), 2 Ward,
3 avgsq (mean squared Euclidean, avg-2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nnchain.c")
_LIBDIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIBDIR, "liboracle.so")
_lock = threading.Lock()
_lib = None

LINKAGES = {"complete": 0, "average": 1, "ward": 2, "avgsq": 3}


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP). Returns the library path."""
    with _lock:
        if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            os.makedirs(_LIBDIR, exist_ok=True)
            tmp = _LIB + ".tmp%d" % os.getpid()
            subprocess.check_call(
                ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC, "-lm"]
            )
            os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.oracle_nnchain.restype = ctypes.c_int
        lib.oracle_nnchain.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            i64p, i64p, f64p, i64p, f64p,
        ]
        lib.oracle_nnchain_grid.restype = ctypes.c_int
        lib.oracle_nnchain_grid.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
            i64p, i64p, f64p, i64p, f64p,
        ]
        lib.oracle_canonical.restype = ctypes.c_int
        lib.oracle_canonical.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        lib.oracle_merge_keys.restype = ctypes.c_int
        lib.oracle_merge_keys.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        lib.oracle_tree_sums.restype = ctypes.c_int
        lib.oracle_tree_sums.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_linkage.restype = ctypes.c_double
        lib.oracle_linkage.argtypes = [
            ctypes.c_void_p, ctypes.c_int, ctypes.c_int, i64p, ctypes.c_int64, i64p, ctypes.c_int64,
        ]
        _lib = lib
    return _lib


def _code(linkage) -> int:
    return LINKAGES[linkage] if isinstance(linkage, str) else int(linkage)


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


# Accelerated mode reports min(plain mode's min_gap, GAP_CAP): candidates it
# skips exceed the best by more than that relative gap.
GAP_CAP = 2.0 ** -23


def nnchain(x: np.ndarray, linkage, threads: int = 0, accel: bool = False):
    """Sequential NN-chain HAC of float32 points ``x`` (n, d).

    Returns ``(Z, cert)``: ``Z`` is (n-1, 4) float64 rows in merge order
    ``[node_a, node_b, height, size]`` (leaves 0..n-1, merge k makes n+k);
    ``cert`` holds the tie certificate: ``min_gap`` (smallest relative gap
    between best and runner-up over all queries), ``zero_best``, ``queries``
    and ``pair_evals``.

    ``accel=True``: the same chain with grid-pruned queries (single thread);
    the rows are those of plain mode bit for bit, ``min_gap`` is
    ``min(plain min_gap, GAP_CAP)`` and ``pair_evals`` counts the point pairs
    actually evaluated (``cand_evals`` the candidate clusters examined).
    """
    x = np.ascontiguousarray(x, dtype=np.float32)
    n, d = x.shape
    m = max(n - 1, 1)
    a = np.zeros(m, np.int64)
    b = np.zeros(m, np.int64)
    h = np.zeros(m, np.float64)
    s = np.zeros(m, np.int64)
    cert = np.zeros(6, np.float64)
    ptrs = (_ptr(a, ctypes.c_int64), _ptr(b, ctypes.c_int64), _ptr(h, ctypes.c_double),
            _ptr(s, ctypes.c_int64), _ptr(cert, ctypes.c_double))
    if accel:
        rc = _load().oracle_nnchain_grid(x.ctypes.data, n, d, _code(linkage), *ptrs)
    else:
        rc = _load().oracle_nnchain(x.ctypes.data, n, d, _code(linkage), int(threads), *ptrs)
    if rc != 0:
        raise ValueError("oracle_nnchain failed with code %d" % rc)
    Z = np.stack([a, b, h, s], axis=1).astype(np.float64)[: n - 1]
    out = dict(min_gap=cert[0], zero_best=int(cert[1]), queries=int(cert[2]), pair_evals=int(cert[3]))
    if accel:
        out.update(cand_evals=int(cert[4]), grid_rebuilds=int(cert[5]))
    return Z, out


def linkage_dist(x: np.ndarray, linkage, A, B) -> float:
    """Linkage distance between member index sets ``A`` and ``B`` (Table 1)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    A = np.ascontiguousarray(A, dtype=np.int64)
    B = np.ascontiguousarray(B, dtype=np.int64)
    return float(_load().oracle_linkage(
        x.ctypes.data, x.shape[1], _code(linkage), _ptr(A, ctypes.c_int64), A.size,
        _ptr(B, ctypes.c_int64), B.size))


def tree_sums(x: np.ndarray, Z: np.ndarray):
    """FP64 coordinate sums and sizes of all 2n-1 nodes of dendrogram Z."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    n, d = x.shape
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    sums = np.zeros((2 * n - 1, d), np.float64)
    sizes = np.zeros(2 * n - 1, np.int64)
    rc = _load().oracle_tree_sums(x.ctypes.data, n, d, Z.ctypes.data, sums.ctypes.data, sizes.ctypes.data)
    if rc != 0:
        raise ValueError("rows are not a valid creation order")
    return sums, sizes


def node_members(Z: np.ndarray, n: int, node: int) -> np.ndarray:
    """Point indices under one node (iterative walk)."""
    out, stack = [], [int(node)]
    while stack:
        v = stack.pop()
        if v < n:
            out.append(v)
        else:
            r = v - n
            stack.append(int(Z[r, 0]))
            stack.append(int(Z[r, 1]))
    return np.array(sorted(out), np.int64)


def members(Z: np.ndarray, n: int):
    """Member lists of every node of a dendrogram in scipy convention."""
    mem = [[i] for i in range(n)] + [None] * (n - 1)
    for r in range(n - 1):
        a, b = int(Z[r, 0]), int(Z[r, 1])
        mem[n + r] = mem[a] + mem[b]
    return mem


def canonical_fast(Z: np.ndarray, n: int) -> np.ndarray:
    """``canonical`` for large row counts (C; the same rule, tested equal)."""
    m = n - 1
    if m <= 0:
        return np.zeros((0, 4), np.float64)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    out = np.zeros((m, 4), np.float64)
    rc = _load().oracle_canonical(Z.ctypes.data, n, out.ctypes.data)
    if rc != 0:
        raise ValueError("rows are not a valid creation order (%d)" % rc)
    return out


def merge_keys(Z: np.ndarray, n: int) -> np.ndarray:
    """Every merge of dendrogram ``Z`` as int64 (lo_a, size_a, lo_b, size_b):
    its children identified by lowest point index and size (smaller pair
    first), rows in the order of ``Z``."""
    m = n - 1
    if m <= 0:
        return np.zeros((0, 4), np.int64)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    out = np.zeros((m, 4), np.int64)
    rc = _load().oracle_merge_keys(Z.ctypes.data, n, out.ctypes.data)
    if rc != 0:
        raise ValueError("rows are not a valid creation order (%d)" % rc)
    return out


def canonical(Z: np.ndarray, n: int) -> np.ndarray:
    """Rows sorted by (height, size, lowest point index of the new cluster).

    "height" here is the largest height in the row's subtree, which equals the
    row's own height whenever the dendrogram is monotone (reducible linkages
    in exact arithmetic); it keeps the order a valid creation order even if
    rounding makes a parent a hair lower than a child.

    Children are relabelled so that row r creates node n+r (scipy's
    convention) and every row has a < b. A parent always has a larger size
    than its children, so the order is also a valid creation order when
    heights tie.
    """
    m = n - 1
    if m <= 0:
        return np.zeros((0, 4), np.float64)
    lo = np.arange(n, dtype=np.int64).tolist() + [0] * m
    eff = [0.0] * n + [0.0] * m
    for r in range(m):
        a, b = int(Z[r, 0]), int(Z[r, 1])
        lo[n + r] = min(lo[a], lo[b])
        eff[n + r] = max(float(Z[r, 2]), eff[a], eff[b])
    key = [(eff[n + r], int(Z[r, 3]), lo[n + r]) for r in range(m)]
    order = sorted(range(m), key=lambda r: key[r])
    newid = list(range(n)) + [0] * m
    for pos, r in enumerate(order):
        newid[n + r] = n + pos
    out = np.zeros((m, 4), np.float64)
    for pos, r in enumerate(order):
        a, b = newid[int(Z[r, 0])], newid[int(Z[r, 1])]
        out[pos] = (min(a, b), max(a, b), Z[r, 2], Z[r, 3])
    return out
