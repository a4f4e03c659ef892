"""GPU parity: libparchain (through its C ABI) against the FP64 oracle.

Pass criteria (on inputs the oracle certifies tie-free):
  * identical trees (same merges, as sets of children);
  * heights: complete and Ward are computed with the oracle's FP64 formulas
    (inputs widened exactly, no FMA contraction), so they must agree to the
    last bit; average sums point distances in another order, so 1e-12
    relative (the stated contract is 1e-5); avg-2 shares the centroid term
    bit for bit but carries each cluster's spread by another (equivalent)
    merge rule, whose rounding is bounded by a few ulps of |x| / separation
    per level, so 1e-10 relative;
  * rows in the documented canonical order.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import _trees

pytestmark = pytest.mark.gpu

LINKS = ["complete", "average", "ward", "avgsq"]
RTOL = {"complete": 0.0, "ward": 0.0, "average": 1e-12, "avgsq": 1e-10}


@pytest.fixture(scope="module")
def pc():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2106_04727_amd as pc

    pc.load_library()
    return pc


def run(pc, x, link, **kw):
    Z, st = pc.hac(x, link, return_stats=True, **kw)
    return Z, st


def check_parity(pc, x, link, tie_free=True, **kw):
    n = x.shape[0]
    Zo, cert = oracle.nnchain(x, link, threads=8)
    if tie_free:
        assert cert["min_gap"] >= 1e-10, "input not certified tie-free"
    Zg, st = run(pc, x, link, **kw)
    _trees.assert_valid(Zg, n)
    assert _trees.same_tree(Zg, Zo, n, rtol=RTOL[link]), (link, n, _trees.max_rel_height_err(Zg, Zo, n))
    C = oracle.canonical(Zo, n)
    if RTOL[link] == 0.0:
        assert np.array_equal(Zg, C)
    else:
        assert np.array_equal(Zg[:, [0, 1, 3]], C[:, [0, 1, 3]]) or _trees.same_tree(Zg, C, n, rtol=1e-12)
    return Zg, st, cert


def test_fig1_worked_example(pc):
    # six points shaped after the paper's worked example (Sec. 1, Fig. 1):
    # four rounds, (a,b) and (c,d) in round 1, e's tie resolved towards {a,b}
    x = np.array([[0.0, 3.0], [0.6, 2.2], [3.2, 0.2], [2.0, 0.0], [0.0, 0.0], [0.0, -3.0]], np.float32)
    # its round-2 tie is exact (the certificate is 0): the cluster-ID rule
    # decides it, in the oracle and on the GPU alike
    Zg, st, _ = check_parity(pc, x, "complete", tie_free=False)
    assert st["rounds"] == 4
    Zo, _ = oracle.nnchain(x, "complete")
    assert np.array_equal(Zg, oracle.canonical(Zo, 6))


@pytest.mark.parametrize("link", LINKS)
@pytest.mark.parametrize("n,d,kind,seed", [
    (2, 2, "u", 1), (3, 2, "u", 2), (64, 2, "u", 3), (257, 1, "u", 4), (1000, 2, "b", 5),
    (2000, 3, "u", 6), (3000, 10, "b", 7), (700, 16, "u", 8), (500, 40, "b", 9),
    (1500, 4, "u", 10), (2000, 64, "b", 11), (2500, 128, "s", 12), (800, 100, "s", 13),
    (400, 200, "b", 14),  # beyond the Gram search: full scan and generic tiles
    (3000, 6, "b", 15), (2500, 8, "u", 16),  # Ward / avg-2: box tree up to d = 8
])
def test_parity_small(pc, link, n, d, kind, seed):
    if kind == "u":
        x = synth.uniform(n, d, seed)
    elif kind == "b":
        x = synth.blobs(n, d, 8, 0.03, seed)
    else:
        x = synth.sphere_blobs(n, d, 25, 0.1, seed)
    _, cert = oracle.nnchain(x, link, threads=8)
    if cert["min_gap"] < 1e-10:
        pytest.skip("input not certified tie-free")
    check_parity(pc, x, link)


def test_parity_c1_complete_2k(pc):
    """n=2,000 uniform points in [0,1]^2, complete linkage, seeds 0-3."""
    for seed in range(4):
        x = synth.uniform(2000, 2, seed)
        check_parity(pc, x, "complete")


@pytest.mark.parametrize("link", LINKS)
def test_parity_blobs_20k(pc, link):
    """Gaussian-mixture data shaped like the 1M workload, at a size the oracle
    finishes in seconds; spans many grid rings, overflow scans and tiles."""
    n = 20_000 if link in ("ward", "avgsq") else 6_000
    x = synth.blobs(n, 2, 50, 0.01, 11)
    Zg, st, cert = check_parity(pc, x, link)
    assert st["rounds"] > 1


@pytest.mark.parametrize("link", LINKS)
def test_prune_on_equals_off(pc, link):
    x = synth.blobs(1500, 2, 6, 0.05, 21)
    Za = pc.hac(x, link, prune=True)
    Zb = pc.hac(x, link, prune=False)
    assert same_rows(Za, Zb, link)


@pytest.mark.parametrize("link", LINKS)
def test_deterministic(pc, link):
    x = synth.blobs(5000, 2, 20, 0.02, 22)
    Z1 = pc.hac(x, link)
    Z2 = pc.hac(x, link)
    assert np.array_equal(Z1, Z2)


def test_host_and_device_points_agree(pc):
    import ctypes

    from paper_2106_04727_amd import parchain

    x = synth.blobs(3000, 2, 5, 0.05, 23)
    Zd = pc.hac(x, "ward")
    ctx = parchain.Context(0)
    out = np.zeros((2999, 4), np.int64)
    ctx.hac(x.ctypes.data, 3000, 2, "ward", out.ctypes.data, points_on_device=False,
            out_on_device=False)
    assert np.array_equal(parchain.rows_to_Z(out), Zd)


def test_special_cases(pc):
    import torch

    for link in LINKS:
        Z = pc.hac(np.zeros((1, 3), np.float32), link)
        assert Z.shape == (0, 4)
        Z = pc.hac(np.array([[0, 0], [3, 4]], np.float32), link)
        assert Z.shape == (1, 4) and Z[0, 2] == (25.0 if link == "avgsq" else 5.0) and Z[0, 3] == 2
        x = synth.uniform(50, 2, 5)
        x[7] = x[3]
        Z = pc.hac(x, link)
        assert Z[0, 2] == 0.0 and {int(Z[0, 0]), int(Z[0, 1])} == {3, 7}
        _trees.assert_valid_hac(x, Z, link, rtol=1e-9)
        # all points identical: every height is 0
        x = np.ones((20, 2), np.float32)
        Z = pc.hac(x, link)
        assert np.all(Z[:, 2] == 0.0)
        _trees.assert_valid_hac(x, Z, link)
        # exact ties between different distances: points on an integer grid
        g = np.stack(np.meshgrid(np.arange(6), np.arange(5)), -1).reshape(-1, 2).astype(np.float32)
        Z = pc.hac(g, link)
        _trees.assert_valid_hac(g, Z, link, rtol=1e-9)


def test_nonfinite_rejected(pc):
    from paper_2106_04727_amd import PCError

    x = synth.uniform(100, 2, 1)
    x[5, 1] = np.nan
    with pytest.raises(PCError) as e:
        pc.hac(x, "ward")
    assert e.value.status == -2
    x[5, 1] = np.inf
    with pytest.raises(PCError):
        pc.hac(x, "complete")


@pytest.mark.parametrize("link", ["complete", "average"])
def test_overflow_paths(pc, link, monkeypatch):
    """Tiny candidate-record and pair-list capacities force the ring re-walk
    fallback and the pair-list regrow; results must not change."""
    x = synth.blobs(4000, 2, 12, 0.03, 31)
    Z0 = pc.hac(x, link)
    monkeypatch.setenv("PC_TEST_CAND_CAP", "16")
    Z1 = pc.hac(x, link)
    monkeypatch.setenv("PC_TEST_PAIR_CAP", "8")
    Z2 = pc.hac(x, link)
    assert same_rows(Z0, Z1, link) and same_rows(Z0, Z2, link)
    Zo, _ = oracle.nnchain(x, link, threads=8)
    assert _trees.same_tree(Z0, Zo, 4000, rtol=RTOL[link])


def same_rows(Za, Zb, link):
    """Identical rows; average-linkage heights may differ in the last bits
    when one run takes a value from cached parts (Lance-Williams, Sec. 5) and
    the other sums the point distances."""
    if link != "average":
        return np.array_equal(Za, Zb)
    return (np.array_equal(Za[:, [0, 1, 3]], Zb[:, [0, 1, 3]])
            and np.allclose(Za[:, 2], Zb[:, 2], rtol=1e-12, atol=0.0))


@pytest.mark.parametrize("link", ["complete", "average"])
def test_cache_on_equals_off(pc, link, monkeypatch):
    """The cluster-pair cache (Alg. 4, Sec. 5) only avoids recomputation: rows
    are the same with it off, on, and squeezed into a tiny table. Values are
    also combined from cached parts of merged clusters (Table 2 rules)."""
    x = synth.blobs(6000, 2, 20, 0.02, 41)
    Z0, s0 = pc.hac(x, link, cache_slots=0, return_stats=True)
    Z1, s1 = pc.hac(x, link, cache_slots=64, return_stats=True)
    assert s0["cache_hits"] == 0 and s1["cache_inserts"] > 0
    assert s1["cache_derived"] > 0
    assert same_rows(Z0, Z1, link)
    monkeypatch.setenv("PC_TEST_CACHE_CAP", "512")
    Z2 = pc.hac(x, link, cache_slots=64)
    assert same_rows(Z0, Z2, link)
    Zo, _ = oracle.nnchain(x, link, threads=8)
    assert _trees.same_tree(Z0, Zo, 6000, rtol=RTOL[link])


def test_cache_d10_average(pc):
    x = synth.blobs(3000, 10, 30, 0.02, 42)
    Z0 = pc.hac(x, "average", cache_slots=0)
    Z1, st = pc.hac(x, "average", cache_slots=64, return_stats=True)
    assert same_rows(Z0, Z1, "average") and st["cache_hits"] > 0


@pytest.mark.parametrize("link,d", [("complete", 12), ("complete", 64), ("average", 64)])
def test_cache_high_dim(pc, link, d):
    """Gram search (d >= 4): cached and combined values against none. Above
    d = 16 the interval tiles settle every larger complete-linkage value
    exactly, so no complete pair reaches the cache there; at d = 12 the
    exact pass, and with it the cache, still serves them."""
    x = synth.sphere_blobs(2000, d, 20, 0.1, 43)
    Z0 = pc.hac(x, link, cache_slots=0)
    Z1, st = pc.hac(x, link, cache_slots=64, return_stats=True)
    assert same_rows(Z0, Z1, link)
    if link == "average" or d <= 16:
        assert st["cache_derived"] > 0
    Zo, _ = oracle.nnchain(x, link, threads=8)
    assert _trees.same_tree(Z1, Zo, 2000, rtol=RTOL[link])


@pytest.mark.parametrize("link", LINKS)
def test_gram_record_overflow(pc, link, monkeypatch):
    """d >= 4 searches with MFMA Gram tiles; a tiny candidate record forces
    the regrow-and-redo path, which must not change the rows."""
    x = synth.blobs(3000, 10, 20, 0.03, 51)
    Z0 = pc.hac(x, link)
    monkeypatch.setenv("PC_TEST_CAND_CAP", "64")
    Z1 = pc.hac(x, link)
    assert same_rows(Z0, Z1, link)


@pytest.mark.parametrize("link", LINKS)
def test_gram_batches(pc, link, monkeypatch):
    """The Gram search takes terminals in batches (each with its own bounded
    candidate record and pair list); the batch size must not change the rows."""
    x = synth.sphere_blobs(2500, 64, 30, 0.1, 52)
    Z0 = pc.hac(x, link)
    monkeypatch.setenv("PC_TEST_GRAM_BATCH", "37")
    Z1 = pc.hac(x, link)
    monkeypatch.setenv("PC_TEST_CAND_CAP", "256")
    Z2 = pc.hac(x, link)
    assert same_rows(Z0, Z1, link) and same_rows(Z0, Z2, link)
    Zo, _ = oracle.nnchain(x, link, threads=8)
    assert _trees.same_tree(Z0, Zo, 2500, rtol=RTOL[link])


@pytest.mark.parametrize("link", ["complete", "average"])
@pytest.mark.parametrize("d", [40, 64, 128])
def test_interval_screening(pc, link, d):
    """Large candidate pairs (d >= 32) are first bracketed by FP16 MFMA point
    tiles with rigorous FP32 error terms; only pairs whose lower end reaches
    the bound are evaluated exactly. The rows must still match the oracle."""
    n = 2000
    x = synth.sphere_blobs(n, d, 12, 0.1, 60 + d)
    Zo, cert = oracle.nnchain(x, link, threads=8)
    if cert["min_gap"] < 1e-10:
        pytest.skip("input not certified tie-free")
    Zg, st = pc.hac(x, link, return_stats=True)
    assert st["kernels"]["block_search"]["visits"] > 0  # point pairs screened
    assert _trees.same_tree(Zg, Zo, n, rtol=RTOL[link])
    Z0 = pc.hac(x, link, cache_slots=0)
    assert same_rows(Zg, Z0, link)


def test_complete_tiles_settle_fallback(pc):
    """Complete linkage above d = 16 takes exact keys inside the interval
    tiles, only of the pairs whose upper bound reaches the candidate's lower
    bound. Groups of near-identical points put every cross pair inside the
    FP16 bracket, so a wavefront meets more qualifying pairs than it settles
    and the candidate must go to the exact FP64 tiles instead: the rows must
    still be the oracle's, bit for bit."""
    rng = np.random.default_rng(71)
    g, m, d = 6, 80, 64
    cen = rng.normal(0.0, 3.0, (g, d))
    x = (np.repeat(cen, m, axis=0) + rng.uniform(-1e-4, 1e-4, (g * m, d))).astype(np.float32)
    Zg, st, _ = check_parity(pc, x, "complete", timing=True)
    assert st["kernels"]["pair_tiles"]["launches"] > 0  # the settling pass and the exact tiles


def test_avgsq_hand_computed_instances(pc):
    """avg-2 heights worked out by hand from the double-sum definition (the
    oracle's own pin), now from the GPU path."""
    from tests.test_oracle import _avgsq_instances

    for inst in _avgsq_instances():
        x = np.array(inst["points"], np.float32).reshape(-1, inst["d"])
        n = x.shape[0]
        got = _trees.heights_by_merge(pc.hac(x, "avgsq"), n)
        for A, B, h in inst["merges"]:
            key = tuple(sorted([(min(A), len(A)), (min(B), len(B))]))
            assert got[key] == pytest.approx(h, rel=1e-15), (inst["name"], A, B)


@pytest.mark.parametrize("link", LINKS)
@pytest.mark.parametrize("d", [2, 3])
def test_ring_search_wave_equals_thread(pc, link, d, monkeypatch):
    """The ring search's first pass takes a thread per terminal or, in rounds
    with few active clusters, a wavefront per terminal: rows must be the same
    with the wavefront search never used, used in every grid round, and used
    with a one-cell budget that hands every terminal on to the block search."""
    x = synth.blobs(12000, d, 30, 0.02, 80 + d)
    monkeypatch.setenv("PC_TREE_MAX_DIM", "0")  # the grid also for Ward / avg-2 at d = 3
    monkeypatch.setenv("PC_WAVE_TERMS", "0")
    Z0 = pc.hac(x, link, cache_slots=0)
    monkeypatch.setenv("PC_WAVE_TERMS", "100000000")
    Z1 = pc.hac(x, link, cache_slots=0)
    monkeypatch.setenv("PC_CELL_BUDGET", "1")  # thread search
    monkeypatch.setenv("PC_WAVE_BUDGET", "1")  # wavefront search
    Z2, st = pc.hac(x, link, cache_slots=0, return_stats=True)
    assert st["overflow_queries"] > 0
    assert same_rows(Z0, Z1, link) and same_rows(Z0, Z2, link)
    Zo, _ = oracle.nnchain(x, link, threads=8)
    assert _trees.same_tree(Z1, Zo, 12000, rtol=RTOL[link])


@pytest.mark.parametrize("d", [2, 3, 5])
def test_avgsq_ring_handoff(pc, d, monkeypatch):
    """avg-2 on the centroid grid (the box tree switched off at d = 3, 5): a
    one-cell budget hands every terminal to the block ring search; rows must
    not change."""
    x = synth.blobs(8000, d, 40, 0.01, 70 + d)
    monkeypatch.setenv("PC_TREE_MAX_DIM", "0")
    Z0 = pc.hac(x, "avgsq")
    monkeypatch.setenv("PC_CELL_BUDGET", "1")
    Z1, st = pc.hac(x, "avgsq", return_stats=True)
    assert np.array_equal(Z0, Z1) and st["overflow_queries"] > 0
    Zo, _ = oracle.nnchain(x, "avgsq", threads=8)
    assert _trees.same_tree(Z0, Zo, 8000, rtol=RTOL["avgsq"])


def test_avgsq_gram_from_dim_four(pc, monkeypatch):
    """The Gram search serves avg-2 from d = 6 by default; forced down to
    d = 4 it must give the grid's rows."""
    x = synth.blobs(3000, 4, 25, 0.02, 75)
    Z0 = pc.hac(x, "avgsq")
    monkeypatch.setenv("PC_GRAM_MIN_DIM", "4")
    Z1 = pc.hac(x, "avgsq")
    assert np.array_equal(Z0, Z1)


@pytest.mark.parametrize("link", ["ward", "avgsq"])
@pytest.mark.parametrize("d,kind", [(3, "u"), (4, "b"), (5, "u"), (5, "b"), (8, "b")])
def test_box_tree_equals_other_searches(pc, link, d, kind, monkeypatch):
    """Ward / avg-2 at 3 <= d <= 8 search a box tree over Morton-ordered
    centroids in the rounds with many active clusters, the Gram search in the
    others; the grid (d <= 5), the Gram search and the full scan evaluate the
    same FP64 keys, so every mix must give identical rows, matching the
    oracle."""
    n = 6000
    x = synth.uniform(n, d, 80 + d) if kind == "u" else synth.blobs(n, d, 30, 0.02, 80 + d)
    monkeypatch.setenv("PC_TREE_MAX_DIM", "8")  # the default stops at d = 5
    monkeypatch.setenv("PC_TREE_GRAM_SWITCH", "0")  # the tree in every round
    Zt, st = pc.hac(x, link, return_stats=True)
    assert st["kernels"]["ring_search"]["visits"] > 0
    monkeypatch.setenv("PC_TREE_GRAM_SWITCH", "1500")  # tree, then Gram (d >= 4)
    assert np.array_equal(Zt, pc.hac(x, link))
    monkeypatch.delenv("PC_TREE_GRAM_SWITCH")
    monkeypatch.delenv("PC_TREE_MAX_DIM")
    assert np.array_equal(Zt, pc.hac(x, link))
    monkeypatch.setenv("PC_TREE_MAX_DIM", "0")
    Zo = pc.hac(x, link)  # grid up to d = 5, Gram search above
    assert np.array_equal(Zt, Zo)
    monkeypatch.setenv("PC_GRAM_MIN_DIM", "4")
    assert np.array_equal(Zt, pc.hac(x, link))
    assert np.array_equal(Zt, pc.hac(x, link, prune=False))
    Zr, cert = oracle.nnchain(x, link, threads=8)
    assert cert["min_gap"] >= 1e-10, "fixed input no longer certified tie-free"
    assert _trees.same_tree(Zt, Zr, n, rtol=RTOL[link])


@pytest.mark.parametrize("link", ["ward", "avgsq"])
@pytest.mark.parametrize("d", [3, 5])
def test_box_tree_edge_cases(pc, link, d, monkeypatch):
    """The box tree in every round on tiny inputs (one partial leaf, leaves
    across one level), duplicated points (zero keys, ties broken by cluster
    ID) and all-equal points; rows against the oracle."""
    monkeypatch.setenv("PC_TREE_GRAM_SWITCH", "0")
    for n in (2, 3, 17, 16 * 16 + 1, 700):
        x = synth.uniform(n, d, 90 + n)
        Zo, cert = oracle.nnchain(x, link)
        Z = pc.hac(x, link)
        _trees.assert_valid(Z, n)
        if cert["min_gap"] >= 1e-10:
            assert _trees.same_tree(Z, Zo, n, rtol=RTOL[link]), (n, d)
        else:
            # ties: any dendrogram of reciprocal-nearest merges is correct
            _trees.assert_valid_hac(x, Z, link, rtol=1e-9)
    x = synth.uniform(300, d, 99)
    x[150:] = x[:150]  # every point twice
    Z = pc.hac(x, link)
    _trees.assert_valid(Z, 300)
    _trees.assert_valid_hac(x, Z, link, rtol=1e-9)
    assert np.all(Z[:150, 2] == 0.0)
    assert {frozenset((int(a), int(b))) for a, b in Z[:150, :2]} == {frozenset((i, i + 150)) for i in range(150)}
    Z = pc.hac(np.ones((40, d), np.float32), link)
    assert np.all(Z[:, 2] == 0.0)


@pytest.mark.parametrize("d", [5, 8, 12])
def test_complete_giant_pairs_block_pruning(pc, d):
    """Two large blobs far apart (d <= 16): the last merges join clusters of
    thousands of points, whose interval tiles are pruned by block boxes; the
    rows must match the oracle exactly."""
    rng = np.random.default_rng(100 + d)
    a = rng.normal(0.0, 1.0, (2500, d))
    b = rng.normal(0.0, 1.0, (2000, d)) + 6.0
    x = np.vstack([a, b]).astype(np.float32)
    Zo, cert = oracle.nnchain(x, "complete", threads=8)
    Z, st = pc.hac(x, "complete", return_stats=True)
    assert st["kernels"]["block_search"]["visits"] > 0  # point pairs screened
    assert cert["min_gap"] >= 1e-10, "fixed input no longer certified tie-free"
    assert _trees.same_tree(Z, Zo, x.shape[0], rtol=0.0)
    C = oracle.canonical(Zo, x.shape[0])
    assert Z[-1, 2] == C[-1, 2]  # the farthest pair of the final merge, bit for bit


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
@pytest.mark.parametrize("link", LINKS)
@pytest.mark.parametrize("n,d,kind,seed", [(3000, 10, "b", 7), (2000, 64, "b", 11), (2500, 128, "s", 12)])
def test_precision_forms(pc, precision, link, n, d, kind, seed):
    """The screening tiles in BF16 or FP32 operands instead of FP16 (pc_precision):
    candidates they cannot rule out are refined in FP64 in every form, so the
    tree matches the oracle's and the rows equal the FP16 form's; only the
    number of refined candidates may differ."""
    if kind == "b":
        x = synth.blobs(n, d, 8, 0.03, seed)
    else:
        x = synth.sphere_blobs(n, d, 25, 0.1, seed)
    _, cert = oracle.nnchain(x, link, threads=8)
    assert cert["min_gap"] >= 1e-10, "fixed input no longer certified tie-free"
    Zg, st, _ = check_parity(pc, x, link, precision=precision)
    Z16, s16 = pc.hac(x, link, return_stats=True)
    assert same_rows(Zg, Z16, link)
    assert st["refined"] > 0 and s16["refined"] > 0
    assert 0 <= st["fp64_fallbacks"] <= st["refined"]


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
@pytest.mark.parametrize("link", ["complete", "average"])
def test_precision_forms_interval_tiles(pc, precision, link):
    """Large candidate pairs bracketed by point-pair tiles of each element type
    (d = 64), then refined exactly: the same rows as the FP16 form."""
    x = synth.sphere_blobs(2000, 64, 12, 0.1, 124)
    Z16 = pc.hac(x, link)
    Zp, st = pc.hac(x, link, precision=precision, return_stats=True)
    assert st["kernels"]["block_search"]["visits"] > 0  # point pairs screened
    assert same_rows(Zp, Z16, link)


def test_round_phase_times(pc):
    """With timing on, the rounds' device time is split into the search, the
    merges and the state update."""
    x = synth.blobs(20_000, 2, 50, 0.01, 11)
    _, st = pc.hac(x, "complete", return_stats=True, timing=True)
    assert st["ms_nn"] > 0 and st["ms_merge"] > 0 and st["ms_update"] > 0
    assert st["ms_nn"] + st["ms_merge"] + st["ms_update"] <= st["ms_rounds"] * 1.05


@pytest.mark.parametrize("link", LINKS)
@pytest.mark.parametrize("law", ["uniform_fill", "gaussian_disc"])
@pytest.mark.parametrize("d,n", [(2, 5000), (5, 3000)])
def test_parity_paper_laws(pc, link, law, d, n):
    """The paper's own synthetic laws (UniformFill, GaussianDisc; Sec. 6 data
    sets), drawn here at sizes the oracle finishes in seconds: every linkage
    on the 2-D grid and the 5-D search paths against the oracle."""
    x = getattr(synth, law)(n, d, 500 + d)
    check_parity(pc, x, link)


@pytest.mark.parametrize("link,d", [("ward", 2), ("avgsq", 2), ("complete", 2), ("average", 2),
                                    ("complete", 3), ("average", 3)])
def test_full_scan_rounds_equal_ring_search(pc, link, d, monkeypatch):
    """Rounds with few active clusters scan them all (a block per terminal)
    instead of walking grid rings; the rows do not depend on where that
    switch happens: never, the default, or from the second round on."""
    x = synth.blobs(20_000 if link in ("ward", "avgsq") else 6_000, d, 50, 0.01, 11 + d)
    monkeypatch.setenv("PC_FULL_SCAN_MAX", "0")
    Z0 = pc.hac(x, link)
    monkeypatch.delenv("PC_FULL_SCAN_MAX")
    Z1 = pc.hac(x, link)
    monkeypatch.setenv("PC_FULL_SCAN_MAX", "1000000000")
    Z2, st = pc.hac(x, link, return_stats=True)
    assert st["kernels"]["block_search"]["visits"] > 0  # the full scan ran
    assert same_rows(Z0, Z1, link) and same_rows(Z0, Z2, link)
