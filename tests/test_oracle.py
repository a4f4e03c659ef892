"""Pins for the FP64 oracle: it is checked against things other than itself.

* brute-force generic HAC (a different algorithm, a different Ward formula,
  avg-2 from its double-sum definition);
* scipy's ``linkage`` (a library routine with the same height conventions;
  avg-2 is its average method over squared Euclidean distances);
* hand-computed values of a six-point instance shaped after the paper's
  worked example (Sec. 1, Fig. 1), and of two small avg-2 instances;
* closed forms: two far-apart blobs, n = 2, duplicates, collinear points;
* the Lance-Williams recurrences of Table 2 (Ward on squared distances);
* reducibility (Sec. 2.1): heights never decrease from child to parent;
* invariance under relabelling and exact translation.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import brute
from tests import _trees

LINKS = ["complete", "average", "ward", "avgsq"]


def _tie_free(x, link):
    _, cert = oracle.nnchain(x, link)
    return cert["min_gap"] > 1e-9 and cert["zero_best"] == 0


@pytest.mark.parametrize("link", LINKS)
@pytest.mark.parametrize("d", [1, 2, 3, 10])
def test_nnchain_equals_generic_hac(link, d):
    checked = 0
    for seed in range(40):
        n = 3 + seed % 23
        x = synth.uniform(n, d, 1000 * d + seed)
        if not _tie_free(x, link):
            continue
        Z, _ = oracle.nnchain(x, link)
        B = brute.generic_hac(x, link)
        _trees.assert_valid(Z, n)
        assert _trees.same_tree(Z, B, n, rtol=1e-9), (link, d, seed)
        checked += 1
    assert checked >= 30


@pytest.mark.parametrize("link", LINKS)
def test_nnchain_generic_hac_blobs(link):
    # clustered data: many merges of multi-point clusters
    for seed in range(6):
        x = synth.blobs(30, 2, 4, 0.05, 77 + seed)
        if not _tie_free(x, link):
            continue
        Z, _ = oracle.nnchain(x, link)
        assert _trees.same_tree(Z, brute.generic_hac(x, link), 30, rtol=1e-9)


@pytest.mark.parametrize("link", LINKS)
@pytest.mark.parametrize("n,d,seed", [(300, 2, 1), (1000, 3, 2), (2000, 2, 0), (500, 10, 3)])
def test_nnchain_matches_scipy(link, n, d, seed):
    from scipy.cluster.hierarchy import linkage

    from scipy.spatial.distance import pdist

    x = synth.uniform(n, d, seed)
    Z, cert = oracle.nnchain(x, link, threads=4)
    assert cert["min_gap"] > 1e-12
    if link == "avgsq":
        S = linkage(pdist(x.astype(np.float64), "sqeuclidean"), method="average")
    else:
        S = linkage(x.astype(np.float64), method=link)
    assert _trees.same_tree(Z, S, n, rtol=1e-9)
    _trees.assert_valid(oracle.canonical(Z, n), n)


def _fixture():
    pts, merges, sec = [], [], None
    with open(__file__.replace("test_oracle.py", "golden/fig1_complete.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line in ("points", "merges"):
                sec = line
                continue
            if sec == "points":
                i, name, a, b = line.split()
                pts.append((name, float(a), float(b)))
            else:
                ca, cb, h, r = [t.strip() for t in line.split("|")]
                merges.append((ca.split(","), cb.split(","), h, int(r)))
    return pts, merges


def test_fig1_worked_example_values():
    pts, merges = _fixture()
    names = [p[0] for p in pts]
    x = np.array([[p[1], p[2]] for p in pts], np.float32)
    Z, _ = oracle.nnchain(x, "complete")
    got = _trees.heights_by_merge(Z, 6)
    for ca, cb, h, _ in merges:
        A = sorted(names.index(c) for c in ca)
        B = sorted(names.index(c) for c in cb)
        key = tuple(sorted([(A[0], len(A)), (B[0], len(B))]))
        want = eval(h, {"sqrt": math.sqrt})
        # points are float32 roundings of the decimal coordinates
        assert key in got and got[key] == pytest.approx(want, rel=1e-6), (ca, cb)


def test_special_cases():
    x1 = np.zeros((1, 3), np.float32)
    Z, _ = oracle.nnchain(x1, "ward")
    assert Z.shape == (0, 4)
    x2 = np.array([[0, 0], [3, 4]], np.float32)
    for link in LINKS:
        Z, _ = oracle.nnchain(x2, link)
        assert Z.shape == (1, 4) and Z[0, 2] == (25.0 if link == "avgsq" else 5.0) and Z[0, 3] == 2
    # a duplicated point merges first, at height 0
    x = synth.uniform(20, 2, 5)
    x[7] = x[3]
    for link in LINKS:
        Z, cert = oracle.nnchain(x, link)
        C = oracle.canonical(Z, 20)
        assert C[0, 2] == 0.0 and {int(C[0, 0]), int(C[0, 1])} == {3, 7}
        assert cert["zero_best"] >= 1
    # collinear points along a line in 3-D == the same points on a line in 1-D
    t = np.sort(synth.uniform(40, 1, 9)[:, 0])
    x3 = np.stack([t, np.zeros_like(t), np.zeros_like(t)], 1).astype(np.float32)
    for link in LINKS:
        Z3, _ = oracle.nnchain(x3, link)
        Z1, _ = oracle.nnchain(t[:, None].astype(np.float32), link)
        assert _trees.same_tree(Z3, Z1, 40, rtol=0.0)


@pytest.mark.parametrize("link", LINKS)
def test_two_far_blobs_closed_form(link):
    rng = np.random.default_rng(3)
    A = rng.normal(0.0, 0.01, (40, 2))
    B = rng.normal(0.0, 0.01, (25, 2)) + np.array([10.0, 3.0])
    x = np.vstack([A, B]).astype(np.float32)
    Z, _ = oracle.nnchain(x, link)
    C = oracle.canonical(Z, 65)
    P, Q = x[:40].astype(np.float64), x[40:].astype(np.float64)
    D = np.sqrt(((P[:, None] - Q[None]) ** 2).sum(-1))
    want = {
        "complete": D.max(),
        "average": D.mean(),
        "avgsq": (D * D).mean(),
        "ward": math.sqrt(2 * 40 * 25 / 65) * np.linalg.norm(P.mean(0) - Q.mean(0)),
    }[link]
    assert C[-1, 2] == pytest.approx(want, rel=1e-12)
    assert C[-1, 3] == 65


def test_ward_closed_form_equals_variance_form():
    rng = np.random.default_rng(7)
    x = rng.random((200, 5)).astype(np.float32)
    for _ in range(50):
        p = rng.permutation(200)
        a, b = rng.integers(1, 40, 2)
        A, B = p[:a], p[a : a + b]
        assert oracle.linkage_dist(x, "ward", A, B) == pytest.approx(
            brute.delta(x, A, B, "ward"), rel=1e-9)
        for link in ("complete", "average", "avgsq"):
            assert oracle.linkage_dist(x, link, A, B) == pytest.approx(
                brute.delta(x, A, B, link), rel=1e-12)


def test_lance_williams_recurrences():
    """Table 2 coefficients; for Ward they apply to squared distances."""
    rng = np.random.default_rng(8)
    x = rng.random((300, 3)).astype(np.float32)
    for _ in range(40):
        p = rng.permutation(300)
        a, b, c = rng.integers(1, 30, 3)
        A, B, C = p[:a], p[a : a + b], p[a + b : a + b + c]
        AB = np.concatenate([A, B])
        D = {k: (oracle.linkage_dist(x, k, AB, C), oracle.linkage_dist(x, k, A, C),
                 oracle.linkage_dist(x, k, B, C), oracle.linkage_dist(x, k, A, B)) for k in LINKS}
        dabc, dac, dbc, dab = D["complete"]
        assert dabc == pytest.approx(0.5 * dac + 0.5 * dbc + 0.5 * abs(dac - dbc), rel=1e-12)
        for k in ("average", "avgsq"):
            dabc, dac, dbc, dab = D[k]
            assert dabc == pytest.approx((a * dac + b * dbc) / (a + b), rel=1e-10)
        dabc, dac, dbc, dab = D["ward"]
        s = a + b + c
        lw = ((a + c) * dac**2 + (b + c) * dbc**2 - c * dab**2) / s
        assert dabc**2 == pytest.approx(lw, rel=1e-9)


def test_cache_update_rules_two_sides_merged():
    """Sec. 5 update rules when both clusters of a pair were just merged
    (A u B against C u D): the average is the size-weighted mean of the four
    cross values, the complete distance the largest of them."""
    rng = np.random.default_rng(9)
    x = rng.random((400, 4)).astype(np.float32)
    for _ in range(30):
        p = rng.permutation(400)
        a, b, c, e = rng.integers(1, 25, 4)
        A, B = p[:a], p[a : a + b]
        C, D = p[a + b : a + b + c], p[a + b + c : a + b + c + e]
        AB, CD = np.concatenate([A, B]), np.concatenate([C, D])
        parts = [(X, Y) for X in (A, B) for Y in (C, D)]
        avg = sum(len(X) * len(Y) * oracle.linkage_dist(x, "average", X, Y) for X, Y in parts)
        avg /= len(AB) * len(CD)
        assert oracle.linkage_dist(x, "average", AB, CD) == pytest.approx(avg, rel=1e-12)
        comp = max(oracle.linkage_dist(x, "complete", X, Y) for X, Y in parts)
        assert oracle.linkage_dist(x, "complete", AB, CD) == comp


@pytest.mark.parametrize("link", LINKS)
def test_reducibility_monotone_heights(link):
    x = synth.blobs(3000, 2, 10, 0.02, 4)
    Z, _ = oracle.nnchain(x, link, threads=8)
    n = 3000
    h = np.zeros(2 * n - 1)
    for r in range(n - 1):
        a, b = int(Z[r, 0]), int(Z[r, 1])
        assert Z[r, 2] >= h[a] and Z[r, 2] >= h[b]
        h[n + r] = Z[r, 2]


@pytest.mark.parametrize("link", LINKS)
def test_relabel_and_translation_invariance(link):
    # coordinates on a 2^-12 lattice plus an integer shift stay exact in float32
    rng = np.random.default_rng(12)
    x = (rng.integers(0, 4096, (150, 2)) / 4096.0).astype(np.float32)
    x = x[np.unique(x, axis=0, return_index=True)[1]]
    n = x.shape[0]
    if not _tie_free(x, link):
        pytest.skip("lattice draw has a tie")
    Z, _ = oracle.nnchain(x, link)
    p = rng.permutation(n)
    Zp, _ = oracle.nnchain(x[p], link)
    # map permuted leaf labels back, then compare trees by member sets
    mem = oracle.members(Zp, n)
    mem0 = oracle.members(Z, n)
    S = {frozenset(int(p[i]) for i in m): None for m in mem[n:]}
    S0 = {frozenset(m): None for m in mem0[n:]}
    assert set(S) == set(S0)
    Zt, _ = oracle.nnchain(x + np.float32(8.0), link)
    assert _trees.same_tree(Z, Zt, n, rtol=1e-12 if link in ("complete", "ward") else 1e-10)


def test_canonical_row_convention():
    x = synth.uniform(500, 2, 13)
    Z, _ = oracle.nnchain(x, "average")
    C = oracle.canonical(Z, 500)
    _trees.assert_valid(C, 500)
    assert np.all(np.diff(C[:, 2]) >= 0)
    assert np.all(C[:, 0] < C[:, 1])
    assert _trees.same_tree(Z, C, 500)


def test_thread_count_does_not_change_result():
    x = synth.blobs(2000, 3, 8, 0.03, 14)
    for link in LINKS:
        Z1, _ = oracle.nnchain(x, link, threads=1)
        Z8, _ = oracle.nnchain(x, link, threads=8)
        assert np.array_equal(Z1, Z8)


def test_spread_identities_used_by_bounds():
    """Table 1's avg-2 row: mean over pairs of |x-y|^2 equals
    |cA-cB|^2 + Var(A)/|A| + Var(B)/|B| (Var = sum of squared deviations);
    and Var(A u B) = Var(A) + Var(B) + |A||B|/(|A|+|B|) |cA-cB|^2 (the merge
    rule of Sec. 2.1 read with its size factor). Complete linkage is at least
    the root of the first quantity, average linkage at most (Jensen)."""
    rng = np.random.default_rng(17)
    x = rng.normal(size=(400, 7)).astype(np.float32)
    for _ in range(30):
        p = rng.permutation(400)
        a, b = rng.integers(1, 60, 2)
        A, B = x[p[:a]].astype(np.float64), x[p[a : a + b]].astype(np.float64)
        D2 = ((A[:, None] - B[None]) ** 2).sum(-1)
        ca, cb = A.mean(0), B.mean(0)
        va, vb = ((A - ca) ** 2).sum(), ((B - cb) ** 2).sum()
        closed = ((ca - cb) ** 2).sum() + va / a + vb / b
        assert D2.mean() == pytest.approx(closed, rel=1e-12)
        U = np.vstack([A, B])
        vu = ((U - U.mean(0)) ** 2).sum()
        assert vu == pytest.approx(va + vb + a * b / (a + b) * ((ca - cb) ** 2).sum(), rel=1e-12)
        comp = oracle.linkage_dist(x, "complete", p[:a], p[a : a + b])
        avg = oracle.linkage_dist(x, "average", p[:a], p[a : a + b])
        assert comp * comp >= closed * (1 - 1e-12)
        assert avg <= np.sqrt(closed) * (1 + 1e-12)


def _avgsq_instances():
    out, cur = [], None
    with open(__file__.replace("test_oracle.py", "golden/avgsq_hand.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            kind, rest = line.split(None, 1)
            if kind == "instance":
                name, d = rest.split()
                cur = {"name": name, "d": int(d), "points": [], "merges": []}
                out.append(cur)
            elif kind == "point":
                cur["points"].append([float(v) for v in rest.split()])
            else:
                a, b, h = [t.strip() for t in rest.split("|")]
                num, _, den = h.partition("/")
                cur["merges"].append(([int(v) for v in a.split(",")], [int(v) for v in b.split(",")],
                                      float(num) / float(den or 1)))
    return out


def test_avgsq_hand_computed_instances():
    """avg-2 merge heights worked out by hand from the double-sum definition."""
    insts = _avgsq_instances()
    assert [i["name"] for i in insts] == ["line", "plane"]
    for inst in insts:
        x = np.array(inst["points"], np.float32).reshape(-1, inst["d"])
        n = x.shape[0]
        Z, _ = oracle.nnchain(x, "avgsq")
        got = _trees.heights_by_merge(Z, n)
        assert len(got) == len(inst["merges"]) == n - 1
        for A, B, h in inst["merges"]:
            key = tuple(sorted([(min(A), len(A)), (min(B), len(B))]))
            assert key in got and got[key] == pytest.approx(h, rel=1e-15), (inst["name"], A, B)
            assert oracle.linkage_dist(x, "avgsq", A, B) == pytest.approx(h, rel=1e-15)
            assert brute.delta(x, A, B, "avgsq") == pytest.approx(h, rel=1e-15)


@pytest.mark.parametrize("d", [2, 7])
def test_avgsq_closed_form_tracks_definition_at_every_merge(d):
    """The chain's avg-2 heights come from centroids and spreads carried
    through every merge (closed form, Sec. 2.1 merge rule); each must equal
    the double-sum definition over the two children's member sets."""
    x = synth.blobs(160, d, 6, 0.05, 21 + d)
    n = x.shape[0]
    Z, _ = oracle.nnchain(x, "avgsq")
    mem = oracle.members(Z, n)
    for r in range(n - 1):
        A, B = mem[int(Z[r, 0])], mem[int(Z[r, 1])]
        want = oracle.linkage_dist(x, "avgsq", np.asarray(A), np.asarray(B))
        assert Z[r, 2] == pytest.approx(want, rel=1e-11, abs=1e-300), r
