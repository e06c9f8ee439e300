"""Pins for the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: hand-derived
results of the paper's algorithms on tiny inputs (tests/golden), library
routines (scipy's cdist and cKDTree), closed forms, and invariants the
algorithms imply (complete graph == Definition 2.1, the greedy result is the
closure of its seeds inside the ball, early stopping never changes a
non-empty answer, ...).
"""
import json
import os
from collections import deque

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.distance import cdist

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")))

MODES = {"plain": oracle.PLAIN, "es": oracle.ES, "adaptive": oracle.ADAPTIVE,
         "doubling": oracle.DOUBLING}


def sq(a, b):
    """Squared L2 matrix from scipy (float64 for float32 input, exact for small ints)."""
    return cdist(a.astype(np.float64), b.astype(np.float64), "sqeuclidean")


# ---------------------------------------------------------------------------
# distances (Section 2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dt", [np.uint8, np.int8, np.float32])
def test_dist_matches_cdist(dt):
    rng = np.random.default_rng(1)
    for d in (1, 3, 100, 128, 257):
        if dt == np.float32:
            a = rng.standard_normal((2, d)).astype(dt)
        else:
            info = np.iinfo(dt)
            a = rng.integers(info.min, info.max + 1, size=(2, d)).astype(dt)
        got = oracle.dist(a[0], a[1])
        want = sq(a[:1], a[1:])[0, 0]
        if dt == np.float32:
            assert got == pytest.approx(want, rel=1e-12)
        else:
            assert got == want


def test_dist_closed_forms():
    # extreme uint8 distance: 128 * 255^2
    a = np.zeros(128, np.uint8)
    b = np.full(128, 255, np.uint8)
    assert oracle.dist(a, b) == 128 * 255 ** 2 == 8_323_200
    # int8 extremes: (127 - (-128))^2 per coordinate
    assert oracle.dist(np.full(100, -128, np.int8), np.full(100, 127, np.int8)) == 100 * 255 ** 2
    # orthogonal unit vectors are at squared distance 2
    e = np.eye(96, dtype=np.float32)
    assert oracle.dist(e[3], e[70]) == 2.0
    # symmetric and zero on the diagonal
    x = np.arange(16, dtype=np.uint8)
    y = x[::-1].copy()
    assert oracle.dist(x, y) == oracle.dist(y, x)
    assert oracle.dist(x, x) == 0


# ---------------------------------------------------------------------------
# Definition 2.1 by enumeration
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dt", [np.uint8, np.int8, np.float32])
def test_brute_force_matches_kdtree_and_cdist(dt):
    rng = np.random.default_rng(7)
    n, nq, d = 300, 25, 6
    if dt == np.float32:
        base = rng.standard_normal((n, d)).astype(dt)
        qs = rng.standard_normal((nq, d)).astype(dt)
        r = 2.5
    else:
        lo, hi = (0, 12) if dt == np.uint8 else (-6, 6)
        base = rng.integers(lo, hi, (n, d)).astype(dt)
        qs = rng.integers(lo, hi, (nq, d)).astype(dt)
        r = 40.0  # integer radius: the inclusive boundary is exercised
    res = oracle.brute_force(base, qs, r)
    D = sq(qs, base)
    tree = cKDTree(base.astype(np.float64))
    for q in range(nq):
        ids, dists = res.query(q)
        want = np.flatnonzero(D[q] <= r)
        assert set(ids.tolist()) == set(want.tolist())
        if dt != np.float32:
            # integers: the KD-tree with a radius strictly between integer squares agrees
            kd = tree.query_ball_point(qs[q].astype(np.float64), np.sqrt(r + 0.5))
            assert set(ids.tolist()) == set(kd)
        # sorted by (d, id), distances exact
        np.testing.assert_allclose(dists, D[q, ids], rtol=1e-12)
        keys = list(zip(dists.tolist(), ids.tolist()))
        assert keys == sorted(keys)


def test_brute_force_inclusive_and_empty():
    base = np.array([[0], [3], [5]], np.uint8)
    q = np.array([[0]], np.uint8)
    assert oracle.brute_force(base, q, 9.0).query(0)[0].tolist() == [0, 1]   # d=9 included
    assert oracle.brute_force(base, q, 8.999).query(0)[0].tolist() == [0]
    assert oracle.brute_force(base, q, -1.0).counts().tolist() == [0]       # negative radius
    assert oracle.brute_force(base, np.zeros((0, 1), np.uint8), 1.0).offsets.tolist() == [0]


def test_nn_dist_matches_cdist():
    rng = np.random.default_rng(3)
    base = rng.integers(0, 256, (500, 16)).astype(np.uint8)
    qs = rng.integers(0, 256, (40, 16)).astype(np.uint8)
    np.testing.assert_array_equal(oracle.nn_dist(base, qs), sq(qs, base).min(1))


# ---------------------------------------------------------------------------
# hand-derived runs of Algorithms 1, 2, 3, 5, 6 (tests/golden)
# ---------------------------------------------------------------------------

def _golden_cases():
    for gname in ("line10", "even10_es", "line10_ip"):
        g = GOLD[gname]
        for c in g["cases"]:
            yield pytest.param(gname, c, id=f"{gname}-{c['name']}")


@pytest.mark.parametrize("gname,case", list(_golden_cases()))
def test_golden_line_graphs(gname, case):
    g = GOLD[gname]
    base = np.array(g["points"], np.uint8)
    adj = np.array(g["adj"], np.int32)
    q = np.array([g["query"]], np.uint8)
    metric = g.get("metric", "l2")
    if case["mode"] == "brute":
        res = oracle.brute_force(base, q, case["radius"], metric=metric)
    else:
        res = oracle.range_search(base, adj, g["entry"], q, case["radius"],
                                  mode=MODES[case["mode"]], beam=case["beam"],
                                  es_enable=case["mode"] == "es",
                                  es_visit_limit=case.get("vl", 0), es_radius=case.get("esr", 0.0),
                                  lam=case.get("lambda", 1.0), max_beam=case.get("max_beam", 1 << 20),
                                  metric=metric)
    ids, dists = res.query(0)
    assert ids.tolist() == case["ids"]
    assert dists.tolist() == case["dists"]
    if res.stats is not None:
        st = res.stats[0]
        for key in ("visits", "es_fired", "expanded", "greedy_visits", "greedy_evals", "rounds",
                    "final_beam", "truncated"):
            if key in case:
                assert st[key] == case[key], key


@pytest.mark.parametrize("gname", ["prune_1d", "prune_2d_alpha"])
def test_golden_robust_prune(gname):
    g = GOLD[gname]
    base = np.array(g["points"], np.uint8)
    for alpha, want in g["expect"].items():
        got = oracle.robust_prune(base, g["p"], g["cand"], float(alpha), g["R"])
        assert got.tolist() == want, alpha


def test_golden_medoid_and_percentile():
    for c in GOLD["medoid"]["cases"]:
        assert oracle.medoid(np.array(c["points"], np.uint8)) == c["entry"]
    g = GOLD["percentile"]
    base = np.array(g["points"], np.uint8)
    qs = np.array(g["queries"], np.uint8)
    for c in g["cases"]:
        assert oracle.percentile_radius(base, qs, c["p"]) == c["radius"]


def test_medoid_matches_numpy_mean():
    rng = np.random.default_rng(11)
    for dt in (np.uint8, np.int8, np.float32):
        if dt == np.float32:
            x = rng.standard_normal((400, 7)).astype(dt)
        else:
            x = rng.integers(-50 if dt == np.int8 else 0, 100, (400, 7)).astype(dt)
        m = x.astype(np.float64).mean(0)
        dd = ((x.astype(np.float64) - m) ** 2).sum(1)
        assert oracle.medoid(x) == int(np.flatnonzero(dd == dd.min())[0])


def test_range_recall_closed_form():
    t = oracle.Result(np.array([0, 3, 3, 4]), np.array([1, 2, 3, 9]), np.zeros(4), None)
    f = oracle.Result(np.array([0, 2, 2, 2]), np.array([1, 3]), np.zeros(2), None)
    assert oracle.range_recall(t, f) == pytest.approx(2 / 4)
    e = oracle.Result(np.array([0, 0]), np.array([], int), np.zeros(0), None)
    assert np.isnan(oracle.range_recall(e, e))


# ---------------------------------------------------------------------------
# invariants of the algorithms on random tiny graphs with many ties
# ---------------------------------------------------------------------------

def _tiny_instance(rng, n=None, R=None):
    n = n or int(rng.integers(5, 60))
    d = int(rng.integers(1, 5))
    R = R or int(rng.integers(1, 8))
    base = rng.integers(0, 6, (n, d)).astype(np.uint8)
    adj = np.full((n, R), -1, np.int32)
    for i in range(n):
        k = int(rng.integers(0, min(R, n - 1) + 1))
        others = np.delete(np.arange(n), i)
        adj[i, :k] = rng.choice(others, size=k, replace=False)
    qs = rng.integers(0, 6, (8, d)).astype(np.uint8)
    r = float(rng.integers(0, 12))
    entry = int(rng.integers(0, n))
    return base, adj, entry, qs, r


def _complete(n):
    return np.array([[j for j in range(n) if j != i] for i in range(n)], np.int32).reshape(n, n - 1)


def test_complete_graph_equals_brute_force():
    """On a complete graph every search mode reaches Definition 2.1 exactly."""
    rng = np.random.default_rng(5)
    for _ in range(60):
        n = int(rng.integers(2, 40))
        d = int(rng.integers(1, 4))
        base = rng.integers(0, 6, (n, d)).astype(np.uint8)
        qs = rng.integers(0, 6, (6, d)).astype(np.uint8)
        r = float(rng.integers(0, 10))
        adj = _complete(n)
        entry = int(rng.integers(0, n))
        bf = oracle.brute_force(base, qs, r)
        runs = [oracle.range_search(base, adj, entry, qs, r, mode=oracle.PLAIN, beam=n)]
        for b in (1, 2, 5):
            runs.append(oracle.range_search(base, adj, entry, qs, r, mode=oracle.ADAPTIVE, beam=b))
            runs.append(oracle.range_search(base, adj, entry, qs, r, mode=oracle.DOUBLING, beam=b))
            runs.append(oracle.range_search(base, adj, entry, qs, r, mode=oracle.ADAPTIVE, beam=b,
                                            es_enable=True, es_visit_limit=1, es_radius=0.0))
        for res in runs:
            np.testing.assert_array_equal(res.offsets, bf.offsets)
            np.testing.assert_array_equal(res.ids, bf.ids)
            np.testing.assert_array_equal(res.dists, bf.dists)


def _closure(adj, dvec, seeds, r):
    """Points reachable from the seeds along edges whose endpoints lie in the ball."""
    seen = set(seeds)
    dq = deque(seeds)
    while dq:
        p = dq.popleft()
        for f in adj[p]:
            if f >= 0 and f not in seen and dvec[f] <= r:
                seen.add(f)
                dq.append(f)
    return seen


def test_invariants_random_graphs():
    rng = np.random.default_rng(2024)
    for _ in range(300):
        base, adj, entry, qs, r = _tiny_instance(rng)
        b = int(rng.integers(1, 6))
        D = sq(qs, base)
        plain = oracle.range_search(base, adj, entry, qs, r, mode=oracle.PLAIN, beam=b)
        es = oracle.range_search(base, adj, entry, qs, r, mode=oracle.ES, beam=b,
                                 es_visit_limit=int(rng.integers(1, 4)),
                                 es_radius=float(rng.integers(0, 10)))
        ad = oracle.range_search(base, adj, entry, qs, r, mode=oracle.ADAPTIVE, beam=b)
        for q in range(len(qs)):
            p_ids, p_d = plain.query(q)
            # soundness (Definition 2.1) and exact distances
            assert np.all(D[q, p_ids] <= r)
            np.testing.assert_array_equal(p_d, D[q, p_ids])
            # I6: plain returns at most b points; adaptive contains plain
            assert len(p_ids) <= b
            a_ids, a_d = ad.query(q)
            assert set(p_ids.tolist()) <= set(a_ids.tolist())
            assert np.all(D[q, a_ids] <= r)
            # I4: early stopping returns the plain answer or nothing
            e_ids, _ = es.query(q)
            assert e_ids.size == 0 or e_ids.tolist() == p_ids.tolist()
            if es.stats[q]["es_fired"]:
                assert e_ids.size == 0
            # I5: the greedy phase returns the closure of N inside the ball
            if ad.stats[q]["expanded"]:
                assert len(p_ids) >= b
                want = _closure(adj, D[q], p_ids.tolist(), r)
                assert set(a_ids.tolist()) == want
                assert ad.stats[q]["greedy_visits"] == len(want)
                nb = {int(f) for v in want for f in adj[v] if f >= 0} - set(p_ids.tolist())
                assert ad.stats[q]["greedy_evals"] == len(nb)
            else:
                assert a_ids.tolist() == p_ids.tolist()


def _beam_seen_filter(base, adj, entry, q, b):
    """Algorithm 1 written the other way round: neighbours are filtered by
    'ever evaluated' instead of by V, and insertion into B de-duplicates.
    Used to pin the claim that both give the same beam and visit count."""
    def dd(i):
        return float(((base[i].astype(np.int64) - q.astype(np.int64)) ** 2).sum())
    B = [(dd(entry), entry, False)]
    seen = {entry}
    visits = 0
    while True:
        cand = [i for i, e in enumerate(B) if not e[2]]
        if not cand:
            break
        i = cand[0]
        dp, p, _ = B[i]
        B[i] = (dp, p, True)
        visits += 1
        new = []
        for u in adj[p]:
            if u < 0 or u in seen:
                continue
            seen.add(u)
            new.append((dd(u), int(u), False))
        B = sorted(B + new, key=lambda e: (e[0], e[1]))[:b]
    return B, visits


def test_seen_filter_gives_same_beam():
    """Filtering by 'ever evaluated' (a cache that may forget) is exact."""
    rng = np.random.default_rng(99)
    for _ in range(200):
        base, adj, entry, qs, r = _tiny_instance(rng)
        b = int(rng.integers(1, 6))
        res = oracle.range_search(base, adj, entry, qs, 1e9, mode=oracle.PLAIN, beam=b)
        for qi in range(len(qs)):
            B, visits = _beam_seen_filter(base, adj, entry, qs[qi], b)
            ids, dists = res.query(qi)
            assert ids.tolist() == [e[1] for e in B]
            assert dists.tolist() == [e[0] for e in B]
            assert res.stats[qi]["visits"] == visits


def test_float_search_sound_and_exact_distances():
    rng = np.random.default_rng(8)
    n, d = 200, 8
    base = rng.standard_normal((n, d)).astype(np.float32)
    base /= np.linalg.norm(base, axis=1, keepdims=True)
    qs = base[rng.integers(0, n, 10)] + 0.05 * rng.standard_normal((10, d)).astype(np.float32)
    adj, entry = oracle.build_vamana(base, 16, 32, 1.2, np.arange(n, dtype=np.int64))
    r = 0.3
    res = oracle.range_search(base, adj, entry, qs, r, mode=oracle.ADAPTIVE, beam=8)
    D = sq(qs, base)
    for q in range(len(qs)):
        ids, dists = res.query(q)
        assert np.all(D[q, ids] <= r)
        np.testing.assert_allclose(dists, D[q, ids], rtol=1e-12)


# ---------------------------------------------------------------------------
# Vamana construction: invariants and determinism
# ---------------------------------------------------------------------------

def _check_graph(adj, n, R):
    assert adj.shape == (n, R)
    for i in range(n):
        row = adj[i]
        nz = row[row >= 0]
        # -1 padding only at the end, ids in range, no self loops, no repeats
        assert np.all(row[len(nz):] == -1)
        assert np.all(nz < n)
        assert i not in nz
        assert len(set(nz.tolist())) == len(nz)


def _reachable(adj, entry):
    seen = {entry}
    dq = deque([entry])
    while dq:
        p = dq.popleft()
        for f in adj[p]:
            if f >= 0 and f not in seen:
                seen.add(f)
                dq.append(f)
    return seen


@pytest.mark.parametrize("dt", [np.uint8, np.float32])
def test_vamana_invariants_and_determinism(dt):
    rng = np.random.default_rng(4)
    n, d, R = 600, 8, 12
    if dt == np.uint8:
        base = rng.integers(0, 256, (n, d)).astype(dt)
    else:
        base = rng.standard_normal((n, d)).astype(dt)
    order = rng.permutation(n).astype(np.int64)
    a1, e1 = oracle.build_vamana(base, R, 24, 1.2, order, threads=1)
    a4, e4 = oracle.build_vamana(base, R, 24, 1.2, order, threads=4)
    np.testing.assert_array_equal(a1, a4)
    assert e1 == e4 == oracle.medoid(base)
    _check_graph(a1, n, R)
    assert len(_reachable(a1, e1)) == n
    # graph quality is only reported: beam search with b=32 should find most true neighbours
    qs = base[:50]
    bf = oracle.brute_force(base, qs, 0.0)
    res = oracle.range_search(base, a1, e1, qs, 0.0, mode=oracle.PLAIN, beam=32)
    assert oracle.range_recall(bf, res) >= 0.9


def test_vamana_pruned_rows_respect_alpha():
    """Rows produced by a prune keep the alpha-RNG property; a row filled by
    back edges without pruning is a prefix of such a row plus appended sources."""
    rng = np.random.default_rng(6)
    n, d, R = 300, 4, 6
    base = rng.integers(0, 256, (n, d)).astype(np.uint8)
    alpha = 1.2
    for p in range(0, n, 17):
        cand = rng.choice(np.delete(np.arange(n), p), size=40, replace=False)
        out = oracle.robust_prune(base, p, cand, alpha, R)
        assert len(out) <= R
        D = sq(base, base)
        # every kept c_j is not dominated by an earlier kept c_i
        for j in range(len(out)):
            for i in range(j):
                assert alpha * alpha * D[out[i], out[j]] > D[p, out[j]]
        # every dropped candidate is dominated by some kept point or R was reached
        if len(out) < R:
            for c in set(cand.tolist()) - set(out.tolist()):
                assert any(alpha * alpha * D[k, c] <= D[p, c] for k in out)


def test_pair_dists_and_percentile_match_cdist():
    rng = np.random.default_rng(12)
    base = rng.integers(0, 256, (300, 9)).astype(np.uint8)
    qs = rng.integers(0, 256, (30, 9)).astype(np.uint8)
    D = sq(qs, base)
    np.testing.assert_array_equal(oracle.pair_dists(base, qs), D)
    for p in (0.001, 0.01, 0.5):
        k = int(np.ceil(p * D.size))
        assert oracle.percentile_radius(base, qs, p) == np.sort(D.ravel())[k - 1]
    nn = np.sort(D.min(1))
    assert oracle.empty_fraction_radius(base, qs, 0.25) == nn[int(np.ceil(0.25 * 30)) - 1]


@pytest.mark.parametrize("case", GOLD["es_profile_line10"]["cases"], ids=lambda c: c["name"])
def test_es_profile_hand_examples(case):
    """The early-stopping metrics at a fixed step, derived by hand on the
    10-point line graph."""
    g = GOLD["line10"]
    base = np.array(g["points"], np.uint8)
    adj = np.array(g["adj"], np.int32)
    q = np.array([g["query"]], np.uint8)
    m, f = oracle.es_profile(base, adj, g["entry"], q, case["radius"], case["beam"], case["step"])
    assert f[0].tolist() == [case["reached"], case["found"]]
    if case["reached"]:
        top10 = np.inf if case["d_top10"] is None else case["d_top10"]
        assert m[0].tolist() == [case["d_visited"], case["d_top1"], top10, case["d_start"]]
    else:
        assert np.isnan(m[0, :3]).all()


def test_es_profile_predicts_the_stop_at_vl():
    """Algorithm 5 stops exactly at v = vl iff at that step no point of B is
    within r and d(p*) > esr: the metrics at step vl must predict which
    queries an early-stopped search ends after vl visits."""
    rng = np.random.default_rng(4)
    base = rng.integers(0, 40, size=(600, 6)).astype(np.uint8)
    queries = rng.integers(0, 40, size=(80, 6)).astype(np.uint8)
    adj, entry = oracle.build_vamana(base, 12, 24, 1.2, np.arange(600))
    r = oracle.percentile_radius(base, queries, 0.003)
    for vl, qt in ((3, 0.3), (6, 0.5), (10, 0.7)):
        m, f = oracle.es_profile(base, adj, entry, queries, r, 16, vl)
        open_q = (f[:, 0] == 1) & (f[:, 1] == 0)
        esr = float(np.quantile(m[open_q, 0], qt))  # a cutoff inside the observed spread
        es = oracle.range_search(base, adj, entry, queries, r, mode=oracle.ES, beam=16,
                                 es_visit_limit=vl, es_radius=esr)
        predicted = (f[:, 0] == 1) & (f[:, 1] == 0) & (m[:, 0] > esr)
        stopped_at_vl = (es.stats["es_fired"] == 1) & (es.stats["visits"] == vl)
        np.testing.assert_array_equal(predicted, stopped_at_vl)
        assert predicted.any() and (open_q & ~predicted).any()



@pytest.mark.parametrize("dt", [np.uint8, np.int8, np.float32])
def test_ip_dist_and_brute_force_closed_forms(dt):
    """Negated inner product: exact int64 dot products for integer data,
    FP64 for float32; Definition 2.1 under it by numpy enumeration."""
    rng = np.random.default_rng(11)
    if dt == np.float32:
        base = rng.standard_normal((300, 20)).astype(dt)
        qs = rng.standard_normal((25, 20)).astype(dt)
        D = -(qs.astype(np.float64) @ base.astype(np.float64).T)
    else:
        lo, hi = (0, 256) if dt == np.uint8 else (-128, 128)
        base = rng.integers(lo, hi, (300, 20)).astype(dt)
        qs = rng.integers(lo, hi, (25, 20)).astype(dt)
        D = -(qs.astype(np.int64) @ base.astype(np.int64).T).astype(np.float64)
    for i in range(5):
        assert oracle.dist(qs[i], base[i], metric="ip") == pytest.approx(D[i, i], rel=1e-12, abs=1e-12)
    r = float(np.quantile(D, 0.05))
    bf = oracle.brute_force(base, qs, r, metric="ip")
    for qi in range(len(qs)):
        hit = np.flatnonzero(D[qi] <= r)
        order = np.lexsort((hit, D[qi, hit]))
        np.testing.assert_array_equal(bf.query(qi)[0], hit[order])
        np.testing.assert_allclose(bf.query(qi)[1], D[qi, hit[order]], rtol=1e-12, atol=1e-12)
    # float32 data: numpy's blocked dot products sum in another order (1e-15)
    tol = dict(rtol=1e-12, atol=1e-12) if dt == np.float32 else dict(rtol=0, atol=0)
    np.testing.assert_allclose(oracle.pair_dists(base, qs, metric="ip"), D, **tol)
    np.testing.assert_allclose(oracle.nn_dist(base, qs, metric="ip"), D.min(1), **tol)


def test_ip_complete_graph_and_closure():
    """Under the inner product: on a complete graph every mode equals brute
    force, and on random graphs the adaptive result is the closure of N in
    the ball (the properties the L2 tests check)."""
    rng = np.random.default_rng(12)
    for _ in range(40):
        n = int(rng.integers(2, 40))
        base = rng.integers(0, 6, (n, 3)).astype(np.uint8)
        qs = rng.integers(0, 6, (5, 3)).astype(np.uint8)
        D = -(qs.astype(np.int64) @ base.astype(np.int64).T)
        r = float(np.quantile(D, 0.3))
        adj = _complete(n)
        entry = int(rng.integers(0, n))
        bf = oracle.brute_force(base, qs, r, metric="ip")
        for b in (1, 3):
            for mode in (oracle.ADAPTIVE, oracle.DOUBLING):
                res = oracle.range_search(base, adj, entry, qs, r, mode=mode, beam=b, metric="ip")
                np.testing.assert_array_equal(res.ids, bf.ids)
                np.testing.assert_array_equal(res.offsets, bf.offsets)
        res = oracle.range_search(base, adj, entry, qs, r, mode=oracle.PLAIN, beam=n, metric="ip")
        np.testing.assert_array_equal(res.ids, bf.ids)
        # random sparse graph: adaptive = closure of N inside the ball
        R = 3
        g = np.full((n, R), -1, np.int32)
        for i in range(n):
            others = np.setdiff1d(np.arange(n), [i])
            k = min(R, len(others))
            g[i, :k] = rng.choice(others, k, replace=False)
        plain = oracle.range_search(base, g, entry, qs, r, mode=oracle.PLAIN, beam=2, metric="ip")
        ada = oracle.range_search(base, g, entry, qs, r, mode=oracle.ADAPTIVE, beam=2, metric="ip")
        for qi in range(len(qs)):
            N = plain.query(qi)[0]
            if len(N) >= 2:
                want = _closure(g, D[qi].astype(np.float64), N, r)
                assert set(ada.query(qi)[0].tolist()) == want
            else:
                np.testing.assert_array_equal(ada.query(qi)[0], N)
