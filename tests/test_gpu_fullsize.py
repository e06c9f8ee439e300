"""Parity at the benchmark's full size: 1M x 128 uint8 base, 10,000
queries, the benchmark's launch configuration (one batched call over all
queries), compared with the CPU oracle on sampled queries, which the oracle
computes one by one; invariants that hold at any size are checked on every
query.

The graph is built by the library's host builder, whose output is
byte-identical to the oracle builder's (pinned in test_abi); the oracle's
builder needs minutes at this size.  The graph is an input to both sides,
not an expected value.  The radius comes from the oracle's nearest-neighbour
distances of the first 1,000 queries (75% of them empty).
"""
import numpy as np
import pytest

import oracle
from paper_2502_13245_amd import synth
from tests.gpu_common import flush_print

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SAMPLE = 300


@pytest.fixture(scope="module")
def rr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_13245_amd import rr as _rr
    _rr.lib()
    return _rr


@pytest.fixture(scope="module")
def c2(rr):
    w = synth.config_1m_u8(1)
    flush_print("building the 1M graph on the host")
    ix = rr.Index.build(w.base, R=64, L=128, alpha=1.2, passes=2, threads=16, seed=1)
    adj, entry = ix.graph()
    ix.to_device("cuda:0")
    r = oracle.empty_fraction_radius(w.base, w.queries[:1000], 0.25)
    flush_print(f"radius {r}")
    q = torch.from_numpy(w.queries).cuda()
    return dict(w=w, adj=adj, entry=entry, r=r, ix=ix, q=q)


def _sample(counts, seed):
    rng = np.random.default_rng(seed)
    heavy = np.argsort(-counts, kind="stable")[:20]
    return np.unique(np.concatenate([rng.choice(len(counts), SAMPLE, replace=False), heavy]))


def _check_sample(g, o, idx, label):
    off, ids, d = g.numpy()
    for k, qi in enumerate(idx):
        oi, od = o.query(k)
        np.testing.assert_array_equal(ids[off[qi]:off[qi + 1]], oi, err_msg=f"{label} q{qi} ids")
        np.testing.assert_array_equal(d[off[qi]:off[qi + 1]].astype(np.int64), od.astype(np.int64),
                                      err_msg=f"{label} q{qi} dists")
        if g.stats is not None:
            for f in ("visits", "es_fired", "expanded", "greedy_visits", "count"):
                assert g.stats[f][qi] == o.stats[f][k], f"{label} q{qi} {f}"
            assert g.stats["truncated"][qi] == 0


@pytest.mark.parametrize("beam", [4, 8])
def test_adaptive_full_size_sampled(rr, c2, beam):
    """Adaptive search with early stop (vl=10, esr=r) over all 10,000
    queries in one call; sampled queries bit-exact against the oracle,
    including the 20 with the most results."""
    w, r = c2["w"], c2["r"]
    es = dict(es_enable=True, es_visit_limit=10, es_radius=r)
    flush_print(f"full size adaptive b={beam}")
    g = rr.range_search(c2["ix"], c2["q"], r, mode="adaptive", beam=beam, **es)
    idx = _sample(np.diff(g.numpy()[0]), beam)
    o = oracle.range_search(w.base, c2["adj"], c2["entry"], w.queries[idx], r,
                            mode=oracle.ADAPTIVE, beam=beam, **es)
    _check_sample(g, o, idx, f"adaptive b={beam}")
    assert g.stats["expanded"].sum() > 100 and np.diff(g.numpy()[0]).max() > 1000


@pytest.mark.parametrize("beam", [2, 3])
@pytest.mark.parametrize("vl", [2, 3])
@pytest.mark.parametrize("esr_scale", [1.0, 15.0, 20.0])
def test_adaptive_narrow_beam_full_size_sampled(rr, c2, beam, vl, esr_scale):
    """The benchmark's own region of settings (adaptive, b = 2 or 3, vl = 2
    or 3, esr = r, 15r or 20r) over all 10,000 queries in one call, in the
    benchmark's launch configuration; sampled queries (with the 20 heaviest)
    bit-exact against the oracle."""
    w, r = c2["w"], c2["r"]
    es = dict(es_enable=True, es_visit_limit=vl, es_radius=r * esr_scale)
    flush_print(f"full size adaptive b={beam} vl={vl} esr={esr_scale}r")
    g = rr.range_search(c2["ix"], c2["q"], r, mode="adaptive", beam=beam, **es)
    idx = _sample(np.diff(g.numpy()[0]), 17 * beam + vl)
    o = oracle.range_search(w.base, c2["adj"], c2["entry"], w.queries[idx], r,
                            mode=oracle.ADAPTIVE, beam=beam, **es)
    _check_sample(g, o, idx, f"adaptive b={beam} vl={vl} esr={esr_scale}r")
    assert g.stats["expanded"].sum() > 0


def test_tuned_setting_full_size_sampled(rr, c2):
    """The tuners' choice, as the benchmark makes it (rr_autotune for the
    beam and kernel shape at recall 0.9, then rr_tune_early_stop for vl and
    esr), fed unchanged to the oracle: sampled queries bit-exact in ids,
    distances and counters."""
    w, r = c2["w"], c2["r"]
    flush_print("full size tuned setting")
    truth = rr.brute_force_async(c2["ix"], c2["q"], r)
    sp, rep = rr.autotune(c2["ix"], c2["q"], r, truth, target=0.9, reps=2, mode="adaptive",
                          es_enable=True, es_visit_limit=10, es_radius=r)
    sp, es_rep = rr.tune_early_stop(c2["ix"], c2["q"], r, truth, target=0.9, reps=2, params=sp)
    flush_print(f"  tuned: beam {sp.beam}, es {sp.es_enable} vl {sp.es_visit_limit} "
                f"esr {sp.es_radius}, shape {sp.waves_per_group}x{sp.cache_slots}")
    g = rr.range_search(c2["ix"], c2["q"], r, params=sp)
    idx = _sample(np.diff(g.numpy()[0]), 99)
    o = oracle.range_search(w.base, c2["adj"], c2["entry"], w.queries[idx], r,
                            mode=oracle.ADAPTIVE, beam=sp.beam, es_enable=bool(sp.es_enable),
                            es_visit_limit=sp.es_visit_limit, es_radius=sp.es_radius)
    _check_sample(g, o, idx, "tuned")
    for k, qi in enumerate(idx):
        assert g.stats["greedy_evals"][qi] == o.stats["greedy_evals"][k], f"tuned q{qi} greedy evals"
    assert es_rep["met_target"] == 1


def test_plain_es_and_brute_force_full_size(rr, c2):
    """Plain and early-stop beam search and the MFMA brute-force scan at
    full size: sampled queries against the oracle; on every query the
    invariants that hold at any size (results within the radius, early stop
    returns either nothing or the plain result, adaptive contains plain at
    the same beam, graph results contained in brute force)."""
    w, r = c2["w"], c2["r"]
    flush_print("full size plain / es / brute force")
    plain = rr.range_search(c2["ix"], c2["q"], r, mode="plain", beam=64)
    es = rr.range_search(c2["ix"], c2["q"], r, mode="es", beam=64, es_visit_limit=10, es_radius=r)
    ada = rr.range_search(c2["ix"], c2["q"], r, mode="adaptive", beam=64)
    bf = rr.brute_force(c2["ix"], c2["q"], r)
    idx = _sample(np.diff(bf.numpy()[0]), 3)
    _check_sample(plain, oracle.range_search(w.base, c2["adj"], c2["entry"], w.queries[idx], r,
                                             mode=oracle.PLAIN, beam=64), idx, "plain")
    _check_sample(es, oracle.range_search(w.base, c2["adj"], c2["entry"], w.queries[idx], r,
                                          mode=oracle.ES, beam=64, es_visit_limit=10, es_radius=r),
                  idx, "es")
    obf = oracle.brute_force(w.base, w.queries[idx], r)
    bo, bi, bd = bf.numpy()
    for k, qi in enumerate(idx):
        oi, od = obf.query(k)
        np.testing.assert_array_equal(bi[bo[qi]:bo[qi + 1]], oi, err_msg=f"bf q{qi}")
        np.testing.assert_array_equal(bd[bo[qi]:bo[qi + 1]].astype(np.int64), od.astype(np.int64))
    po, pi, pd = plain.numpy()
    eo, ei, _ = es.numpy()
    ao, ai, ad = ada.numpy()
    assert (pd <= r).all() and (ad <= r).all()
    for qi in range(len(w.queries)):
        p_ids = pi[po[qi]:po[qi + 1]]
        e_ids = ei[eo[qi]:eo[qi + 1]]
        assert len(e_ids) == 0 or np.array_equal(e_ids, p_ids), f"q{qi}: early stop changed a result"
        a_ids = ai[ao[qi]:ao[qi + 1]]
        assert np.isin(p_ids, a_ids).all(), f"q{qi}: adaptive lost a plain result"
        assert np.isin(a_ids, bi[bo[qi]:bo[qi + 1]]).all(), f"q{qi}: result outside brute force"


# ---------------------------------------------------------------------------
# float workloads: 1M x 96 at full size (exact, bf16 and 8-bit first passes)
# and the serving workload's 768-wide rows.  Their graphs are one-pass Vamana
# graphs (R=32, L=64) from the library's host builder, so searches find the
# in-ball points and the checks below see real result lists.
# ---------------------------------------------------------------------------

def _fp64_dists(base, q, ids):
    x = base[ids].astype(np.float64) - q.astype(np.float64)
    return (x * x).sum(1)


def test_float32_1m_exact_bf16_sq8_sampled(rr):
    """1M x 96 float32 unit embeddings, 10,000 queries, radius at the 0.01th
    percentile (of a 50,000 x 200 sample of pairs).  Exact float path:
    sampled queries within 1e-5 of the FP64 oracle (sets equal outside the
    +-1e-5 band).  bf16 and 8-bit passes with recheck: every returned point
    is in the FP64 ball with its exact distance; the membership difference
    against the FP64 oracle's exact traversal on the sample is reported (an
    approximate traversal may differ, so in-ball points can be missed or
    added)."""
    w = synth.config_1m_f32(2)
    flush_print("building the 1M float graph on the host")
    ix = rr.Index.build(w.base, R=32, L=64, alpha=1.2, passes=1, threads=16, seed=2)
    adj, entry = ix.graph()
    ix.to_device("cuda:0")
    r = oracle.percentile_radius(w.base[:50_000], w.queries[:200], 0.0001)
    q = torch.from_numpy(w.queries).cuda()
    flush_print(f"1M f32 radius {r}")
    ex = rr.range_search(ix, q, r, mode="adaptive", beam=32)
    idx = np.random.default_rng(5).choice(len(w.queries), 200, replace=False)
    o = oracle.range_search(w.base, adj, entry, w.queries[idx], r, mode=oracle.ADAPTIVE, beam=32)
    eo, ei, ed = ex.numpy()
    assert len(o.ids) > 0
    for k, qi in enumerate(idx):
        oi, od = o.query(k)
        gi, gd = ei[eo[qi]:eo[qi + 1]], ed[eo[qi]:eo[qi + 1]].astype(np.float64)
        common, a, b = np.intersect1d(gi, oi, return_indices=True)
        np.testing.assert_allclose(gd[a], od[b], rtol=1e-5)
        for x in np.setxor1d(gi, oi):
            dx = _fp64_dists(w.base, w.queries[qi], np.array([x]))[0]
            assert abs(dx - r) <= 1e-5 * r, f"q{qi}: id {x} at {dx} outside the band"
    for prec, name in ((rr.BF16_RECHECK, "bf16"), (rr.SQ8_RERANK, "sq8")):
        _approx_sampled(rr, w, ix, q, r, idx, o, prec, name)


def _approx_sampled(rr, w, ix, q, r, idx, o, prec, name):
    bf = rr.range_search(ix, q, r, mode="adaptive", beam=32, precision=prec)
    bo, bi, bd = bf.numpy()
    missing = extra = total = 0
    for k, qi in enumerate(idx):
        oi, od = o.query(k)
        hi, hd = bi[bo[qi]:bo[qi + 1]], bd[bo[qi]:bo[qi + 1]].astype(np.float64)
        dd = _fp64_dists(w.base, w.queries[qi], hi)
        assert (dd <= r).all(), f"q{qi}: {name} result outside the ball"
        np.testing.assert_allclose(hd, dd, rtol=1e-6)
        missing += len(np.setdiff1d(oi, hi))
        extra += len(np.setdiff1d(hi, oi))
        total += len(oi)
    # an approximate pass traverses differently from the exact one, so it may
    # miss or add in-ball points (each one it returns was checked above)
    flush_print(f"  {name} vs FP64 oracle on {len(idx)} queries: {total} results, "
                f"{missing} missing, {extra} extra (in the ball), "
                f"band {int(bf.stats['rechecked'].sum())}")
    assert total > 0 and missing <= 0.05 * total + 5


def test_serving_d768_bf16(rr):
    """The serving workload's rows at their real width: 200,000 x 768
    float32 unit embeddings (the 2M-point workload's kernels and row layout
    on a tenth of its points; its graph takes the host about a minute), bf16
    first pass with exact recheck, 2,000 requests each with one of three
    radii (0.005, 0.01, 0.02th percentiles of a 20,000 x 100 sample of
    pairs), a step budget that suspends searches between ticks: every served
    result equals the batched result for its query and radius, and sampled
    results are inside the FP64 ball with their exact distances."""
    w = synth.latent_mixture_f32(200_000, 2_000, 768, 5_000, 0.35, 17)
    flush_print("building the d768 graph on the host")
    ix = rr.Index.build(w.base, R=32, L=64, alpha=1.2, passes=1, threads=16, seed=13)
    levels = [oracle.percentile_radius(w.base[:20_000], w.queries[:100], p)
              for p in (0.00005, 0.0001, 0.0002)]
    radii = np.asarray(levels)[np.arange(len(w.queries)) % 3]
    ix.to_device("cuda:0")
    flush_print(f"d768 radii {levels}")
    sp = rr.search_params(mode="adaptive", beam=16, precision=rr.BF16_RECHECK)
    batch = rr.range_search(ix, torch.from_numpy(w.queries).cuda(), torch.from_numpy(radii),
                            params=sp)
    off, ids, d = batch.numpy()
    flush_print(f"  batched results {len(ids)}")
    assert len(ids) > 0
    got = {}
    with rr.Server(ix, sp, slots=512, step_budget=8) as srv:
        for qi in range(len(w.queries)):
            assert srv.submit(w.queries[qi], float(radii[qi]), qi)
        srv.drain(timeout=120.0)
        comps = srv.poll(len(w.queries) + 8)
        for c in comps:
            got[c.tag] = srv.result(c.tag)
        info = srv.info()
    assert len(got) == len(w.queries)
    flush_print(f"  served {len(got)} in {info['ticks']} ticks, max resident {info['max_resident']}")
    for qi in range(len(w.queries)):
        gi, gd = got[qi]
        np.testing.assert_array_equal(gi, ids[off[qi]:off[qi + 1]], err_msg=f"q{qi}")
        np.testing.assert_array_equal(gd, d[off[qi]:off[qi + 1]], err_msg=f"q{qi}")
    for qi in np.random.default_rng(9).choice(len(w.queries), 100, replace=False):
        gi, gd = got[qi]
        dd = _fp64_dists(w.base, w.queries[qi], gi)
        assert (dd <= radii[qi]).all()
        np.testing.assert_allclose(gd.astype(np.float64), dd, rtol=1e-6)


# ---------------------------------------------------------------------------
# int8 at the batching workload's full size: 10M x 100 base, 100,000 queries
# in uneven batches.  The graph is a seeded shifted random graph (a Vamana
# build of 10M points takes the host many minutes); parity does not depend
# on graph quality.  At this size adjacency offsets pass 2^31 bytes, each
# task's membership bitmap is 1.25 MB, and the heaviest query returns over
# 100,000 points (the sort's global merge path).
# ---------------------------------------------------------------------------

def test_int8_10m_uneven_batches(rr):
    """Every query's result is the same in one 100,000-query launch and in
    batches of 1k, 4k, 16k, 64k and 15k; sampled queries equal the oracle
    (ids, distances, visit counts)."""
    w = synth.config_i8(3)
    adj = synth.shifted_graph(len(w.base), 64, 17)
    # radius: 75% of 200 sampled queries empty (the oracle's nearest neighbours)
    r = oracle.empty_fraction_radius(w.base, w.queries[:200], 0.25)
    ix = rr.Index.from_graph(w.base, adj, 0).to_device("cuda:0")
    q = torch.from_numpy(w.queries).cuda()
    flush_print(f"10M int8 radius {r}")
    kw = dict(mode="adaptive", beam=16, es_enable=True, es_visit_limit=10, es_radius=r,
              result_capacity=20_000_000)
    one = rr.range_search(ix, q, r, **kw)
    off, ids, d = one.numpy()
    counts = np.diff(off)
    flush_print(f"  one launch: {int(off[-1])} results, {int((counts > 0).sum())} non-empty, "
                f"max {counts.max()}, expanded {int(one.stats['expanded'].sum())}")
    assert counts.max() > 0
    start = 0
    for size in (1_000, 4_000, 16_000, 64_000, 15_000):
        part = rr.range_search(ix, q[start:start + size], r, **kw)
        po, pi, pd = part.numpy()
        for k in range(size):
            qi = start + k
            np.testing.assert_array_equal(pi[po[k]:po[k + 1]], ids[off[qi]:off[qi + 1]])
            np.testing.assert_array_equal(pd[po[k]:po[k + 1]], d[off[qi]:off[qi + 1]])
        np.testing.assert_array_equal(part.stats["visits"], one.stats["visits"][start:start + size])
        start += size
    assert start == len(w.queries)
    rng = np.random.default_rng(9)
    idx = np.unique(np.concatenate([rng.choice(len(counts), 100, replace=False),
                                    np.argsort(-counts, kind="stable")[:20]]))
    o = oracle.range_search(w.base, adj, 0, w.queries[idx], r, mode=oracle.ADAPTIVE, beam=16,
                            es_enable=True, es_visit_limit=10, es_radius=r)
    for k, qi in enumerate(idx):
        oi, od = o.query(k)
        np.testing.assert_array_equal(ids[off[qi]:off[qi + 1]], oi, err_msg=f"q{qi} ids")
        np.testing.assert_array_equal(d[off[qi]:off[qi + 1]].astype(np.int64), od.astype(np.int64))
        assert one.stats["visits"][qi] == o.stats["visits"][k]
