"""GPU parity of the negated inner-product distance (Section 2: maximum inner
product search as range search with d(p, q) = -<p, q>) against the oracle.

Integer data is bit-exact (ids, distances, visit counters) in every search
mode, the dense scan and the early-stopping metrics; float32 data is within
1e-5 relative with equal sets outside a +-1e-5 band around the radius; the
bfloat16 pass returns only points inside the ball by the exact distance.
Radii are negative here (the points of largest inner product), as in the
paper's inner-product workloads.
"""
import numpy as np
import pytest

import oracle
from paper_2502_13245_amd import synth
from tests.gpu_common import compare_exact, compare_float, flush_print

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_13245_amd import rr as _rr
    _rr.lib()
    return _rr


def _ctx(rr, w, adj, entry, r):
    ix = rr.Index.from_graph(w.base, adj, entry, metric="ip").to_device("cuda:0")
    return dict(w=w, adj=adj, entry=entry, r=r, ix=ix, q=torch.from_numpy(w.queries).cuda())


@pytest.fixture(scope="module")
def ip_u8(rr):
    """8,000 x 128 uint8 base (low intrinsic dimension), 500 queries; the
    radius keeps the 0.2% largest inner products of all pairs."""
    w = synth.latent_mixture_u8(8000, 500, 128, 60, 25.0, 51)
    adj, entry = oracle.build_vamana(w.base, 32, 64, 1.2, synth.permutation(8000, 51))
    r = oracle.percentile_radius(w.base, w.queries, 0.002, metric="ip")
    return _ctx(rr, w, adj, entry, r)


@pytest.fixture(scope="module")
def ip_f32(rr):
    """4,000 x 96 float32 embeddings with row norms spread over [0.5, 2]
    (the inner product is not a function of L2 there), 300 queries."""
    w = synth.latent_mixture_f32(4000, 300, 96, 40, 0.35, 61)
    rng = np.random.default_rng(61)
    w.base[:] = w.base * rng.uniform(0.5, 2.0, (len(w.base), 1)).astype(np.float32)
    w.queries[:] = w.queries * rng.uniform(0.5, 2.0, (len(w.queries), 1)).astype(np.float32)
    adj, entry = oracle.build_vamana(w.base, 32, 64, 1.2, synth.permutation(4000, 61))
    r = oracle.percentile_radius(w.base, w.queries, 0.003, metric="ip")
    return _ctx(rr, w, adj, entry, r)


def _orc(ctx, **kw):
    return oracle.range_search(ctx["w"].base, ctx["adj"], ctx["entry"], ctx["w"].queries,
                               kw.pop("radius", ctx["r"]), metric="ip", **kw)


@pytest.mark.parametrize("mode,om,beam,es", [("plain", oracle.PLAIN, 16, False),
                                             ("es", oracle.ES, 32, True),
                                             ("adaptive", oracle.ADAPTIVE, 8, True),
                                             ("adaptive", oracle.ADAPTIVE, 16, False)])
def test_ip_u8_modes_bit_exact(rr, ip_u8, mode, om, beam, es):
    ctx = ip_u8
    assert ctx["r"] < 0
    kw = dict(es_enable=es, es_visit_limit=5, es_radius=ctx["r"] * 0.5)
    flush_print(f"ip u8 {mode} beam={beam} es={es} r={ctx['r']}")
    g = rr.range_search(ctx["ix"], ctx["q"], ctx["r"], mode=mode, beam=beam, **kw)
    o = _orc(ctx, mode=om, beam=beam, **kw)
    compare_exact(g, o, label=f"ip {mode} b={beam}")
    assert len(o.ids) > 0 and (o.dists < 0).all()
    if mode == "adaptive" and not es:
        assert o.stats["expanded"].any()


def test_ip_u8_doubling_and_per_query_radii(rr, ip_u8):
    """Algorithm 3 under the inner product, then per-query radii (on uint8
    data every inner product is >= 0, so a radius >= 0 would admit all n)."""
    ctx = ip_u8
    flush_print("ip u8 doubling")
    g = rr.range_search(ctx["ix"], ctx["q"], ctx["r"], mode="doubling", beam=4, max_beam=1024)
    o = _orc(ctx, mode=oracle.DOUBLING, beam=4, max_beam=1024)
    off, ids, d = g.numpy()
    np.testing.assert_array_equal(off, o.offsets)
    np.testing.assert_array_equal(ids, o.ids)
    np.testing.assert_array_equal(d.astype(np.int64), o.dists.astype(np.int64))
    for f in ("visits", "rounds", "final_beam", "truncated", "count"):
        np.testing.assert_array_equal(g.stats[f], o.stats[f], err_msg=f)
    rng = np.random.default_rng(7)
    radii = ctx["r"] * rng.choice([1.0, 0.8, 1.2, 2.0], size=len(ctx["w"].queries))
    flush_print("ip u8 per-query radii")
    g = rr.range_search(ctx["ix"], ctx["q"], torch.from_numpy(radii).cuda(), mode="adaptive",
                        beam=8, result_capacity=2_000_000)
    o = _orc(ctx, radius=radii, mode=oracle.ADAPTIVE, beam=8)
    compare_exact(g, o, label="ip radii")


def test_ip_int8_and_ragged_dims(rr):
    """int8 (inner products of both signs) with d=100 and uint8 with d=7."""
    for d, signed in ((100, True), (7, False)):
        w = synth.gaussian_mixture_int(3000, 200, d, 30, 12.0, 19, signed=signed, spread=0.3)
        adj, entry = oracle.build_vamana(w.base, 24, 48, 1.2, synth.permutation(3000, 19))
        r = oracle.percentile_radius(w.base, w.queries, 0.002, metric="ip")
        ix = rr.Index.from_graph(w.base, adj, entry, metric="ip").to_device("cuda:0")
        q = torch.from_numpy(w.queries).cuda()
        flush_print(f"ip int d={d} signed={signed} r={r}")
        for mode, om in (("plain", oracle.PLAIN), ("adaptive", oracle.ADAPTIVE)):
            g = rr.range_search(ix, q, r, mode=mode, beam=16)
            o = oracle.range_search(w.base, adj, entry, w.queries, r, mode=om, beam=16,
                                    metric="ip")
            compare_exact(g, o, label=f"ip d={d} {mode}")


def test_ip_dense_scan_and_nn(rr, ip_u8, ip_f32):
    """The MFMA scan (uint8 through the shifted int8 products, int8 direct,
    float32 in FP64) against the oracle's brute force and nearest neighbours."""
    ctx = ip_u8
    flush_print("ip scan u8")
    g = rr.brute_force(ctx["ix"], ctx["q"], ctx["r"])
    o = oracle.brute_force(ctx["w"].base, ctx["w"].queries, ctx["r"], metric="ip")
    off, ids, d = g.numpy()
    np.testing.assert_array_equal(off, o.offsets)
    np.testing.assert_array_equal(ids, o.ids)
    np.testing.assert_array_equal(d.astype(np.int64), o.dists.astype(np.int64))
    nn = rr.nn_dist(ctx["ix"], ctx["q"]).cpu().numpy()
    np.testing.assert_array_equal(nn, oracle.nn_dist(ctx["w"].base, ctx["w"].queries, metric="ip"))
    w = synth.gaussian_mixture_int(2000, 130, 64, 20, 12.0, 23, signed=True, spread=0.3)
    r = oracle.percentile_radius(w.base, w.queries, 0.01, metric="ip")
    ix = rr.Index.from_graph(w.base, synth.random_graph(2000, 8, 23), 0,
                             metric="ip").to_device("cuda:0")
    q = torch.from_numpy(w.queries).cuda()
    flush_print("ip scan i8")
    g = rr.brute_force(ix, q, r)
    o = oracle.brute_force(w.base, w.queries, r, metric="ip")
    off, ids, d = g.numpy()
    np.testing.assert_array_equal(ids, o.ids)
    np.testing.assert_array_equal(d.astype(np.int64), o.dists.astype(np.int64))
    np.testing.assert_array_equal(rr.nn_dist(ix, q).cpu().numpy(),
                                  oracle.nn_dist(w.base, w.queries, metric="ip"))
    ctx = ip_f32
    flush_print("ip scan f32")
    g = rr.brute_force(ctx["ix"], ctx["q"], ctx["r"])
    o = oracle.brute_force(ctx["w"].base, ctx["w"].queries, ctx["r"], metric="ip")
    compare_float(g, o, ctx["r"], label="ip scan f32")
    np.testing.assert_allclose(rr.nn_dist(ctx["ix"], ctx["q"]).cpu().numpy(),
                               oracle.nn_dist(ctx["w"].base, ctx["w"].queries, metric="ip"),
                               rtol=1e-9)


def test_ip_float32_within_tolerance(rr, ip_f32):
    ctx = ip_f32
    r = ctx["r"]
    for mode, om in (("plain", oracle.PLAIN), ("es", oracle.ES), ("adaptive", oracle.ADAPTIVE),
                     ("doubling", oracle.DOUBLING)):
        flush_print(f"ip f32 {mode} r={r}")
        kw = dict(es_visit_limit=10, es_radius=r * 0.5)
        g = rr.range_search(ctx["ix"], ctx["q"], r, mode=mode, beam=16, max_beam=1024, **kw)
        o = _orc(ctx, mode=om, beam=16, max_beam=1024, **kw)
        compare_float(g, o, r, label=f"ip f32 {mode}")
        np.testing.assert_array_equal(g.stats["visits"], o.stats["visits"])
        assert len(o.ids) > 0


@pytest.mark.parametrize("mode,om", [("plain", oracle.PLAIN), ("adaptive", oracle.ADAPTIVE)])
def test_ip_bf16_recheck_sound(rr, ip_f32, mode, om):
    """bfloat16 pass under the inner product: returned points are inside the
    ball by the FP64 distance, carry that distance, are ordered by it, and
    recall stays close to the exact path's."""
    ctx = ip_f32
    r = ctx["r"]
    flush_print(f"ip bf16 {mode}")
    g = rr.range_search(ctx["ix"], ctx["q"], r, mode=mode, beam=24, precision=rr.BF16_RECHECK)
    e = rr.range_search(ctx["ix"], ctx["q"], r, mode=mode, beam=24)
    D = oracle.pair_dists(ctx["w"].base, ctx["w"].queries, metric="ip")
    off, ids, d = g.numpy()
    for qi in range(len(off) - 1):
        gi, gd = ids[off[qi]:off[qi + 1]], d[off[qi]:off[qi + 1]].astype(np.float64)
        assert np.all(D[qi, gi] <= r), f"q{qi}: point outside the ball"
        np.testing.assert_allclose(gd, D[qi, gi], rtol=1e-6, atol=1e-12)
        assert np.all(np.diff(gd) >= 0), f"q{qi} not ordered"
    bf = oracle.brute_force(ctx["w"].base, ctx["w"].queries, r, metric="ip")
    rec_b = oracle.range_recall(bf, oracle.Result(off, ids, d, None))
    eo, ei, ed = e.numpy()
    rec_e = oracle.range_recall(bf, oracle.Result(eo, ei, ed, None))
    flush_print(f"  recall bf16 {rec_b:.4f} exact {rec_e:.4f}, rechecked {g.stats['rechecked'].sum()}")
    assert rec_e >= 0.25 and rec_b >= rec_e - 0.02
    assert g.stats["truncated"].sum() == 0


@pytest.mark.parametrize("beam,step", [(8, 5), (32, 10), (16, 0)])
def test_ip_es_profile_matches_oracle(rr, ip_u8, beam, step):
    ctx = ip_u8
    flush_print(f"ip es profile beam={beam} step={step}")
    m, f = rr.es_profile(ctx["ix"], ctx["q"], ctx["r"], beam, step)
    om, of = oracle.es_profile(ctx["w"].base, ctx["adj"], ctx["entry"], ctx["w"].queries,
                               ctx["r"], beam, step, metric="ip")
    np.testing.assert_array_equal(f, of)
    np.testing.assert_array_equal(m, om)


def test_ip_served_equals_oracle(rr, ip_u8):
    """The serving loop under the inner product (a step budget suspends the
    searches between ticks)."""
    ctx = ip_u8
    w = ctx["w"]
    flush_print("ip serve")
    sp = rr.search_params(mode="adaptive", beam=12, es_enable=True, es_visit_limit=10,
                          es_radius=ctx["r"] * 0.5)
    got = {}
    with rr.Server(ctx["ix"], sp, slots=64, step_budget=3) as srv:
        for qi in range(len(w.queries)):
            assert srv.submit(w.queries[qi], float(ctx["r"]), qi)
        srv.drain(timeout=60.0)
        comps = srv.poll(len(w.queries) + 8)
        for c in comps:
            got[c.tag] = (srv.result(c.tag), c)
    o = _orc(ctx, mode=oracle.ADAPTIVE, beam=12, es_enable=True, es_visit_limit=10,
             es_radius=ctx["r"] * 0.5)
    assert len(got) == len(w.queries)
    for qi in range(len(w.queries)):
        (ids, d), c = got[qi]
        oi, od = o.query(qi)
        np.testing.assert_array_equal(ids, oi)
        np.testing.assert_array_equal(d.astype(np.int64), od.astype(np.int64))
        assert c.stats.visits == o.stats["visits"][qi]


def test_metric_is_fixed_on_device(rr, ip_u8):
    with pytest.raises(rr.RRError):
        ctx = ip_u8
        ctx["ix"].set_metric("l2")
