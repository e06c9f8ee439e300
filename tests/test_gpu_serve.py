"""GPU parity of the serving loop (continuous batching with resumable beam
searches) against the CPU oracle and the batched search.

A served query may be suspended and resumed many times and shares each tick
with whatever else is resident; its result must not change: ids, distances
and the beam-phase visit counts equal the oracle's for integer data.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2502_13245_amd import synth
from tests.gpu_common import flush_print

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_13245_amd import rr as _rr
    _rr.lib()
    return _rr


@pytest.fixture(scope="module")
def nav(rr):
    """8,000 x 128 uint8 base (low intrinsic dimension), 600 queries,
    radius with 75% of the queries empty, per-query radii mixed in."""
    w = synth.latent_mixture_u8(8000, 600, 128, 60, 25.0, 31)
    adj, entry = oracle.build_vamana(w.base, 32, 64, 1.2, synth.permutation(8000, 31))
    r = oracle.empty_fraction_radius(w.base, w.queries, 0.25)
    rng = np.random.default_rng(31)
    radii = r * rng.choice([1.0, 1.0, 1.0, 2.0, 0.0, -1.0], size=len(w.queries))
    ix = rr.Index.from_graph(w.base, adj, entry).to_device("cuda:0")
    return dict(w=w, adj=adj, entry=entry, r=r, radii=radii, ix=ix)


def _serve(rr, ctx, params, slots, budget, radii, order=None, bursts=1, pause=0.0):
    w = ctx["w"]
    nq = len(w.queries)
    order = np.arange(nq) if order is None else order
    out = {}
    with rr.Server(ctx["ix"], params, slots=slots, step_budget=budget) as srv:
        for chunk in np.array_split(order, bursts):
            for qi in chunk:
                assert srv.submit(w.queries[qi], float(radii[qi]), int(qi) + 1000)
            if pause:
                time.sleep(pause)
        srv.drain(timeout=60.0)
        comps = []
        while True:
            c = srv.poll()
            if not c:
                break
            comps.extend(c)
        info = srv.info()
        for c in comps:
            ids, d = srv.result(c.tag)
            out[c.tag - 1000] = (ids, d, c)
    assert len(out) == nq and info["completed"] == nq and info["submitted"] == nq
    return out, info


def _check_vs_oracle(out, o, label):
    for q in range(len(out)):
        ids, d, c = out[q]
        oi, od = o.query(q)
        np.testing.assert_array_equal(ids, oi, err_msg=f"{label} q{q} ids")
        np.testing.assert_array_equal(d.astype(np.int64), od.astype(np.int64),
                                      err_msg=f"{label} q{q} dists")
        assert c.count == len(oi)
        assert c.stats.visits == o.stats["visits"][q], f"{label} q{q} visits"
        assert c.stats.es_fired == o.stats["es_fired"][q], f"{label} q{q} es"
        assert c.stats.expanded == o.stats["expanded"][q], f"{label} q{q} expanded"
        assert c.stats.greedy_visits == o.stats["greedy_visits"][q]
        assert c.truncated == 0
        assert c.t_arrival <= c.t_admit <= c.t_done


@pytest.mark.parametrize("slots,budget", [(64, 3), (1000, 0), (7, 1)])
def test_served_adaptive_es_equals_oracle(rr, nav, slots, budget):
    """Fewer slots than requests (queueing), a step budget that suspends
    most searches many times, per-query radii incl. 0 and negative."""
    flush_print(f"serve adaptive slots={slots} budget={budget}")
    es = dict(es_enable=True, es_visit_limit=10, es_radius=nav["r"])
    sp = rr.search_params(mode="adaptive", beam=12, **es)
    out, info = _serve(rr, nav, sp, slots, budget, nav["radii"])
    o = oracle.range_search(nav["w"].base, nav["adj"], nav["entry"], nav["w"].queries,
                            nav["radii"], mode=oracle.ADAPTIVE, beam=12, **es)
    _check_vs_oracle(out, o, f"s={slots} b={budget}")
    ticks = np.array([out[q][2].ticks for q in range(len(out))])
    flush_print(f"  ticks {info['ticks']} max resident {info['max_resident']} "
                f"per-query ticks max {ticks.max()}")
    assert info["max_resident"] <= slots
    if budget:
        # a query resident for t ticks made at most t * budget visits
        visits = np.array([out[q][2].stats.visits for q in range(len(out))])
        assert np.all(visits <= ticks * budget)
        assert ticks.max() > 1


def test_served_plain_and_es_staggered(rr, nav):
    """Requests arrive in bursts while earlier ones are on the device."""
    w = nav["w"]
    order = np.random.default_rng(3).permutation(len(w.queries))
    for mode, om, kw in (("plain", oracle.PLAIN, {}),
                         ("es", oracle.ES, dict(es_visit_limit=5, es_radius=nav["r"] * 1.5))):
        flush_print(f"serve {mode} staggered")
        sp = rr.search_params(mode=mode, beam=48, **kw)
        out, _ = _serve(rr, nav, sp, 128, 8, nav["radii"], order=order, bursts=6, pause=0.01)
        o = oracle.range_search(w.base, nav["adj"], nav["entry"], w.queries, nav["radii"],
                                mode=om, beam=48, **kw)
        _check_vs_oracle(out, o, mode)


def test_served_bf16_equals_batched(rr):
    """float32 data, bf16 first pass with exact recheck: the served result
    of every query is the batched result, byte for byte."""
    w = synth.latent_mixture_f32(4000, 300, 96, 40, 0.35, 41)
    adj, entry = oracle.build_vamana(w.base, 32, 64, 1.2, synth.permutation(4000, 41))
    r = oracle.percentile_radius(w.base, w.queries, 0.002)
    ix = rr.Index.from_graph(w.base, adj, entry).to_device("cuda:0")
    q = torch.from_numpy(w.queries).cuda()
    for prec in (rr.EXACT, rr.BF16_RECHECK):
        flush_print(f"serve f32 precision={prec}")
        sp = rr.search_params(mode="adaptive", beam=16, precision=prec)
        g = rr.range_search(ix, q, r, params=sp)
        off, ids, d = g.numpy()
        assert len(ids) > 0
        ctx = dict(w=w, ix=ix)
        out, _ = _serve(rr, ctx, sp, 50, 2, np.full(len(w.queries), r))
        for qi in range(len(w.queries)):
            si, sd, c = out[qi]
            np.testing.assert_array_equal(si, ids[off[qi]:off[qi + 1]])
            np.testing.assert_array_equal(sd, d[off[qi]:off[qi + 1]])
            assert c.stats.visits == g.stats["visits"][qi]


def test_shared_capacity_overflow_is_retried_alone(rr, nav):
    """A tick's greedy items and result arena are shared by its queries.  The
    queries chosen here each fit the capacity alone while any two of them
    overflow it, so every tick holding two of them overflows; the queries it
    cut are run again in ticks of their own, and every served result equals
    the oracle with no truncation flag.  With a capacity below the largest
    result, that query comes back truncated even alone, and the queries that
    fit stay exact."""
    w = nav["w"]
    b = 2
    sp = rr.search_params(mode="adaptive", beam=b)
    o = oracle.range_search(w.base, nav["adj"], nav["entry"], w.queries, nav["radii"],
                            mode=oracle.ADAPTIVE, beam=b)
    counts = np.diff(o.offsets)
    # C: the largest result a tick can hold; chosen queries have counts in
    # [C/2 + 5, C], so any two exceed C + 8
    sel = None
    for c in sorted(set(counts.tolist()), reverse=True):
        cand = np.flatnonzero((counts >= c // 2 + 5) & (counts <= c))
        if len(cand) >= 8:
            sel, cap_items = cand, c
            break
    assert sel is not None, "the workload has too few heavy queries"
    slots = len(sel)
    gcap = cap_items + 8 - slots * b  # item and arena capacity = slots * b + gcap = C + 8
    assert gcap >= 1
    flush_print(f"serve overflow: {slots} queries with {counts[sel].min()}..{counts[sel].max()} "
                f"results, capacity {cap_items + 8}")
    reps = 4  # every chosen query is submitted 4 times, so ticks hold several
    with rr.Server(nav["ix"], sp, slots=slots, result_capacity=gcap) as srv:
        for k in range(reps):
            for qi in sel:
                assert srv.submit(w.queries[qi], float(nav["radii"][qi]), k * 100000 + int(qi))
        srv.drain(timeout=120.0)
        comps = {c.tag: c for c in srv.poll(reps * slots + 8)}
        got = {t: srv.result(t) for t in comps}
        info = srv.info()
    flush_print(f"  retried {info['retried']}, ticks {info['ticks']}")
    assert info["retried"] > 0 and len(comps) == reps * slots
    for tag, c in comps.items():
        oi, od = o.query(tag % 100000)
        assert c.truncated == 0, f"request {tag} truncated"
        np.testing.assert_array_equal(got[tag][0], oi, err_msg=f"request {tag} ids")
        np.testing.assert_array_equal(got[tag][1].astype(np.int64), od.astype(np.int64))
    # a capacity below the heaviest result: that query is truncated even alone
    heavy = int(np.argmax(counts))
    light = np.flatnonzero((counts > 0) & (counts <= 8))[:20]
    with rr.Server(nav["ix"], sp, slots=4, result_capacity=int(counts[heavy]) // 2) as srv:
        for qi in [heavy] + light.tolist():
            assert srv.submit(w.queries[qi], float(nav["radii"][qi]), int(qi))
        srv.drain(timeout=120.0)
        comps = {c.tag: c for c in srv.poll(64)}
        got = {t: srv.result(t) for t in comps}
    assert comps[heavy].truncated == 1
    for qi in light:
        oi, od = o.query(int(qi))
        assert comps[qi].truncated == 0, f"q{qi} truncated"
        np.testing.assert_array_equal(got[qi][0], oi, err_msg=f"q{qi} ids")


def test_server_errors(rr, nav):
    sp = rr.search_params(mode="adaptive", beam=8)
    with pytest.raises(rr.RRError):
        rr.Server(nav["ix"], sp, slots=0)
    with pytest.raises(rr.RRError):
        rr.Server(nav["ix"], rr.search_params(mode="doubling", beam=8))
    with rr.Server(nav["ix"], sp, slots=4, max_pending=2) as srv:
        with pytest.raises(ValueError):
            srv.submit(nav["w"].queries[0][:5], 1.0, 1)
        with pytest.raises(rr.RRError):
            srv.submit(nav["w"].queries[0], float("nan"), 1)
        with pytest.raises(rr.RRError):
            srv.result(12345)
        accepted = [t for t in range(200) if srv.submit(nav["w"].queries[t], nav["r"], t)]
        srv.drain(timeout=30.0)
        got = sorted(c.tag for c in srv.poll(1000))
        assert got == accepted and len(accepted) >= 2
        for t in accepted:
            srv.result(t)
        with pytest.raises(rr.RRError):
            srv.result(accepted[0])  # results are released once fetched


def test_admission_by_footprint(rr, nav):
    """slots = 0: the slot count is the largest whose buffers fit the given
    device-memory budget; served results are unchanged."""
    sp = rr.search_params(mode="adaptive", beam=12)
    with pytest.raises(rr.RRError):
        rr.Server(nav["ix"], sp, slots=0, hbm_budget=1000)
    with pytest.raises(rr.RRError):
        rr.Server(nav["ix"], sp, slots=0)
    budgets = []
    for budget in (64 << 20, 256 << 20):
        with rr.Server(nav["ix"], sp, slots=0, hbm_budget=budget) as srv:
            inf = srv.info()
            assert 1 <= inf["slots"] and inf["device_bytes"] <= budget
            budgets.append(inf["slots"])
    assert budgets[1] > budgets[0]
    flush_print(f"footprint admission: slots {budgets}")
    w = nav["w"]
    with rr.Server(nav["ix"], sp, slots=0, hbm_budget=64 << 20, step_budget=4) as srv:
        for qi in range(len(w.queries)):
            assert srv.submit(w.queries[qi], float(nav["radii"][qi]), qi)
        srv.drain(timeout=60.0)
        got = {c.tag: srv.result(c.tag) for c in srv.poll(len(w.queries) + 8)}
    o = oracle.range_search(w.base, nav["adj"], nav["entry"], w.queries, nav["radii"],
                            mode=oracle.ADAPTIVE, beam=12)
    for qi in range(len(w.queries)):
        oi, od = o.query(qi)
        np.testing.assert_array_equal(got[qi][0], oi)
        np.testing.assert_array_equal(got[qi][1].astype(np.int64), od.astype(np.int64))
