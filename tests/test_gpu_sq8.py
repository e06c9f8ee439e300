"""GPU tests of the 8-bit scalar-quantized first pass with exact re-decision
(the paper's setting for float data, Section 5).

The quantized traversal may visit other points than the exact one, so the
result is not compared with the oracle's element by element. What is fixed
is: every returned point is inside the ball by the oracle's FP64 distance,
its reported distance is that distance, lists are ordered by it, recall is
close to the exact path's, and the served result equals the batched one.
"""
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


def _workload(n, nq, d, seed, spread_norms):
    w = synth.latent_mixture_f32(n, nq, d, 40, 0.35, seed)
    if spread_norms:
        rng = np.random.default_rng(seed)
        w.base[:] = w.base * rng.uniform(0.5, 2.0, (n, 1)).astype(np.float32)
        w.queries[:] = w.queries * rng.uniform(0.5, 2.0, (nq, 1)).astype(np.float32)
    adj, entry = oracle.build_vamana(w.base, 32, 64, 1.2, synth.permutation(n, seed))
    return w, adj, entry


def _check_sound(rr, w, ix, r, mode, metric, beam, min_recall_gap=0.05):
    q = torch.from_numpy(w.queries).cuda()
    g = rr.range_search(ix, q, r, mode=mode, beam=beam, precision=rr.SQ8_RERANK)
    e = rr.range_search(ix, q, r, mode=mode, beam=beam)
    D = oracle.pair_dists(w.base, w.queries, metric=metric)
    off, ids, d = g.numpy()
    for qi in range(len(off) - 1):
        gi, gd = ids[off[qi]:off[qi + 1]], d[off[qi]:off[qi + 1]].astype(np.float64)
        assert np.all(D[qi, gi] <= r), f"q{qi}: point outside the ball"
        assert len(np.unique(gi)) == len(gi), f"q{qi}: repeated id"
        np.testing.assert_allclose(gd, D[qi, gi], rtol=1e-6, atol=1e-12)
        assert np.all(np.diff(gd) >= 0), f"q{qi} not ordered"
    assert g.stats["truncated"].sum() == 0
    bf = oracle.brute_force(w.base, w.queries, r, metric=metric)
    rec_q = oracle.range_recall(bf, oracle.Result(off, ids, d, None))
    eo, ei, ed = e.numpy()
    rec_e = oracle.range_recall(bf, oracle.Result(eo, ei, ed, None))
    flush_print(f"  recall sq8 {rec_q:.4f} exact {rec_e:.4f}, band {g.stats['rechecked'].sum()}, "
                f"results {len(ids)}")
    assert rec_e >= 0.25 and rec_q >= rec_e - min_recall_gap
    return g


@pytest.mark.parametrize("mode", ["plain", "adaptive"])
def test_sq8_l2_sound(rr, mode):
    w, adj, entry = _workload(8000, 400, 96, 71, False)
    r = oracle.percentile_radius(w.base, w.queries, 0.002)
    ix = rr.Index.from_graph(w.base, adj, entry).to_device("cuda:0")
    flush_print(f"sq8 l2 {mode}")
    _check_sound(rr, w, ix, r, mode, "l2", 24)


@pytest.mark.parametrize("mode", ["plain", "adaptive"])
def test_sq8_inner_product_sound(rr, mode):
    w, adj, entry = _workload(4000, 300, 96, 73, True)
    r = oracle.percentile_radius(w.base, w.queries, 0.003, metric="ip")
    ix = rr.Index.from_graph(w.base, adj, entry, metric="ip").to_device("cuda:0")
    flush_print(f"sq8 ip {mode}")
    _check_sound(rr, w, ix, r, mode, "ip", 24)


def test_sq8_wide_rows_and_ragged_dim(rr):
    """d=768 (codes split over 16 lanes, 3 chunks each) and d=37 (padded)."""
    for d, n in ((768, 3000), (37, 4000)):
        w, adj, entry = _workload(n, 150, d, 75 + d, False)
        r = oracle.percentile_radius(w.base, w.queries, 0.003)
        ix = rr.Index.from_graph(w.base, adj, entry).to_device("cuda:0")
        flush_print(f"sq8 d={d}")
        _check_sound(rr, w, ix, r, "adaptive", "l2", 16)


def test_sq8_served_equals_batched(rr):
    w, adj, entry = _workload(4000, 200, 96, 77, False)
    r = oracle.percentile_radius(w.base, w.queries, 0.002)
    ix = rr.Index.from_graph(w.base, adj, entry).to_device("cuda:0")
    sp = rr.search_params(mode="adaptive", beam=16, precision=rr.SQ8_RERANK)
    g = rr.range_search(ix, torch.from_numpy(w.queries).cuda(), r, params=sp)
    off, ids, d = g.numpy()
    flush_print("sq8 serve")
    got = {}
    with rr.Server(ix, sp, slots=50, step_budget=2) as srv:
        for qi in range(len(w.queries)):
            assert srv.submit(w.queries[qi], float(r), qi)
        srv.drain(timeout=60.0)
        for c in srv.poll(len(w.queries) + 8):
            got[c.tag] = (srv.result(c.tag), c)
    assert len(got) == len(w.queries)
    for qi in range(len(w.queries)):
        (si, sd), c = got[qi]
        np.testing.assert_array_equal(si, ids[off[qi]:off[qi + 1]])
        np.testing.assert_array_equal(sd, d[off[qi]:off[qi + 1]])
        assert c.stats.visits == g.stats["visits"][qi]


def test_sq8_needs_float_data(rr):
    w = synth.gaussian_mixture_int(500, 10, 32, 5, 12.0, 3)
    ix = rr.Index.from_graph(w.base, synth.random_graph(500, 8, 3), 0).to_device("cuda:0")
    with pytest.raises(rr.RRError):
        rr.range_search(ix, torch.from_numpy(w.queries).cuda(), 1000.0,
                        precision=rr.SQ8_RERANK)
