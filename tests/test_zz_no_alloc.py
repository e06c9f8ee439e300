"""rr_range_search_noalloc (the entry point for callers that cannot
allocate device memory) against rr_range_search on the same inputs, called
through the C ABI: two calls in a row, the second with a smaller input, each
bit-exact in offsets, ids, distances and per-query counters (integer data);
a capacity below the total leaves the tail unwritten; a request that does
not fit the scratch array is refused before anything runs."""
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
def ctx(rr):
    w = synth.config_small_u8(0)
    adj, entry = oracle.build_vamana(w.base, 32, 64, 1.2, synth.permutation(len(w.base), 0))
    r = oracle.percentile_radius(w.base, w.queries, 0.001)
    ix = rr.Index.from_graph(w.base, adj, entry).to_device("cuda:0")
    q = torch.from_numpy(w.queries).cuda()
    return dict(w=w, r=r, ix=ix, q=q)


def _same(rr, ref, got, label):
    off, ids, d = ref.numpy()
    g_off, g_ids, g_d, g_st = got
    total = int(off[-1])
    np.testing.assert_array_equal(g_off.cpu().numpy(), off, err_msg=f"{label} offsets")
    np.testing.assert_array_equal(g_ids[:total].cpu().numpy(), ids, err_msg=f"{label} ids")
    np.testing.assert_array_equal(g_d[:total].cpu().numpy(), d, err_msg=f"{label} dists")
    st = rr.stats_from_bytes(g_st)
    for f in ("visits", "evals", "greedy_visits", "greedy_evals", "count", "es_fired",
              "expanded", "truncated", "edges", "greedy_edges"):
        np.testing.assert_array_equal(st[f], ref.stats[f], err_msg=f"{label} {f}")


@pytest.mark.parametrize("mode,beam,es", [("adaptive", 8, True), ("adaptive", 2, True),
                                          ("plain", 32, False)])
def test_noalloc_equals_range_search_twice(rr, ctx, mode, beam, es):
    kw = dict(mode=mode, beam=beam, es_enable=es, es_visit_limit=3, es_radius=ctx["r"] * 15)
    for n in (len(ctx["w"].queries), 377):
        flush_print(f"noalloc {mode} b={beam} nq={n}")
        q = ctx["q"][:n]
        ref = rr.range_search(ctx["ix"], q, ctx["r"], **kw)
        got = rr.range_search_noalloc(ctx["ix"], q, ctx["r"], capacity=200_000, **kw)
        torch.cuda.synchronize()
        _same(rr, ref, got, f"{mode} b={beam} nq={n}")


def test_noalloc_capacity_and_refusal(rr, ctx):
    kw = dict(mode="adaptive", beam=4)
    ref = rr.range_search(ctx["ix"], ctx["q"], ctx["r"], **kw)
    off, ids, d = ref.numpy()
    total = int(off[-1])
    assert total > 10
    cap = total // 2
    flush_print(f"noalloc capacity {cap} of {total}")
    g_off, g_ids, g_d, _ = rr.range_search_noalloc(ctx["ix"], ctx["q"], ctx["r"], capacity=cap,
                                                   with_stats=False, **kw)
    g_ids.fill_(-7)
    g_off, g_ids2, g_d2, _ = rr.range_search_noalloc(ctx["ix"], ctx["q"], ctx["r"], capacity=cap,
                                                     with_stats=False, **kw)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(g_off.cpu().numpy(), off)
    np.testing.assert_array_equal(g_ids2[:cap].cpu().numpy(), ids[:cap])
    np.testing.assert_array_equal(g_d2[:cap].cpu().numpy(), d[:cap])
    # more than the scratch array holds: refused with a clear error
    with pytest.raises(rr.RRError) as e:
        rr.range_search_noalloc(ctx["ix"], ctx["q"], ctx["r"], capacity=16, mode="adaptive",
                                beam=8, result_capacity=1 << 26)
    assert "scratch" in str(e.value)
    with pytest.raises(rr.RRError):
        rr.range_search_noalloc(ctx["ix"], ctx["q"], ctx["r"], capacity=16, mode="doubling", beam=8)
