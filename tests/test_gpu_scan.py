"""GPU parity of the dense MFMA scan (ground truth of Definition 2.1 and
nearest-neighbour distances) against the CPU oracle's enumeration."""
import numpy as np
import pytest

import oracle
from paper_2502_13245_amd import synth
from tests.gpu_common import compare_float, flush_print

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_13245_amd import rr as _rr
    _rr.lib()
    return _rr


def _dummy_graph(n):
    return np.full((n, 1), -1, np.int32)


@pytest.mark.parametrize("d,signed,n,nq", [(128, False, 10000, 1000), (100, True, 5003, 77),
                                           (7, False, 3001, 130), (200, False, 2000, 65)])
def test_int_brute_force_and_nn_bit_exact(rr, d, signed, n, nq):
    w = synth.gaussian_mixture_int(n, nq, d, 40, 15.0, 31, signed=signed, spread=0.3)
    r = oracle.percentile_radius(w.base, w.queries, 0.003)
    ix = rr.Index.from_graph(w.base, _dummy_graph(n), 0).to_device("cuda:0")
    q = torch.from_numpy(w.queries).cuda()
    flush_print(f"scan d={d} signed={signed} n={n} nq={nq}")
    g = rr.brute_force(ix, q, r)
    o = oracle.brute_force(w.base, w.queries, r)
    off, ids, dd = g.numpy()
    np.testing.assert_array_equal(off, o.offsets)
    np.testing.assert_array_equal(ids, o.ids)
    np.testing.assert_array_equal(dd.astype(np.int64), o.dists.astype(np.int64))
    nn = rr.nn_dist(ix, q).cpu().numpy()
    np.testing.assert_array_equal(nn, oracle.nn_dist(w.base, w.queries))


def test_brute_force_per_query_radius_and_capacity_retry(rr):
    """Per-query radii (some negative) and a result count above the first
    capacity guess (the call re-sizes itself)."""
    w = synth.config_small_u8(0)
    D = oracle.pair_dists(w.base, w.queries[:300])
    r = np.quantile(D, 0.5, axis=1)
    r[::7] = -1.0
    ix = rr.Index.from_graph(w.base, _dummy_graph(len(w.base)), 0).to_device("cuda:0")
    q = torch.from_numpy(w.queries[:300]).cuda()
    flush_print("scan capacity retry")
    g = rr.brute_force(ix, q, torch.from_numpy(r))
    o = oracle.brute_force(w.base, w.queries[:300], r)
    assert o.offsets[-1] > (1 << 20)
    off, ids, dd = g.numpy()
    np.testing.assert_array_equal(off, o.offsets)
    np.testing.assert_array_equal(ids, o.ids)
    e = rr.brute_force(ix, q[:0], 1.0)
    assert e.offsets.cpu().tolist() == [0]


def test_float_brute_force_and_nn(rr):
    w = synth.gaussian_mixture_unit(6000, 150, 96, 30, 0.3 / np.sqrt(96), 8, spread=0.3)
    r = oracle.percentile_radius(w.base, w.queries, 0.003)
    ix = rr.Index.from_graph(w.base, _dummy_graph(len(w.base)), 0).to_device("cuda:0")
    q = torch.from_numpy(w.queries).cuda()
    flush_print("scan f32")
    g = rr.brute_force(ix, q, r)
    o = oracle.brute_force(w.base, w.queries, r)
    compare_float(g, o, r, rel=1e-5, label="bf f32")
    nn = rr.nn_dist(ix, q).cpu().numpy()
    np.testing.assert_allclose(nn, oracle.nn_dist(w.base, w.queries), rtol=1e-9, atol=1e-12)


def test_select_radius_matches_percentile_definition(rr):
    """rr_select_radius (count, collect, radix select on the GPU) against the
    oracle's enumeration of all pairs: the 10,000 x 1,000 uint8 workload's
    10^7 pairs at several percentiles (bit-exact, in one call), int8 with the
    inner product (negative radii), and float32 (FP64 distances within 1e-9)."""
    w = synth.config_small_u8(0)
    ix = rr.Index.from_graph(w.base, _dummy_graph(len(w.base)), 0).to_device("cuda:0")
    q = torch.from_numpy(w.queries).cuda()
    ps = [0.001, 0.0005, 1e-7, 0.02, 1.0]
    flush_print("select radius u8")
    got = rr.select_radius(ix, q, ps)
    want = [oracle.percentile_radius(w.base, w.queries, p) for p in ps]
    np.testing.assert_array_equal(got, want)
    assert rr.select_radius(ix, q, 0.001) == want[0]
    wi = synth.gaussian_mixture_int(4000, 90, 100, 30, 12.0, 9, signed=True, spread=0.3)
    ixi = rr.Index.from_graph(wi.base, _dummy_graph(4000), 0, metric="ip").to_device("cuda:0")
    qi = torch.from_numpy(wi.queries).cuda()
    flush_print("select radius i8 ip")
    for p in (0.002, 0.3):
        assert rr.select_radius(ixi, qi, p) == oracle.percentile_radius(wi.base, wi.queries, p,
                                                                        metric="ip")
    wf = synth.latent_mixture_f32(6000, 120, 96, 40, 0.35, 14)
    ixf = rr.Index.from_graph(wf.base, _dummy_graph(6000), 0).to_device("cuda:0")
    qf = torch.from_numpy(wf.queries).cuda()
    flush_print("select radius f32")
    for p in (0.0005, 0.01):
        np.testing.assert_allclose(rr.select_radius(ixf, qf, p),
                                   oracle.percentile_radius(wf.base, wf.queries, p), rtol=1e-9)
    with pytest.raises(rr.RRError):
        rr.select_radius(ix, q, 0.0)
