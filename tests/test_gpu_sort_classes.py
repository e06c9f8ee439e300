"""GPU parity of the result-list sort at the edges of its size classes.

The finalization sorts each list by the smallest unit that holds it: one
wave in registers (up to 64 entries), one wave in LDS (up to 512; 256 for
FP64 distances), a whole workgroup in LDS (up to 8,192; 4,096), and merge
passes through global memory beyond that.  Brute-force range search sends
every query's in-ball points through the same sort, so queries whose balls
hold exactly these counts test each edge.

Each list is a cluster: the query is 255 on one coordinate, and its points
add 1, 2 or 3 on one of 64 other coordinates, so their squared distances are
1, 4 or 9 (exact in integer and in FP64 arithmetic) and every other cluster
is far outside the radius 9.  Ids are shuffled, so the many equal distances
test the (distance, id) order.  The oracle's brute force (the definition of
the range search) is the reference; lists must match entry for entry."""
import numpy as np
import pytest

import oracle
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


def _clusters(sizes, dtype, seed):
    d = 128
    pts, qs = [], []
    for c, k in enumerate(sizes):
        q = np.zeros(d, np.int64)
        q[c] = 255
        qs.append(q)
        j = np.arange(k)
        p = np.tile(q, (k, 1))
        p[j, 64 + j % 64] = 1 + (j // 64) % 3
        pts.append(p)
    base = np.concatenate(pts)
    perm = np.random.default_rng(seed).permutation(len(base))
    return base[perm].astype(dtype), np.stack(qs).astype(dtype)


def _check(rr, base, queries, sizes, label):
    ix = rr.Index.from_graph(base, np.full((len(base), 1), -1, np.int32), 0).to_device("cuda:0")
    q = torch.from_numpy(queries).cuda()
    flush_print(f"sort classes {label}: list sizes {sizes}")
    g = rr.brute_force(ix, q, 9.0)
    o = oracle.brute_force(base, queries, 9.0)
    np.testing.assert_array_equal(np.diff(o.offsets), np.asarray(sizes))
    off, ids, dd = g.numpy()
    np.testing.assert_array_equal(off, o.offsets)
    np.testing.assert_array_equal(ids, o.ids)
    np.testing.assert_array_equal(dd.astype(np.float64), o.dists.astype(np.float64))


def test_sort_class_edges_u8(rr):
    """32-bit distances: edges at 64, 512 and 8,192 entries, one list past
    two merge passes, and an empty one."""
    sizes = [0, 1, 2, 63, 64, 65, 100, 511, 512, 513, 1000, 8191, 8192, 8193, 16385, 20000]
    base, queries = _clusters(sizes, np.uint8, 7)
    _check(rr, base, queries, sizes, "u8")


def test_sort_class_edges_f32(rr):
    """FP64 distances (float data): edges at 64, 256 and 4,096 entries."""
    sizes = [0, 1, 64, 65, 255, 256, 257, 4095, 4096, 4097, 9000]
    base, queries = _clusters(sizes, np.float32, 8)
    _check(rr, base, queries, sizes, "f32")
