"""Shared helpers for the GPU parity tests (imported by tests only)."""
import numpy as np

import oracle


def flush_print(*a):
    print(*a, flush=True)


def compare_exact(gpu, orc, check_evals=True, label=""):
    """Bit-exact comparison of a GPU result with the oracle's on integer data:
    offsets, ids, distances and per-query visit counters."""
    off, ids, dists = gpu.numpy()
    np.testing.assert_array_equal(off, orc.offsets, err_msg=f"{label} offsets")
    np.testing.assert_array_equal(ids, orc.ids, err_msg=f"{label} ids")
    np.testing.assert_array_equal(dists.astype(np.int64), orc.dists.astype(np.int64),
                                  err_msg=f"{label} dists")
    gs, os_ = gpu.stats, orc.stats
    np.testing.assert_array_equal(gs["visits"], os_["visits"], err_msg=f"{label} visits")
    np.testing.assert_array_equal(gs["es_fired"], os_["es_fired"], err_msg=f"{label} es_fired")
    np.testing.assert_array_equal(gs["expanded"], os_["expanded"], err_msg=f"{label} expanded")
    np.testing.assert_array_equal(gs["greedy_visits"], os_["greedy_visits"],
                                  err_msg=f"{label} greedy visits")
    np.testing.assert_array_equal(gs["count"], np.diff(orc.offsets), err_msg=f"{label} count")
    assert not gs["truncated"].any(), f"{label} truncated"
    if check_evals:
        ok = gs["cache_overflow"] == 0
        np.testing.assert_array_equal(gs["evals"][ok], os_["evals"][ok], err_msg=f"{label} evals")
        np.testing.assert_array_equal(gs["greedy_evals"], os_["greedy_evals"],
                                      err_msg=f"{label} greedy evals")


def check_greedy_edges(gpu, adj, label=""):
    """greedy_edges of a query that expanded counts the adjacency entries its
    greedy phase scanned: each in-ball point it visited is expanded once
    (Algorithm 2), and with nothing truncated those points are exactly the
    returned list, so the count is the sum of their out-degrees in the graph;
    a query that did not expand reports 0."""
    off, ids, _ = gpu.numpy()
    deg = (np.asarray(adj) >= 0).sum(axis=1).astype(np.int64)
    st = gpu.stats
    assert not st["truncated"].any(), f"{label} truncated"
    for q in range(len(off) - 1):
        want = int(deg[ids[off[q]:off[q + 1]]].sum()) if st["expanded"][q] else 0
        assert int(st["greedy_edges"][q]) == want, f"{label} q{q} greedy_edges"


def compare_float(gpu, orc, radius, rel=1e-5, label=""):
    """Float data: distances within `rel` (relative) of the FP64 oracle and
    equal result sets outside a +-rel band around the radius."""
    off, ids, dists = gpu.numpy()
    r = np.broadcast_to(np.asarray(radius, np.float64), (len(off) - 1,))
    for q in range(len(off) - 1):
        g_ids = ids[off[q]:off[q + 1]]
        g_d = dists[off[q]:off[q + 1]].astype(np.float64)
        o_ids, o_d = orc.query(q)
        common, gi, oi = np.intersect1d(g_ids, o_ids, return_indices=True)
        np.testing.assert_allclose(g_d[gi], o_d[oi], rtol=rel, atol=1e-12,
                                   err_msg=f"{label} q{q} dists")
        only_g = np.setdiff1d(g_ids, o_ids)
        only_o = np.setdiff1d(o_ids, g_ids)
        for s, dd, idl in ((only_g, g_d, g_ids), (only_o, o_d, o_ids)):
            for x in s:
                dx = dd[np.flatnonzero(idl == x)[0]]
                assert abs(dx - r[q]) <= rel * abs(r[q]), f"{label} q{q}: id {x} at {dx} outside band"
