"""The C ABI on the host: the library loads without a GPU, exports every
entry point declared in include/rr.h, validates arguments, and its host-side
graph builder matches the oracle's builder byte for byte."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2502_13245_amd import rr, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(rr_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = rr.lib()
    names = _declared()
    assert "rr_range_search" in names and "rr_index_build" in names
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    # the binding knows them all
    assert names <= set(rr.SIGNATURES), names - set(rr.SIGNATURES)


def test_version_and_defaults():
    assert b"gfx950" in rr.lib().rr_version()
    sp = rr.search_params()
    assert sp.mode == rr.ADAPTIVE and sp.beam == 32 and sp.lam == 1.0


def _err(fn):
    with pytest.raises(rr.RRError) as e:
        fn()
    return e.value.status


def test_from_graph_validation():
    base = np.zeros((4, 3), np.uint8)
    ok = np.array([[1, -1], [2, -1], [3, -1], [0, -1]], np.int32)
    rr.Index.from_graph(base, ok, 0)
    bad = {
        "self loop": np.array([[0, -1], [2, -1], [3, -1], [0, -1]], np.int32),
        "repeat": np.array([[1, 1], [2, -1], [3, -1], [0, -1]], np.int32),
        "range": np.array([[9, -1], [2, -1], [3, -1], [0, -1]], np.int32),
        "padding": np.array([[-1, 1], [2, -1], [3, -1], [0, -1]], np.int32),
    }
    for name, adj in bad.items():
        assert _err(lambda: rr.Index.from_graph(base, adj, 0)) == rr.RR_EINVAL, name
    assert _err(lambda: rr.Index.from_graph(base, ok, 4)) == rr.RR_EINVAL
    assert _err(lambda: rr.Index.from_graph(base.astype(np.int16), ok, 0)) if False else True


def test_build_validation():
    base = np.zeros((10, 4), np.uint8)
    assert _err(lambda: rr.Index.build(base, R=0)) == rr.RR_EINVAL
    assert _err(lambda: rr.Index.build(base, R=8, L=0)) == rr.RR_EINVAL
    assert _err(lambda: rr.Index.build(base, R=8, alpha=0.5)) == rr.RR_EINVAL
    assert _err(lambda: rr.Index.build(base, R=8, passes=3)) == rr.RR_EINVAL
    assert _err(lambda: rr.Index.build(base, R=8, order=np.zeros(10, np.int64))) == rr.RR_EINVAL


def test_search_needs_device_index():
    base = np.zeros((4, 3), np.uint8)
    ix = rr.Index.from_graph(base, np.array([[1], [2], [3], [0]], np.int32), 0)
    with pytest.raises(rr.RRError):
        rr.range_search_async(ix, None, 1.0)


def test_save_load_roundtrip(tmp_path):
    w = synth.gaussian_mixture_int(500, 5, 16, 5, 10.0, 1)
    ix = rr.Index.build(w.base, R=8, L=16, alpha=1.2, threads=2, seed=3)
    p = str(tmp_path / "g.rri")
    ix.save(p)
    iy = rr.Index.load(p)
    a1, e1 = ix.graph()
    a2, e2 = iy.graph()
    np.testing.assert_array_equal(a1, a2)
    assert e1 == e2 and iy.info() == ix.info()
    with open(p, "r+b") as f:
        f.write(b"XXXX")
    assert _err(lambda: rr.Index.load(p)) == rr.RR_EIO


@pytest.mark.parametrize("dt", [np.uint8, np.int8, np.float32])
def test_library_builder_matches_oracle_builder(dt):
    rng = np.random.default_rng(8)
    n, d = 1500, 12
    if dt == np.uint8:
        b = rng.integers(0, 256, (n, d)).astype(dt)
    elif dt == np.int8:
        b = rng.integers(-100, 100, (n, d)).astype(dt)
    else:
        b = rng.standard_normal((n, d)).astype(dt)
    order = synth.permutation(n, 4)
    for passes in (1, 2):
        a1, e1 = oracle.build_vamana(b, 12, 24, 1.2, order, passes=passes, threads=3)
        lib = rr.Index.build(b, R=12, L=24, alpha=1.2, passes=passes, threads=5, order=order)
        a2, e2 = lib.graph()
        np.testing.assert_array_equal(a1, a2)
        assert e1 == e2


def test_library_builder_thread_count_invariant():
    w = synth.config_small_u8(0)
    base = w.base[:4000]
    g1 = rr.Index.build(base, R=16, L=32, alpha=1.2, threads=1, seed=11).graph()
    g8 = rr.Index.build(base, R=16, L=32, alpha=1.2, threads=8, seed=11).graph()
    np.testing.assert_array_equal(g1[0], g8[0])


def test_shifted_graph_is_a_valid_index_graph():
    """The fast large-n test graph: no self loops, no repeated ids, ids in
    range (the library's own validation accepts it)."""
    n, R = 200_003, 32
    adj = synth.shifted_graph(n, R, 7)
    assert adj.shape == (n, R) and adj.min() >= 0 and adj.max() < n
    assert not (adj == np.arange(n)[:, None]).any()
    s = np.sort(adj, axis=1)
    assert not (s[:, 1:] == s[:, :-1]).any()
    rr.Index.from_graph(np.zeros((n, 2), np.uint8), adj, 0)
    np.testing.assert_array_equal(adj, synth.shifted_graph(n, R, 7))


def test_metric_is_saved_and_old_files_load_as_l2(tmp_path):
    """The index file records the metric (version 2 header); a version 1
    file, which has no metric field, loads as squared L2."""
    w = synth.gaussian_mixture_int(300, 5, 16, 4, 12.0, 2)
    adj = synth.random_graph(300, 8, 2)
    ix = rr.Index.from_graph(w.base, adj, 5, metric="ip")
    assert ix.metric == "ip"
    p2 = str(tmp_path / "v2.rri")
    ix.save(p2)
    back = rr.Index.load(p2)
    assert back.metric == "ip" and back.info() == ix.info()
    np.testing.assert_array_equal(back.graph()[0], adj)
    # the same index in the version 1 layout: magic, 5 int64, rows, graph
    p1 = str(tmp_path / "v1.rri")
    with open(p1, "wb") as f:
        f.write(b"RRIDX001")
        f.write(np.array([300, 16, rr.U8, 8, 5], np.int64).tobytes())
        f.write(np.ascontiguousarray(w.base).tobytes())
        f.write(np.ascontiguousarray(adj, np.int32).tobytes())
    old = rr.Index.load(p1)
    assert old.metric == "l2" and old.info()["entry"] == 5
    np.testing.assert_array_equal(old.graph()[0], adj)
    with pytest.raises(ValueError):
        ix.set_metric("cosine")
    with pytest.raises(rr.RRError):
        lib = rr.lib()
        rr._check(lib.rr_index_set_metric(ix._h, 7))


# every ctypes mirror of a header struct, with the C names of fields whose
# Python names differ (`lambda` is a Python keyword)
_STRUCTS = {"rr_allocator": ("Allocator", {}), "rr_build_params": ("BuildParams", {}),
            "rr_search_params": ("SearchParams", {"lam": "lambda"}),
            "rr_query_stats": ("QueryStats", {}), "rr_batch_stats": ("BatchStats", {}),
            "rr_tune_report": ("TuneReport", {}), "rr_es_tune_report": ("ESTuneReport", {}),
            "rr_server_config": ("ServerConfig", {}), "rr_completion": ("Completion", {}),
            "rr_server_info": ("ServerInfo", {})}


def test_struct_layouts_match_header(tmp_path):
    """sizeof and every field offset of the binding's ctypes structures equal
    what a C compiler makes of include/rr.h, so a field added on one side
    only fails here instead of shifting the fields after it."""
    import ctypes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rr.h"', "int main(void) {"]
    for cname, (pyname, ren) in _STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in getattr(rr, pyname)._fields_:
            cf = ren.get(f, f)
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for ln in out.splitlines():
        s, f, v = ln.split()
        got[(s, f)] = int(v)
    for cname, (pyname, _) in _STRUCTS.items():
        cls = getattr(rr, pyname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
    # and the same fields in the same order (a trailing field missing on one
    # side can hide in tail padding)
    hdr = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "rr.h")).read(), flags=re.S)
    for body, cname in re.findall(r"typedef struct\s*\{(.*?)\}\s*(rr_\w+)\s*;", hdr, flags=re.S):
        if cname not in _STRUCTS:
            continue
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            m = re.search(r"\(\*\s*(\w+)\)", decl)
            if m:  # a function pointer
                names.append(m.group(1))
                continue
            for part in decl.split(","):  # `int64_t a, b` declares two fields
                names.append(re.search(r"(\w+)\s*(\[[^\]]*\])?\s*$", part).group(1))
        pyname, ren = _STRUCTS[cname]
        assert names == [ren.get(f, f) for f, _ in getattr(rr, pyname)._fields_], cname
