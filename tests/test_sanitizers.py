"""Host code under the sanitizers (CPU only).

* The library's host graph builder (the code behind rr_index_build) built
  with AddressSanitizer + UndefinedBehaviorSanitizer, and again with
  ThreadSanitizer at several threads, driven by tests/sanitize/build_driver.cpp:
  no report, and the graph equals the oracle builder's byte for byte.
* The oracle built with AddressSanitizer + UndefinedBehaviorSanitizer and
  loaded into a Python subprocess: graph builder, every search mode, brute
  force, nearest-neighbour distances, percentile radius and the early-stop
  profile run without a report and give the plain build's results.
* The oracle's threaded routines built with ThreadSanitizer, driven by
  tests/sanitize/oracle_driver.c at 4 threads: no report, same digest as the
  plain build.
* The serving loop's host side (rr::ServerCore) with a CPU test double of the
  device, under ThreadSanitizer and under ASan + UBSan.

The GPU kernels are not covered: device code runs without sanitizers."""
import os
import shutil
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import oracle
from paper_2502_13245_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2502_13245_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")
ROCM_INCLUDE = "/opt/rocm/include"

GXX = shutil.which("g++")
GCC = shutil.which("gcc")
pytestmark = pytest.mark.skipif(GXX is None or GCC is None, reason="no host compilers")

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
           "TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"}


def _env(**extra):
    env = dict(os.environ)
    env.update(SAN_ENV)
    env.update(extra)
    return env


def _run(cmd, env, timeout=600):
    p = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=timeout)
    report = [m for m in ("AddressSanitizer", "runtime error", "ThreadSanitizer", "LeakSanitizer")
              if m in p.stderr]
    assert p.returncode == 0 and not report, (p.returncode, report, p.stderr[-4000:])
    return p


def _builder(tmp_path, flags, name):
    exe = str(tmp_path / name)
    subprocess.run([GXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags,
                    "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE, "-I", os.path.join(ROOT, "include"),
                    "-I", CSRC, os.path.join(CSRC, "rr_build.cpp"), os.path.join(SAN, "build_driver.cpp"),
                    "-o", exe, "-lpthread"], check=True, capture_output=True)
    return exe


@pytest.fixture(scope="module")
def small():
    w = synth.config_small_u8(0)
    base = np.ascontiguousarray(w.base[:1500])
    order = synth.permutation(len(base), 5)
    queries = np.ascontiguousarray(w.queries[:60])
    return base, order, queries


def _write_inputs(tmp_path, base, order, queries=None):
    b, o = tmp_path / "base.bin", tmp_path / "order.bin"
    base.tofile(b)
    np.asarray(order, np.int64).tofile(o)
    q = None
    if queries is not None:
        q = tmp_path / "queries.bin"
        queries.tofile(q)
    return str(b), str(o), (str(q) if q else None)


@pytest.mark.parametrize("kind,flags,threads", [
    ("asan_ubsan", ["-fsanitize=address,undefined"], 3),
    ("tsan", ["-fsanitize=thread"], 4),
])
def test_host_builder_under_sanitizer(tmp_path, small, kind, flags, threads):
    if not os.path.isdir(ROCM_INCLUDE):
        pytest.skip("no HIP headers")
    base, order, _ = small
    exe = _builder(tmp_path, flags, f"build_{kind}")
    b, o, _ = _write_inputs(tmp_path, base, order)
    out = str(tmp_path / "graph.bin")
    _run([exe, b, o, str(len(base)), str(base.shape[1]), "12", "24", "1.2", "2", str(threads), out],
         _env())
    raw = np.fromfile(out, dtype=np.int32)
    entry, adj = int(raw[0]), raw[1:].reshape(len(base), 12)
    want_adj, want_entry = oracle.build_vamana(base, 12, 24, 1.2, order, passes=2, threads=2)
    assert entry == want_entry
    np.testing.assert_array_equal(adj, want_adj)


ORACLE_SCRIPT = textwrap.dedent("""
    import sys, numpy as np
    sys.path.insert(0, {root!r})
    import oracle
    from paper_2502_13245_amd import synth
    oracle._LIB = {lib!r}
    w = synth.config_small_u8(0)
    base, q = np.ascontiguousarray(w.base[:1500]), np.ascontiguousarray(w.queries[:60])
    adj, entry = oracle.build_vamana(base, 12, 24, 1.2, synth.permutation(len(base), 5), threads=2)
    r = oracle.percentile_radius(base, q, 0.002)
    parts = [adj.sum(), entry, r]
    for mode, kw in ((oracle.PLAIN, {{}}), (oracle.ES, dict(es_visit_limit=3, es_radius=r)),
                     (oracle.ADAPTIVE, {{}}), (oracle.DOUBLING, dict(max_beam=64))):
        res = oracle.range_search(base, adj, entry, q, r, mode=mode, beam=8, threads=2, **kw)
        parts += [res.offsets.sum(), res.ids.astype(np.int64).sum(), float(res.dists.sum())]
    bf = oracle.brute_force(base, q, r, threads=2)
    parts += [bf.offsets.sum(), bf.ids.astype(np.int64).sum()]
    parts += [float(np.nansum(oracle.nn_dist(base, q, threads=2)))]
    m, f = oracle.es_profile(base, adj, entry, q, r, beam=8, step=3, threads=2)
    parts += [float(np.nansum(m)), int(f.sum())]
    print("DIGEST", repr([float(x) for x in parts]))
""")


def test_oracle_under_asan_ubsan(tmp_path):
    asan = subprocess.run([GCC, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no libasan runtime")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.run([GCC, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fPIC", "-shared", "-o", lib,
                    os.path.join(ROOT, "oracle", "rr_oracle.c"), "-lpthread", "-lm"],
                   check=True, capture_output=True)
    plain = str(tmp_path / "liboracle_plain.so")
    subprocess.run([GCC, "-std=c11", "-O2", "-fPIC", "-shared", "-o", plain,
                    os.path.join(ROOT, "oracle", "rr_oracle.c"), "-lpthread", "-lm"],
                   check=True, capture_output=True)
    digests = []
    for so, pre in ((lib, asan), (plain, None)):
        script = tmp_path / "run.py"
        script.write_text(ORACLE_SCRIPT.format(root=ROOT, lib=so))
        env = _env(**({"LD_PRELOAD": pre} if pre else {}))
        p = _run([sys.executable, str(script)], env)
        line = [x for x in p.stdout.splitlines() if x.startswith("DIGEST")]
        assert line, p.stdout[-2000:]
        digests.append(line[0])
    assert digests[0] == digests[1]


def test_oracle_threads_under_tsan(tmp_path, small):
    base, order, queries = small
    b, o, q = _write_inputs(tmp_path, base, order, queries)
    r = oracle.percentile_radius(base, queries, 0.002)
    outs = []
    for name, flags in (("tsan", ["-fsanitize=thread", "-O1", "-g"]), ("plain", ["-O2"])):
        exe = str(tmp_path / f"oracle_{name}")
        subprocess.run([GCC, "-std=c11", *flags, "-I", os.path.join(ROOT, "oracle"),
                        os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "rr_oracle.c"),
                        "-o", exe, "-lpthread", "-lm"], check=True, capture_output=True)
        out = str(tmp_path / f"digest_{name}.bin")
        _run([exe, b, o, q, str(len(base)), str(len(queries)), str(base.shape[1]), "4", repr(r), out],
             _env())
        outs.append(np.fromfile(out, dtype=np.uint8))
    np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("kind,flags", [
    ("tsan", ["-fsanitize=thread"]),
    ("asan_ubsan", ["-fsanitize=address,undefined"]),
])
def test_server_core_double(tmp_path, kind, flags):
    """The serving loop's host side (rr::ServerCore, the code behind
    rr_server_*) with a scripted device instead of the GPU: four submitting
    threads and a polling one, forced shared-capacity overflows; every request
    completes once and complete, retried requests run alone, the latency
    accounting is ordered and the counters agree, a full queue is refused and
    a failed worker start reaches every caller (tests/sanitize/server_double.cpp)."""
    exe = str(tmp_path / f"server_double_{kind}")
    subprocess.run([GXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags,
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(SAN, "server_double.cpp"), "-o", exe, "-lpthread"],
                   check=True, capture_output=True)
    p = _run([exe, "300"], _env())
    assert p.stdout.startswith("OK requests 1200"), p.stdout
