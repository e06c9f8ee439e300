#!/usr/bin/env python
"""Range-search benchmark on one MI355X.

Workload: 1,000,000 uint8 base vectors (d=128) and 10,000 queries from a
seeded mixture of 1,000 clusters with low intrinsic dimension (centres on a
16-dim Gaussian sheet, a 10-dim basis per cluster, near-duplicate groups,
Zipf cluster sizes; synth.latent_mixture_u8), a Vamana graph (R=64, L=128,
alpha=1.2), and a squared-L2 radius at which 75% of the queries have no
result (the 25th percentile of per-query nearest-neighbour distances).
Ground truth comes from the library's MFMA scan.

For each search mode (plain beam, beam + early stop, adaptive = beam + early
stop + greedy expansion) the beam width is swept; the fastest setting whose
range recall is >= 0.9 is kept (the Pareto point at 0.9).  The headline
adaptive setting is tuned on the even-numbered queries and its recall is
reported on the odd-numbered ones (held out) and on all.  The timed steps
run it: one step = one rr_range_search call over the whole batch (query
prep, beam kernel, greedy phase, compaction) plus the copy of the CSR
result, with the queries already in HBM.

Prints one JSON line (the last line of output).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("rr_search.h", "rr_inst.hip", "rr_kernels.hip", "rr_internal.h")


def kernel_source_sha1():
    """sha1 over the search kernels' sources (the traffic records name it)."""
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2502_13245_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def load_traffic(tag):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/), or
    None when the kernel sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}.md")
    if not os.path.exists(path):
        return None
    sha = kernel_source_sha1()
    for line in open(path):
        if line.startswith("TRAFFIC "):
            rec = json.loads(line[len("TRAFFIC "):])
            if rec.get("kernel_source_sha1") == sha:
                return rec["bytes_per_launch"]
    return None


def sorted_member(sorted_keys, keys):
    """keys[i] in sorted_keys, by binary search (np.isin sorts both arrays
    on every call: too slow for one short list against millions of keys)."""
    if len(sorted_keys) == 0:
        return np.zeros(len(keys), dtype=bool)
    pos = np.minimum(np.searchsorted(sorted_keys, keys), len(sorted_keys) - 1)
    return sorted_keys[pos] == keys


def recall_of(found_off, found_ids, truth_keys, n, truth_total, qmap=None):
    """Range recall (average precision of the paper): sum |K & K'| / sum |K|.
    qmap[j] is the query number of found list j (default j)."""
    nq = len(found_off) - 1
    q = np.repeat(np.arange(nq, dtype=np.int64) if qmap is None else np.asarray(qmap, np.int64),
                  np.diff(found_off))
    keys = q * n + found_ids.astype(np.int64)
    hit = sorted_member(truth_keys, keys).sum()
    return float(hit) / truth_total if truth_total else float("nan")


def cpu_share():
    """Host cores: the count the OS reports, the ones this process may run
    on (affinity), the cgroup CPU quota, the thread count used (the smallest
    of these and OMP_NUM_THREADS, the box's per-GPU CPU share) and the model."""
    nproc = os.cpu_count() or 1
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else nproc
    quota = None
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = int(q) / int(per)
    except (OSError, ValueError):
        pass
    use = aff if quota is None else max(1, min(aff, int(quota)))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        use = max(1, min(use, int(os.environ["OMP_NUM_THREADS"])))
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(nproc=nproc, affinity=aff, cgroup_quota=quota, threads=use, model=model)


def serve_leg(rr, ix, queries, q, n, levels, sp, args):
    """Open-loop serving run per offered rate: arrival times from a Poisson
    process, queries drawn from `queries` (host; q is the same on the
    device), each request's radius drawn from the three `levels`.  Latency =
    completion time (results on the host) minus scheduled arrival time, so
    submitter lag counts against the server; the submitter's own lag (submit
    call - scheduled time) is reported beside it.  Served results are scored
    against the brute-force truth of their own radius (range recall per
    rate).  The early-stop radius esr is the tuned absolute value for every
    request, whatever its radius."""
    if args.serve_seconds <= 0:
        return None
    nq = len(queries)
    truth = []
    for lv in levels:
        t0 = time.time()
        off, ids, _ = rr.brute_force(ix, q, lv).numpy()
        qq = np.repeat(np.arange(nq, dtype=np.int64), np.diff(off))
        truth.append((np.sort(qq * n + ids.astype(np.int64)), np.diff(off)))
        log(f"serving truth at radius {lv:.6g}: {int(off[-1])} results ({time.time() - t0:.1f}s)")
    rng = np.random.default_rng(7)
    rates = [float(x) for x in args.serve_rates.split(",")]
    # one untimed server first: the first ticks of a process load the serving
    # kernels' code, which would otherwise land in the first rate's tail
    wm = min(256, nq)
    with rr.Server(ix, sp, slots=args.serve_slots, step_budget=args.serve_budget) as srv:
        for i in range(wm):
            srv.submit(queries[i], levels[i % 3], i)
        srv.drain(timeout=120.0)
        srv.poll(wm + 16)
        warm_tick_ms = round(srv.info()["max_tick_s"] * 1e3, 3)
    out = []
    for rate in rates:
        m = max(1, int(rate * args.serve_seconds))
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=m)) + 0.01
        qidx = rng.integers(0, nq, size=m)
        lvl = rng.integers(0, 3, size=m)
        radii = np.asarray(levels)[lvl]
        qs = np.ascontiguousarray(queries[qidx])
        lag = np.zeros(m)
        with rr.Server(ix, sp, slots=args.serve_slots, step_budget=args.serve_budget) as srv:
            t_base = srv.clock()
            arr = arrivals + t_base
            i = 0
            while i < m:
                now = srv.clock()
                while i < m and arr[i] <= now:
                    if not srv.submit(qs[i], radii[i], i, float(arr[i])):
                        break
                    lag[i] = now - arr[i]
                    i += 1
                if i < m:
                    wait = arr[i] - srv.clock()
                    if wait > 2e-4:
                        time.sleep(min(wait, 2e-3) - 1e-4)
            srv.drain(timeout=120.0)
            comps = srv.poll(m + 16)
            info = srv.info()
            hits = found = 0
            want = 0
            for c in comps:
                ids, _ = srv.result(c.tag)
                k = int(c.tag)
                tk, tc = truth[lvl[k]]
                keys = int(qidx[k]) * n + ids.astype(np.int64)
                hits += int(sorted_member(tk, keys).sum())
                found += len(ids)
                want += int(tc[qidx[k]])
        lat = np.array([c.t_done - c.t_arrival for c in comps]) * 1e3
        qwait = np.array([c.t_admit - c.t_arrival for c in comps]) * 1e3
        span = max(c.t_done for c in comps) - (arr[0])
        ticks = np.array([c.ticks for c in comps])
        trunc = int(sum(c.truncated for c in comps))
        rec = dict(offered_qps=rate, requests=m, achieved_qps=round(m / span, 1),
                   p50_ms=round(float(np.percentile(lat, 50)), 3),
                   p99_ms=round(float(np.percentile(lat, 99)), 3),
                   mean_ms=round(float(lat.mean()), 3),
                   queue_p99_ms=round(float(np.percentile(qwait, 99)), 3),
                   submit_lag_p99_ms=round(float(np.percentile(lag, 99)) * 1e3, 3),
                   recall=round(hits / want, 4) if want else None,
                   mean_ticks=round(float(ticks.mean()), 2), max_ticks=int(ticks.max()),
                   server_ticks=info["ticks"], max_resident=info["max_resident"],
                   mean_tick_ms=round(info["busy_s"] / max(info["ticks"], 1) * 1e3, 3),
                   max_tick_ms=round(info["max_tick_s"] * 1e3, 3),
                   retried=info["retried"], truncated=trunc)
        log(f"serve {rate:>8,.0f} QPS offered: achieved {rec['achieved_qps']:,.0f}, "
            f"p50 {rec['p50_ms']:.3f} ms, p99 {rec['p99_ms']:.3f} ms (queue p99 "
            f"{rec['queue_p99_ms']:.3f}, submitter lag p99 {rec['submit_lag_p99_ms']:.3f}), recall "
            f"{rec['recall']}, mean ticks {rec['mean_ticks']}, server ticks {info['ticks']}, "
            f"max resident {info['max_resident']}")
        out.append(rec)
    return dict(slots=args.serve_slots, step_budget=args.serve_budget, radius_levels=levels,
                warmup_requests=wm, warmup_max_tick_ms=warm_tick_ms,
                es_radius="fixed (the tuned value) for every request radius",
                mode="adaptive", beam=sp.beam, rates=out)


# ---------------------------------------------------------------------------
# the other workloads (float embeddings with the bf16 and 8-bit passes, the
# 10M int8 batching workload, serving 768-wide float rows): bench.py
# --workload c3|c4|c5 prints one JSON line for that workload
# ---------------------------------------------------------------------------

def median_time(fn, reps=5, warm=2):
    """Median wall time of fn() (seconds), synchronizing around each call;
    settings slower than a second get one warm-up and one timed call."""
    import torch
    for k in range(warm):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        if time.perf_counter() - t > 1.0:
            reps = 1
            break
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts))


def truth_keys_of(rr, ix, q, radius, n):
    """Brute-force truth (MFMA scan) as sorted keys q * n + id, plus counts."""
    off, ids, _ = rr.brute_force(ix, q, radius).numpy()
    counts = np.diff(off)
    qq = np.repeat(np.arange(len(counts), dtype=np.int64), counts)
    return np.sort(qq * n + ids.astype(np.int64)), counts


def sweep_mode(rr, ix, q, radius, keys, n, total, mode, beams, target, tag, **kw):
    """Beam sweep of one mode: recall and QPS per beam; the fastest setting
    at recall >= target (two settings past it end the sweep)."""
    best, curve, past = None, [], 0
    nq = q.shape[0]
    for b in beams:
        try:
            off, ids, _ = rr.range_search(ix, q, radius, mode=mode, beam=b, with_stats=False,
                                          **kw).numpy()
        except rr.RRError as e:
            log(f"{tag} b={b}: {e}")
            break
        rec = recall_of(off, ids, keys, n, total)
        sec = median_time(lambda: rr.range_search(ix, q, radius, mode=mode, beam=b,
                                                  with_stats=False, **kw), reps=3, warm=1)
        curve.append(dict(beam=b, recall=round(rec, 4), qps=round(nq / sec, 1)))
        log(f"{tag:10s} b={b:5d} recall={rec:.4f} qps={nq / sec:,.0f}")
        if rec >= target:
            if best is None or nq / sec > best["qps"]:
                best = dict(beam=b, recall=rec, qps=nq / sec)
            past += 1
            if past >= 2:
                break
    return best, curve


def kernel_roofline(rr, ix, q, radius, reps=5, **kw):
    """Beam and greedy kernel times (HIP events the library records on the
    launch stream) and their algorithmic bytes, as in the 1M u8 run."""
    bm, gk, tot = [], [], []
    st = None
    for _ in range(reps):
        st = rr.range_search(ix, q, radius, timing=True, **kw).batch
        bm.append(st["beam_ms"])
        gk.append(st["greedy_kernel_ms"])
        tot.append(st["total_ms"])

    def roof(kernel, nbytes, ms):
        ach = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        return dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4), traffic=None, kernel=kernel,
                    bytes_per_launch=int(nbytes), avg_ms=round(ms, 4))
    rb = roof("k_beam", st["bytes_beam"], float(np.mean(bm)))
    rg = roof("k_greedy", st["bytes_greedy"], float(np.mean(gk))) if np.mean(gk) > 0 else None
    dom = rg if rg and rg["avg_ms"] > rb["avg_ms"] else rb
    return dom, rb, rg, st, float(np.mean(tot))


def build_index(rr, base, args, label, **bp):
    """The index from --graph if the file exists, else the host Vamana build
    (saved to --graph when given)."""
    t0 = time.time()
    if args.graph and os.path.exists(args.graph):
        ix = rr.Index.load(args.graph)
        log(f"{label}: index loaded from {args.graph}")
        return ix, None
    ix = rr.Index.build(base, verbose=True, **bp)
    dt = time.time() - t0
    log(f"{label}: graph built on the host in {dt:.1f}s ({bp})")
    if args.graph:
        ix.save(args.graph)
    return ix, round(dt, 1)


def only_run(rr, ix, q, args):
    """Profiling mode: the setting from --choice, --steps calls, nothing else
    (after the --copy-ref-mb reference copies, if asked)."""
    import torch
    ch = json.load(open(args.choice))
    if args.copy_ref_mb:
        src = torch.empty(args.copy_ref_mb << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"copy reference: {args.copy_ref_mb} MiB device-to-device x3")
    for _ in range(args.steps):
        rr.range_search(ix, q, ch["radius"], mode=ch["mode"], beam=ch["beam"], with_stats=False,
                        **ch["kw"])
    torch.cuda.synchronize()
    teardown(ix)
    log(f"profiling run done: {args.steps} x {ch['mode']} b={ch['beam']} {ch['kw']}")


def teardown(ix):
    """Free every library object and torch's cached blocks before returning,
    so that no HIP call is left for garbage collection at interpreter exit."""
    import gc
    import torch
    gc.collect()
    torch.cuda.synchronize()
    ix.free()
    torch.cuda.empty_cache()
    torch.cuda.synchronize()


def run_c3(args, rr, synth, cpus):
    """1M x 96 float32 unit-norm embeddings (2,000 clusters), 10,000 queries,
    L2 radius at the 0.05th percentile of all query-base distances (selected
    on the GPU).  Adaptive search in three precisions (exact FP64
    accumulation, bf16 first pass + exact recheck, 8-bit first pass + exact
    re-decision) and plain beam search, each swept for recall >= target; the
    timed steps run the bf16 setting.  Membership of the approximate passes
    is checked against FP64 distances on sampled queries."""
    import torch
    import oracle
    threads = args.threads or cpus["threads"]
    w = synth.config_1m_f32(2, n=args.n, nq=args.nq)
    ix, build_s = build_index(rr, w.base, args, "c3", R=64, L=128, alpha=1.2, passes=1,
                              threads=threads, seed=2)
    ix.to_device("cuda:0")
    q = torch.from_numpy(w.queries).cuda()
    nq, n = len(w.queries), len(w.base)
    if args.only:
        return only_run(rr, ix, q, args)
    t0 = time.time()
    radius = rr.select_radius(ix, q, 0.0005)
    log(f"radius (squared L2, 0.05th percentile of {nq * n:.3g} pairs) {radius:.6g} "
        f"selected in {time.time() - t0:.2f}s")
    keys, counts = truth_keys_of(rr, ix, q, radius, n)
    total = int(counts.sum())
    log(f"ground truth: {total} results, empty {(counts == 0).sum()}/{nq}, max {counts.max()}")
    # the greedy phase's result capacity: the library's default (2M) is below
    # this workload's 5M results
    es = dict(es_enable=True, es_visit_limit=10, es_radius=radius,
              result_capacity=max(2 * total, 1 << 22))
    beams = [2, 4, 8, 16, 32, 64, 128, 256]
    modes = {}
    for name, prec in (("exact", rr.EXACT), ("bf16", rr.BF16_RECHECK), ("sq8", rr.SQ8_RERANK)):
        best, curve = sweep_mode(rr, ix, q, radius, keys, n, total, "adaptive", beams, args.target,
                                 f"ada-{name}", precision=prec, **es)
        modes[name] = dict(best=best, curve=curve)
    pbest, pcurve = sweep_mode(rr, ix, q, radius, keys, n, total, "plain",
                               [64, 128, 256, 512, 1024, 2048, 4096], args.target, "plain")
    # membership of the approximate passes against FP64 distances: every
    # returned point of 300 sampled queries (and the 20 heaviest), and the
    # oracle's FP64 ball for them
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([rng.choice(nq, 300, replace=False),
                                    np.argsort(-counts, kind="stable")[:20]]))
    ball = oracle.brute_force(w.base, w.queries[idx], radius, threads=threads)
    member = {}
    for name, prec in (("bf16", rr.BF16_RECHECK), ("sq8", rr.SQ8_RERANK), ("exact", rr.EXACT)):
        b = modes[name]["best"]["beam"] if modes[name]["best"] else 16
        res = rr.range_search(ix, q, radius, mode="adaptive", beam=b, precision=prec, **es)
        off, ids, d = res.numpy()
        extra = missing = returned = 0
        max_rel = 0.0
        for k, qi in enumerate(idx):
            g = ids[off[qi]:off[qi + 1]]
            gd = d[off[qi]:off[qi + 1]].astype(np.float64)
            x = w.base[g].astype(np.float64) - w.queries[qi].astype(np.float64)
            d64 = (x * x).sum(1)
            extra += int((d64 > radius).sum())
            returned += len(g)
            if len(g):
                max_rel = max(max_rel, float(np.max(np.abs(gd - d64) / np.maximum(d64, 1e-30))))
            oi, _ = ball.query(k)
            missing += int(len(np.setdiff1d(oi, g)))
        member[name] = dict(beam=b, sampled_queries=len(idx), returned=returned,
                            outside_fp64_ball=extra, fp64_ball_points_missed=missing,
                            max_rel_dist_error=max_rel,
                            rechecked=int(res.stats["rechecked"].sum()))
        log(f"membership {name} b={b}: returned {returned}, outside the FP64 ball {extra}, "
            f"missed {missing} of {ball.offsets[-1]}, max rel distance error {max_rel:.2e}")
    head = modes["bf16"]["best"] or dict(beam=16, recall=float("nan"))
    kw = dict(mode="adaptive", beam=head["beam"], precision=rr.BF16_RECHECK, **es)
    if args.choice:
        json.dump(dict(radius=radius, mode="adaptive", beam=head["beam"],
                       kw=dict(precision=rr.BF16_RECHECK, **es)), open(args.choice, "w"))
    sec = median_time(lambda: rr.range_search(ix, q, radius, with_stats=False, **kw),
                      reps=args.steps, warm=args.warmup)
    dom, rb, rg, st, call_ms = kernel_roofline(rr, ix, q, radius, **kw)
    out = {
        "metric": "range QPS at 0.9 range recall (float embeddings, bf16 first pass + exact recheck, 1 GPU)",
        "value": round(nq / sec, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 rows, f32 accumulation, f64 recheck",
        "data": "synthetic",
        "config": {"workload": f"f32 d=96 unit-norm, {n} base, {nq} queries, latent mixture of 2000 "
                               f"clusters (synth.config_1m_f32 seed 2); Vamana R=64 L=128 alpha=1.2 "
                               f"one pass; squared-L2 radius at the 0.05th percentile of all pairs",
                   "radius": radius, "beam": head["beam"], "recall": round(head["recall"], 4),
                   "results": total, "empty": int((counts == 0).sum()), "max_results": int(counts.max())},
        "roofline": dom, "roofline_beam": rb, "roofline_greedy": rg,
        "adaptive": {k: v["best"] for k, v in modes.items()},
        "plain_at_target": pbest, "adaptive_bf16_vs_plain": round(head.get("qps", 0) / pbest["qps"], 2)
        if pbest and head.get("qps") else None,
        "membership_vs_fp64": member, "curves": {**{k: v["curve"] for k, v in modes.items()},
                                                 "plain": pcurve},
        "graph_build_s": build_s, "call_ms": round(call_ms, 4),
    }
    print(json.dumps(out), flush=True)
    profile_tail(rr, ix, q, radius, args, **kw)


def run_c4(args, rr, synth, cpus):
    """10M x 100 int8 base, 100,000 queries, radius at which 75% of the
    queries are empty; the setting tuned on the first 10,000 queries, then
    all 100,000 in one launch and in uneven batches (1k / 4k / 16k / 64k /
    15k), results compared per query between the two."""
    import torch
    threads = args.threads or cpus["threads"]
    n = 10_000_000 if args.n == 1_000_000 else args.n
    nq = 100_000 if args.nq == 10_000 else args.nq
    t0 = time.time()
    w = synth.config_10m_i8(4, n=n, nq=nq)
    log(f"workload {w.name}: generated in {time.time() - t0:.1f}s")
    ix, build_s = build_index(rr, w.base, args, "c4", R=64, L=64, alpha=1.2, passes=1,
                              threads=threads, seed=4)
    ix.to_device("cuda:0")
    q = torch.from_numpy(w.queries).cuda()
    if args.only:
        return only_run(rr, ix, q, args)
    nn = np.sort(rr.nn_dist(ix, q).cpu().numpy())
    radius = float(nn[math.ceil(0.25 * nq) - 1])
    keys, counts = truth_keys_of(rr, ix, q, radius, n)
    total = int(counts.sum())
    hist = [int((counts == 0).sum())] + [int(((counts > 10 ** (k - 1) if k > 1 else counts > 0)
                                              & (counts <= 10 ** k)).sum()) for k in range(1, 6)]
    log(f"radius {radius:.0f}; ground truth: {total} results, bins(0,<=10,..,<=1e5) {hist}, "
        f"max {counts.max()}")
    nt = min(10_000, nq)
    q_t = q[:nt].contiguous()
    truth_t = rr.brute_force_async(ix, q_t, radius)
    sp, tune = rr.autotune(ix, q_t, radius, truth_t, target=args.target, reps=3, mode="adaptive",
                           es_enable=True, es_visit_limit=10, es_radius=radius)
    sp, es_tune = rr.tune_early_stop(ix, q_t, radius, truth_t, target=args.target, reps=3, params=sp)
    log(f"tuned on the first {nt} queries: {tune} / {es_tune}")
    kw = dict(mode="adaptive", beam=sp.beam, es_enable=bool(sp.es_enable),
              es_visit_limit=sp.es_visit_limit, es_radius=sp.es_radius,
              waves_per_group=sp.waves_per_group, cache_slots=sp.cache_slots,
              result_capacity=max(4 * total, 1 << 22))
    if args.choice:
        json.dump(dict(radius=radius, mode="adaptive", beam=sp.beam,
                       kw={k: v for k, v in kw.items() if k not in ("mode", "beam")}),
                  open(args.choice, "w"))
    one = rr.range_search(ix, q, radius, **kw)
    off, ids, d = one.numpy()
    rec_all = recall_of(off, ids, keys, n, total)
    held = keys // n >= nt
    ho_off = off[nt:] - off[nt]
    rec_ho = recall_of(ho_off, ids[off[nt]:], keys[held], n, int(held.sum()),
                       qmap=np.arange(nt, nq))
    sec = median_time(lambda: rr.range_search(ix, q, radius, with_stats=False, **kw),
                      reps=args.steps, warm=args.warmup)
    sizes = [1000, 4000, 16000, 64000]
    sizes.append(nq - sum(sizes)) if nq > sum(sizes) else None
    bounds = np.cumsum([0] + sizes)

    def batches():
        return [rr.range_search(ix, q[a:b].contiguous(), radius, with_stats=False, **kw)
                for a, b in zip(bounds[:-1], bounds[1:])]
    same = True
    for (a, b), r in zip(zip(bounds[:-1], bounds[1:]), batches()):
        bo, bi, bd = r.numpy()
        same &= np.array_equal(bo, off[a:b + 1] - off[a]) and np.array_equal(bi, ids[off[a]:off[b]])
    sec_b = median_time(batches, reps=3, warm=1)
    log(f"one launch {nq / sec:,.0f} QPS, uneven batches {nq / sec_b:,.0f} QPS, same results {same}, "
        f"recall {rec_all:.4f} (held-out {rec_ho:.4f})")
    dom, rb, rg, st, call_ms = kernel_roofline(rr, ix, q, radius, **kw)
    out = {
        "metric": "range QPS at 0.9 range recall (10M int8, one batched launch, 1 GPU)",
        "value": round(nq / sec, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i8", "data": "synthetic",
        "config": {"workload": f"i8 d=100 (rows padded to 128 B), {n} base, {nq} queries, latent "
                               f"mixture of 10000 clusters centred at 0 (synth.config_10m_i8 seed 4); "
                               f"Vamana R=64 L=64 alpha=1.2 one pass; radius at 75% empty queries",
                   "radius": radius, "beam": sp.beam, "es_visit_limit": sp.es_visit_limit,
                   "es_radius": sp.es_radius, "recall": round(rec_ho, 4),
                   "recall_scope": f"queries {nt}..{nq} (tuned on the first {nt})",
                   "recall_all": round(rec_all, 4), "results": total,
                   "result_hist_0_10_1e2_1e3_1e4_1e5": hist, "max_results": int(counts.max())},
        "uneven_batches": {"sizes": sizes, "qps": round(nq / sec_b, 1), "same_results": bool(same)},
        "roofline": dom, "roofline_beam": rb, "roofline_greedy": rg,
        "autotune": tune, "es_tune": es_tune, "graph_build_s": build_s, "call_ms": round(call_ms, 4),
    }
    print(json.dumps(out), flush=True)
    profile_tail(rr, ix, q, radius, args, **kw)


def profile_tail(rr, ix, q, radius, args, **kw):
    """--profile-tail K: K more calls of the chosen setting, the last dispatches
    of the run (a kernel trace of the whole run averages them), then an
    explicit teardown."""
    import torch
    if args.profile_tail > 0:
        for _ in range(args.profile_tail):
            rr.range_search(ix, q, radius, with_stats=False, **kw)
        torch.cuda.synchronize()
        log(f"profile tail done: {args.profile_tail} x {kw}")
    teardown(ix)


def run_c5(args, rr, synth, cpus):
    """Serving 768-wide float32 rows: 2M unit-norm base (5,000 clusters),
    bf16 first pass + exact recheck; radii at the 0.02th, 0.05th and 0.1th
    percentiles of the pairs of a 10,000-query calibration set (selected on
    the GPU); open-loop Poisson arrivals of 10,000 other queries, each
    request with one of the three radii, at several offered rates."""
    import torch
    threads = args.threads or cpus["threads"]
    n = 2_000_000 if args.n == 1_000_000 else args.n
    nc = 10_000 if args.nq == 10_000 else args.nq
    t0 = time.time()
    w = synth.latent_mixture_f32(n, 2 * nc, 768, 5_000, 0.35, 5, name=f"f32-{n // 1000}k-d768")
    log(f"workload {w.name}: generated in {time.time() - t0:.1f}s")
    ix, build_s = build_index(rr, w.base, args, "c5", R=32, L=64, alpha=1.2, passes=1,
                              threads=threads, seed=5)
    ix.to_device("cuda:0")
    q_cal = torch.from_numpy(w.queries[:nc]).cuda()
    pool = np.ascontiguousarray(w.queries[nc:])
    q_pool = torch.from_numpy(pool).cuda()
    if args.only:
        return only_run(rr, ix, q_cal, args)
    t0 = time.time()
    levels = [float(x) for x in rr.select_radius(ix, q_cal, [0.0002, 0.0005, 0.001])]
    log(f"radii (0.02/0.05/0.1th percentiles of {nc * n:.3g} pairs) {levels} in {time.time() - t0:.1f}s")
    mid = levels[1]
    truth_c = rr.brute_force_async(ix, q_cal, mid)
    sp, tune = rr.autotune(ix, q_cal, mid, truth_c, target=args.target, reps=3, mode="adaptive",
                           precision=rr.BF16_RECHECK, es_enable=True, es_visit_limit=10,
                           es_radius=mid)
    sp, es_tune = rr.tune_early_stop(ix, q_cal, mid, truth_c, target=args.target, reps=3, params=sp)
    log(f"tuned on the calibration queries at the middle radius: {tune} / {es_tune}")
    rates = [float(x) for x in args.serve_rates.split(",")]
    serving = serve_leg(rr, ix, pool, q_pool, n, levels, sp, args)
    worst = max(serving["rates"], key=lambda r: r["p99_ms"])
    out = {
        "metric": "served range queries: p99 latency at the offered rates (768-wide float rows, bf16 "
                  "first pass + exact recheck, 1 GPU)",
        "value": worst["p99_ms"], "unit": "ms (p99, worst offered rate)", "n_gpus": 1,
        "steps": len(rates), "warmup": 0, "ms_per_step": None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 rows, f32 accumulation, f64 recheck",
        "data": "synthetic",
        "config": {"workload": f"f32 d=768 unit-norm, {n} base, latent mixture of 5000 clusters "
                               f"(synth.latent_mixture_f32 seed 5); {nc} calibration + {nc} served "
                               f"queries; Vamana R=32 L=64 alpha=1.2 one pass",
                   "radius_levels": levels, "beam": sp.beam, "es_visit_limit": sp.es_visit_limit,
                   "es_radius": sp.es_radius},
        "serving": serving, "autotune": tune, "es_tune": es_tune, "graph_build_s": build_s,
    }
    print(json.dumps(out), flush=True)
    teardown(ix)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--nq", type=int, default=10_000)
    ap.add_argument("--target", type=float, default=0.9)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--graph", default="", help="load the index from this file if present")
    ap.add_argument("--choice", default="", help="write (full run) / read (--only) the chosen "
                                                 "setting as JSON")
    ap.add_argument("--only", action="store_true",
                    help="profiling mode: skip sweeps, run the setting from --choice --steps times")
    ap.add_argument("--scan-only", action="store_true",
                    help="profiling mode: run the MFMA nearest-distance scan and the brute-force "
                         "range scan --steps times on the workload and exit (no graph is built)")
    ap.add_argument("--copy-ref-mb", type=int, default=0,
                    help="also run a device-to-device copy of this size (counter calibration)")
    ap.add_argument("--serve-seconds", type=float, default=1.0,
                    help="arrival window per offered rate of the serving run (0: skip)")
    ap.add_argument("--serve-rates", default="2000,10000,50000")
    ap.add_argument("--serve-slots", type=int, default=1024)
    ap.add_argument("--serve-budget", type=int, default=8)
    ap.add_argument("--profile-tail", type=int, default=0,
                    help="c3/c4: after the JSON line, run the chosen setting this many more times "
                         "(the last dispatches of a kernel trace of the whole run)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5"],
                    help="c2: 1M u8 (default, the headline); c3: 1M x 96 float32 in three "
                         "precisions; c4: 10M int8 batching; c5: serving 2M x 768 float32")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; this build has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2502_13245_amd import rr, synth

    cpus = cpu_share()
    threads = args.threads or cpus["threads"]
    if args.workload != "c2":
        return {"c3": run_c3, "c4": run_c4, "c5": run_c5}[args.workload](args, rr, synth, cpus)
    t0 = time.time()
    w = synth.config_1m_u8(1, n=args.n, nq=args.nq)
    log(f"workload {w.name}: generated in {time.time() - t0:.1f}s")
    if args.scan_only:
        # the scans read only the vectors: any valid graph serves
        ix = rr.Index.from_graph(w.base, synth.shifted_graph(len(w.base), 8, 1), 0).to_device("cuda:0")
        q = torch.from_numpy(w.queries).cuda()
        nn = rr.nn_dist(ix, q)
        radius = float(np.sort(nn.cpu().numpy())[math.ceil(0.25 * len(w.queries)) - 1])
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.steps):
            rr.nn_dist(ix, q)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        tops = 2.0 * len(w.queries) * len(w.base) * 128 / (ms * 1e-3) / 1e12
        ev0.record()
        for _ in range(args.steps):
            res = rr.brute_force(ix, q, radius)
        ev1.record()
        torch.cuda.synchronize()
        ms_r = ev0.elapsed_time(ev1) / args.steps
        log(f"scan-only run done: {args.steps} x nn scan ({ms:.3f} ms, {tops:.0f} TOP/s) "
            f"and {args.steps} x range scan at radius {radius:.0f} ({ms_r:.3f} ms per call with "
            f"its result assembly, {int(res.offsets[-1])} results)")
        return
    t0 = time.time()
    if args.graph and os.path.exists(args.graph):
        ix = rr.Index.load(args.graph)
        build_s = None
        log(f"index loaded from {args.graph}")
    else:
        ix = rr.Index.build(w.base, R=64, L=128, alpha=1.2, passes=2, threads=threads, seed=1,
                            verbose=True)
        build_s = time.time() - t0
        log(f"graph built on the host in {build_s:.1f}s ({threads} threads)")
        if args.graph:
            ix.save(args.graph)
    ix.to_device("cuda:0")
    q = torch.from_numpy(w.queries).cuda()
    n, nq, d = args.n, args.nq, 128
    torch.cuda.synchronize()

    if args.only:
        ch = json.load(open(args.choice))
        if args.copy_ref_mb:
            src = torch.empty(args.copy_ref_mb << 20, dtype=torch.uint8, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            log(f"copy reference: {args.copy_ref_mb} MiB device-to-device x3")
        for _ in range(args.steps):
            rr.range_search(ix, q, ch["radius"], mode=ch["mode"], beam=ch["beam"],
                            with_stats=False, **ch["kw"])
        torch.cuda.synchronize()
        if args.copy_ref_mb:
            del src, dst
        teardown(ix)
        log(f"profiling run done: {args.steps} x {ch['mode']} b={ch['beam']}")
        return

    # radius: 75% of queries empty (nearest-neighbour distance quantile), on the GPU
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rr.nn_dist(ix, q)
    ev0.record()
    nn = rr.nn_dist(ix, q)
    ev1.record()
    torch.cuda.synchronize()
    nn_ms = ev0.elapsed_time(ev1)
    nn_sorted = np.sort(nn.cpu().numpy())
    radius = float(nn_sorted[math.ceil(0.25 * nq) - 1])
    scan_tops = 2.0 * nq * n * d / (nn_ms * 1e-3) / 1e12
    log(f"radius {radius:.0f} (nn scan {nn_ms:.2f} ms, {scan_tops:.0f} TOP/s int8 MFMA)")
    # context for the search kernels' rooflines: the rate at which the GPU
    # reads whole base rows at random when no read waits on another (the
    # library's probe kernel, rows split over lanes as the search splits them)
    g_rows = 16_000_000
    rr.probe_row_gather(ix, g_rows, seed=7)
    g_ts = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rr.probe_row_gather(ix, g_rows, seed=7)
        e1.record()
        torch.cuda.synchronize()
        g_ts.append(e0.elapsed_time(e1))
    g_ms = float(np.median(g_ts))
    row_bytes = w.base.shape[1] * w.base.itemsize  # 128: no row padding at this width
    gather = {"op": "rr_probe_row_gather: independent random reads of whole base rows", "rows": g_rows,
              "row_bytes": row_bytes, "ms": round(g_ms, 4), "rows_per_s": round(g_rows / (g_ms * 1e-3), 1),
              "random_read_GBs": round(g_rows * row_bytes / (g_ms * 1e-3) / 1e9, 1)}
    log(f"random row gather (context): {gather['rows_per_s'] / 1e9:.1f}G rows/s, "
        f"{gather['random_read_GBs']:.0f} GB/s of random reads")
    t0 = time.time()
    truth_h = rr.brute_force_async(ix, q, radius)
    truth = truth_h.fetch(False)
    toff, tids, _ = truth.numpy()
    counts = np.diff(toff)
    truth_total = int(toff[-1])
    tq = np.repeat(np.arange(nq, dtype=np.int64), counts)
    truth_keys = np.sort(tq * n + tids.astype(np.int64))
    hist = [int((counts == 0).sum())] + [int(((counts > 10 ** (k - 1) if k > 1 else counts > 0)
                                              & (counts <= 10 ** k)).sum()) for k in range(1, 6)]
    log(f"ground truth: {truth_total} results, empty {hist[0]}/{nq}, max {counts.max()}, "
        f"bins(0,<=10,..,<=1e5) {hist} ({time.time() - t0:.1f}s)")

    def run(mode, beam, timing=False, **kw):
        return rr.range_search(ix, q, radius, mode=mode, beam=beam, timing=timing, **kw)

    def timed(mode, beam, reps=3, **kw):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            rr.range_search(ix, q, radius, mode=mode, beam=beam, with_stats=False, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    es_kw = dict(es_enable=True, es_visit_limit=10, es_radius=radius)
    sweeps = {
        "plain": (dict(), [32, 64, 128, 256, 512, 1024, 2048, 4096]),
        "es": (dict(es_visit_limit=10, es_radius=radius), [32, 64, 128, 256, 512, 1024, 2048, 4096]),
        "adaptive": (es_kw, [2, 4, 8, 16, 24, 32, 48, 64, 96, 128]),
        "adaptive_noes": (dict(es_enable=False), [2, 4, 8, 16, 24, 32, 48, 64, 96, 128]),
        "doubling": (dict(max_beam=8192, result_capacity=4_000_000), [2, 4, 8, 16, 32, 64]),
        "doubling_es": (dict(max_beam=8192, result_capacity=4_000_000, es_enable=True,
                             es_visit_limit=10, es_radius=radius), [2, 4, 8, 16, 32, 64]),
    }
    best = {}
    curves = {}
    for name, (kw, beams) in sweeps.items():
        mode = name.split("_")[0]
        curves[name] = []
        for b in beams:
            try:
                res = run(mode, b, **kw)
            except rr.RRError as e:
                log(f"{name} b={b}: {e}")
                break
            off, ids, _ = res.numpy()
            rec = recall_of(off, ids, truth_keys, n, truth_total)
            sec = timed(mode, b, **kw)
            curves[name].append(dict(beam=b, recall=round(rec, 4), qps=round(nq / sec, 1)))
            log(f"{name:14s} b={b:5d} recall={rec:.4f} qps={nq / sec:,.0f}")
            if rec >= args.target:
                if name not in best or nq / sec > best[name]["qps"]:
                    best[name] = dict(beam=b, recall=rec, qps=nq / sec, kw=kw, mode=mode)
                if rec >= args.target + 0.03:
                    break
    if "adaptive" not in best:
        raise SystemExit("adaptive search did not reach the recall target")
    # the baselines get the beam kernel's shape tuned at their beam too (the
    # visited cache's size sets how many waves fit a CU at wide beams)
    for name in ("plain", "es"):
        if name not in best:
            continue
        bb = best[name]
        for cs in (512, 1024, 4096):
            kw2 = dict(bb["kw"], cache_slots=cs)
            sec = timed(bb["mode"], bb["beam"], **kw2)
            log(f"{name:14s} b={bb['beam']:5d} cache_slots={cs}: qps={nq / sec:,.0f}")
            if nq / sec > bb["qps"]:
                best[name] = dict(bb, qps=nq / sec, kw=kw2)
                bb = best[name]
    # the library's autotuner picks the adaptive setting on the even-numbered
    # queries (beam for the target, then the beam kernel's shape), then
    # Algorithm 5's parameters for that beam from the early-stopping metrics
    # (the hand setting vl=10, esr=r competes); the odd-numbered queries are
    # held out to report the setting's recall
    q_tune = q[0::2].contiguous()
    truth_tune = rr.brute_force_async(ix, q_tune, radius)
    sp, tune = rr.autotune(ix, q_tune, radius, truth_tune, target=args.target, reps=5,
                           mode="adaptive", **es_kw)
    log(f"autotune (even queries): {tune}")
    sp, es_tune = rr.tune_early_stop(ix, q_tune, radius, truth_tune, target=args.target, reps=5,
                                     params=sp)
    es_kw = dict(es_enable=bool(sp.es_enable), es_visit_limit=sp.es_visit_limit,
                 es_radius=sp.es_radius)
    log(f"early-stop tuning (even queries): {es_tune}")
    odd = np.arange(1, nq, 2)
    ho = rr.range_search(ix, q[1::2].contiguous(), radius, params=sp, with_stats=False)
    ho_off, ho_ids, _ = ho.numpy()
    odd_mask = np.isin(truth_keys // n, odd)
    rec_heldout = recall_of(ho_off, ho_ids, truth_keys[odd_mask], n, int(odd_mask.sum()), qmap=odd)
    al = rr.range_search(ix, q, radius, params=sp, with_stats=False)
    al_off, al_ids, _ = al.numpy()
    rec_all = recall_of(al_off, al_ids, truth_keys, n, truth_total)
    log(f"tuned setting: recall {rec_heldout:.4f} on the held-out odd queries, {rec_all:.4f} on all")
    A = dict(mode="adaptive", beam=sp.beam, recall=rec_heldout, recall_all=rec_all,
             recall_tuning=es_tune["recall"],
             kw=dict(es_kw, waves_per_group=sp.waves_per_group, cache_slots=sp.cache_slots))
    if args.choice:
        json.dump(dict(radius=radius, mode=A["mode"], beam=A["beam"], kw=A["kw"]),
                  open(args.choice, "w"))

    # timed steps: the chosen adaptive setting
    for _ in range(args.warmup):
        run(A["mode"], A["beam"], **A["kw"])
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        rr.range_search(ix, q, radius, mode=A["mode"], beam=A["beam"], with_stats=False, **A["kw"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    ms_step = wall / args.steps * 1e3
    qps = nq / (wall / args.steps)

    # roofline of the dominant kernel, HIP events recorded by the library on
    # the stream the kernels run on
    beam_ms, gk_ms, greedy_ms, total_ms = [], [], [], []
    st = None
    for _ in range(5):
        res = run(A["mode"], A["beam"], timing=True, **A["kw"])
        st = res.batch
        beam_ms.append(st["beam_ms"])
        gk_ms.append(st["greedy_kernel_ms"])
        greedy_ms.append(st["greedy_ms"])
        total_ms.append(st["total_ms"])
    traffic = load_traffic(f"u8-1M-d128_adaptive-b{A['beam']}") if n == 1_000_000 else None

    def roof(kernel, nbytes, ms, tkey):
        ach = nbytes / (ms * 1e-3) / 1e9
        # the record's keys are the profiler's kernel names, arguments included
        t = next((v for k, v in (traffic or {}).items() if k.startswith(tkey)), None)
        return dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4), traffic=t, kernel=kernel,
                    bytes_per_launch=int(nbytes), avg_ms=round(ms, 4))

    r_beam = roof("k_beam", st["bytes_beam"], float(np.mean(beam_ms)), "k_beam<0, 1, 8>")
    r_greedy = (roof("k_greedy", st["bytes_greedy"], float(np.mean(gk_ms)), "k_greedy<0, 1, 8>")
                if st["greedy_kernel_ms"] > 0 else None)
    dominant = r_greedy if r_greedy and r_greedy["avg_ms"] > r_beam["avg_ms"] else r_beam
    log(f"adaptive b={A['beam']}: {qps:,.0f} QPS; beam kernel {r_beam['avg_ms']:.3f} ms "
        f"({r_beam['achieved']:.0f} GB/s), greedy kernel {np.mean(gk_ms):.3f} ms "
        f"({r_greedy['achieved'] if r_greedy else 0:.0f} GB/s), greedy phase {np.mean(greedy_ms):.3f} ms, "
        f"call {np.mean(total_ms):.3f} ms; greedy levels {st['greedy_levels']}, items {st['greedy_items']}, "
        f"set ops {st['greedy_set_ops']}, "
        f"tasks {st['expanded']}, evals {st['greedy_evals']}, beam visits {st['visits']}, "
        f"beam evals {st['evals']}, cache overflow {st['cache_overflow']}")

    # serving: Poisson arrivals, each request with its own radius, continuous
    # batching over resident slots (the library's serving loop)
    levels = [float(nn_sorted[math.ceil(f * nq) - 1]) for f in (0.20, 0.25, 0.30)]
    serving = serve_leg(rr, ix, w.queries, q, n, levels, sp, args)

    # CPU oracle on the host cores, bounded sample
    cpu = None
    if not args.no_cpu:
        import oracle
        adj, entry = ix.graph()
        # batches of growing size from the start of the query set, wrapping
        # around to its start again, until about cpu_seconds of work
        ids_done, t_cpu, m = 0, 0.0, 64
        while t_cpu < args.cpu_seconds and ids_done < 100 * nq:
            s0 = ids_done % nq
            k = min(m, nq - s0)
            t = time.perf_counter()
            oracle.range_search(w.base, adj, entry, w.queries[s0:s0 + k], radius,
                                mode=oracle.ADAPTIVE, beam=A["beam"],
                                es_enable=es_kw["es_enable"], es_visit_limit=es_kw["es_visit_limit"],
                                es_radius=es_kw["es_radius"], threads=threads)
            t_cpu += time.perf_counter() - t
            ids_done += k
            m = min(2 * m, nq)
        # the same oracle on one thread, over the first 2,000 queries
        k1 = min(2000, nq)
        t = time.perf_counter()
        oracle.range_search(w.base, adj, entry, w.queries[:k1], radius, mode=oracle.ADAPTIVE,
                            beam=A["beam"], es_enable=es_kw["es_enable"],
                            es_visit_limit=es_kw["es_visit_limit"], es_radius=es_kw["es_radius"],
                            threads=1)
        t1 = time.perf_counter() - t
        cpu = dict(value=round(ids_done / t_cpu, 1), unit="queries/s", cores=threads, kind="oracle",
                   sample=f"{ids_done} query searches ({ids_done / nq:.1f} passes over the {nq} queries), "
                          f"adaptive b={A['beam']} with the tuned early stop, {t_cpu:.1f}s",
                   host=cpus, one_thread_qps=round(k1 / t1, 1),
                   one_thread_sample=f"the first {k1} queries once, {t1:.1f}s")
        log(f"cpu oracle: {cpu['value']:,.0f} QPS on {threads} threads ({cpus['model']}; nproc "
            f"{cpus['nproc']}, affinity {cpus['affinity']}, quota {cpus['cgroup_quota']}), "
            f"{cpu['one_thread_qps']:,.0f} QPS on one thread")

    plain = best.get("plain")
    dbl = max((best[k] for k in ("doubling", "doubling_es") if k in best), key=lambda x: x["qps"],
              default=None)
    out = {
        "metric": "range QPS at 0.9 range recall (adaptive search, 1 GPU)",
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"u8 d=128, {n} base, {nq} queries, latent mixture of 1000 clusters "
                               f"(16-dim centre sheet, 10-dim cluster bases, 10% near-duplicate "
                               f"groups, Zipf sizes; synth.latent_mixture_u8 seed 1); Vamana R=64 "
                               f"L=128 alpha=1.2; radius at 75% empty queries",
                   "radius": radius, "beam": A["beam"], "es_enable": es_kw["es_enable"],
                   "es_visit_limit": es_kw["es_visit_limit"], "es_radius": es_kw["es_radius"],
                   "recall": round(A["recall"], 4), "recall_scope": "held-out odd queries "
                   "(setting tuned on the even ones)", "recall_all": round(A["recall_all"], 4),
                   "result_hist_0_10_1e2_1e3_1e4_1e5": hist, "max_results": int(counts.max())},
        "roofline": dominant,
        "roofline_beam": r_beam,
        "roofline_greedy": r_greedy,
        "cpu_baseline": cpu,
        "autotune": tune,
        "es_tune": es_tune,
        "plain_qps_at_0.9": round(plain["qps"], 1) if plain else None,
        "plain_beam_at_0.9": plain["beam"] if plain else None,
        "plain_setting": plain["kw"] if plain else None,
        "es_qps_at_0.9": round(best["es"]["qps"], 1) if "es" in best else None,
        "adaptive_vs_plain": round(qps / plain["qps"], 2) if plain else None,
        "doubling_qps_at_0.9": round(dbl["qps"], 1) if dbl else None,
        "doubling_beam_at_0.9": dbl["beam"] if dbl else None,
        "adaptive_vs_doubling": round(qps / dbl["qps"], 2) if dbl else None,
        "p50_latency_ms": max(r["p50_ms"] for r in serving["rates"]) if serving else None,
        "p99_latency_ms": max(r["p99_ms"] for r in serving["rates"]) if serving else None,
        "p99_latency_note": "worst offered rate; per rate in serving.rates",
        "serving": serving,
        "batch_latency_ms": round(ms_step, 4),
        "gt_scan": {"kernel": "k_scan_int (MFMA i32_16x16x64_i8)", "ms": round(nn_ms, 3),
                    "tops": round(scan_tops, 1), "peak_tops": INT8_PEAK_TOPS,
                    "frac": round(scan_tops / INT8_PEAK_TOPS, 4)},
        "graph_build_s": round(build_s, 1) if build_s else None,
        "random_row_gather": gather,
        "greedy": {"phase_ms": round(float(np.mean(greedy_ms)), 4),
                   "kernel_ms": round(float(np.mean(gk_ms)), 4),
                   "levels": st["greedy_levels"], "items": st["greedy_items"],
                   "tasks": st["expanded"], "set_ops": st["greedy_set_ops"],
                   "level_profile": st["levels"]},
        "curves": curves,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
