#!/usr/bin/env python
"""Range-search benchmark on one MI355X.

Workload: 1,000,000 uint8 base vectors (d=128) and 10,000 queries from a
seeded 1,000-centre Gaussian mixture (per-cluster scale spread, Zipf weights),
a Vamana graph (R=64, L=128, alpha=1.2), and a squared-L2 radius at which 75%
of the queries have no result (the 25th percentile of per-query nearest-
neighbour distances).  Ground truth comes from the library's MFMA scan.

For each search mode (plain beam, beam + early stop, adaptive = beam + early
stop + greedy expansion) the beam width is swept; the fastest setting whose
range recall is >= 0.9 is kept (the Pareto point at 0.9).  The timed steps
run the adaptive setting: one step = one rr_range_search call over the whole
batch (query prep, beam kernel, greedy phase, compaction) plus the copy of
the CSR result, with the queries already in HBM.

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


def load_traffic(tag):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/), or
    None when the kernel source changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}.md")
    if not os.path.exists(path):
        return None
    src = os.path.join(ROOT, "paper_2502_13245_amd", "csrc", "rr_kernels.hip")
    sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    for line in open(path):
        if line.startswith("TRAFFIC "):
            rec = json.loads(line[len("TRAFFIC "):])
            if rec.get("kernel_source_sha1") == sha:
                return rec["bytes_per_launch"]
    return None


def recall_of(found_off, found_ids, truth_keys, n, truth_total):
    """Range recall (average precision of the paper): sum |K & K'| / sum |K|."""
    nq = len(found_off) - 1
    q = np.repeat(np.arange(nq, dtype=np.int64), np.diff(found_off))
    keys = q * n + found_ids.astype(np.int64)
    hit = np.isin(keys, truth_keys, assume_unique=True).sum()
    return float(hit) / truth_total if truth_total else float("nan")


def serve_leg(rr, ix, w, nn_sorted, sp, args):
    """Open-loop serving run per offered rate: arrival times from a Poisson
    process, queries cycled from the query set, each request's radius drawn
    from three levels (the radii at which 80%, 75% and 70% of the queries
    have no result).  Latency = completion time (results on the host) minus
    scheduled arrival time, so submitter lag counts against the server."""
    if args.serve_seconds <= 0:
        return None
    nq = len(w.queries)
    levels = [float(nn_sorted[math.ceil(f * nq) - 1]) for f in (0.20, 0.25, 0.30)]
    rng = np.random.default_rng(7)
    rates = [float(x) for x in args.serve_rates.split(",")]
    out = []
    for rate in rates:
        m = max(1, int(rate * args.serve_seconds))
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=m)) + 0.01
        qidx = rng.integers(0, nq, size=m)
        radii = np.asarray(levels)[rng.integers(0, 3, size=m)]
        qs = np.ascontiguousarray(w.queries[qidx])
        with rr.Server(ix, sp, slots=args.serve_slots, step_budget=args.serve_budget) as srv:
            t_base = srv.clock()
            arr = arrivals + t_base
            i = 0
            while i < m:
                now = srv.clock()
                while i < m and arr[i] <= now:
                    if not srv.submit(qs[i], radii[i], i, float(arr[i])):
                        break
                    i += 1
                if i < m:
                    wait = arr[i] - srv.clock()
                    if wait > 2e-4:
                        time.sleep(min(wait, 2e-3) - 1e-4)
            srv.drain(timeout=120.0)
            comps = srv.poll(m + 16)
            info = srv.info()
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
                   mean_ticks=round(float(ticks.mean()), 2), server_ticks=info["ticks"],
                   max_resident=info["max_resident"], truncated=trunc)
        log(f"serve {rate:>8,.0f} QPS offered: achieved {rec['achieved_qps']:,.0f}, "
            f"p50 {rec['p50_ms']:.3f} ms, p99 {rec['p99_ms']:.3f} ms, mean ticks "
            f"{rec['mean_ticks']}, server ticks {info['ticks']}, max resident {info['max_resident']}")
        out.append(rec)
    return dict(slots=args.serve_slots, step_budget=args.serve_budget, radius_levels=levels,
                mode="adaptive", beam=sp.beam, rates=out)


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
    ap.add_argument("--serve-budget", type=int, default=32)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; this build has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2502_13245_amd import rr, synth

    threads = args.threads or min(16, os.cpu_count() or 1)
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
    # the library's autotuner picks the adaptive setting: beam for the target,
    # then the beam kernel's shape
    sp, tune = rr.autotune(ix, q, radius, truth_h, target=args.target, reps=5, mode="adaptive",
                           **es_kw)
    log(f"autotune: {tune}")
    # then Algorithm 5's parameters for that beam, from the early-stopping
    # metrics (the hand setting vl=10, esr=r competes)
    sp, es_tune = rr.tune_early_stop(ix, q, radius, truth_h, target=args.target, reps=5, params=sp)
    es_kw = dict(es_enable=bool(sp.es_enable), es_visit_limit=sp.es_visit_limit,
                 es_radius=sp.es_radius)
    log(f"early-stop tuning: {es_tune}")
    A = dict(mode="adaptive", beam=sp.beam, recall=es_tune["recall"],
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
        t = None
        if traffic and tkey in traffic:
            t = traffic[tkey]
        return dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4), traffic=t, kernel=kernel,
                    bytes_per_launch=int(nbytes), avg_ms=round(ms, 4))

    log(f"greedy levels: {st['levels']}")
    r_beam = roof("k_beam", st["bytes_beam"], float(np.mean(beam_ms)), "k_beam<0, 1, 8>")
    r_greedy = (roof("k_greedy", st["bytes_greedy"], float(np.mean(gk_ms)), "k_greedy<0, 1, 8>")
                if st["greedy_kernel_ms"] > 0 else None)
    dominant = r_greedy if r_greedy and r_greedy["avg_ms"] > r_beam["avg_ms"] else r_beam
    log(f"adaptive b={A['beam']}: {qps:,.0f} QPS; beam kernel {r_beam['avg_ms']:.3f} ms "
        f"({r_beam['achieved']:.0f} GB/s), greedy kernel {np.mean(gk_ms):.3f} ms "
        f"({r_greedy['achieved'] if r_greedy else 0:.0f} GB/s), greedy phase {np.mean(greedy_ms):.3f} ms, "
        f"call {np.mean(total_ms):.3f} ms; greedy levels {st['greedy_levels']}, items {st['greedy_items']}, "
        f"tasks {st['expanded']}, evals {st['greedy_evals']}, beam visits {st['visits']}, "
        f"beam evals {st['evals']}, cache overflow {st['cache_overflow']}")

    # serving: Poisson arrivals, each request with its own radius, continuous
    # batching over resident slots (the library's serving loop)
    serving = serve_leg(rr, ix, w, nn_sorted, sp, args)

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
        cpu = dict(value=round(ids_done / t_cpu, 1), unit="queries/s", cores=threads, kind="oracle",
                   sample=f"{ids_done} query searches ({ids_done / nq:.1f} passes over the {nq} queries), "
                          f"adaptive b={A['beam']} with the tuned early stop, {t_cpu:.1f}s")
        log(f"cpu oracle: {cpu['value']:,.0f} QPS on {threads} threads")

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
        "config": {"workload": f"u8 d=128, {n} base, {nq} queries, 1000-centre mixture; "
                               f"Vamana R=64 L=128 alpha=1.2; radius at 75% empty queries",
                   "radius": radius, "beam": A["beam"], "es_enable": es_kw["es_enable"],
                   "es_visit_limit": es_kw["es_visit_limit"], "es_radius": es_kw["es_radius"], "recall": round(A["recall"], 4),
                   "result_hist_0_10_1e2_1e3_1e4_1e5": hist, "max_results": int(counts.max())},
        "roofline": dominant,
        "roofline_beam": r_beam,
        "roofline_greedy": r_greedy,
        "cpu_baseline": cpu,
        "autotune": tune,
        "es_tune": es_tune,
        "plain_qps_at_0.9": round(plain["qps"], 1) if plain else None,
        "plain_beam_at_0.9": plain["beam"] if plain else None,
        "es_qps_at_0.9": round(best["es"]["qps"], 1) if "es" in best else None,
        "adaptive_vs_plain": round(qps / plain["qps"], 2) if plain else None,
        "doubling_qps_at_0.9": round(dbl["qps"], 1) if dbl else None,
        "doubling_beam_at_0.9": dbl["beam"] if dbl else None,
        "adaptive_vs_doubling": round(qps / dbl["qps"], 2) if dbl else None,
        "p50_latency_ms": serving["rates"][-1]["p50_ms"] if serving else None,
        "p99_latency_ms": serving["rates"][-1]["p99_ms"] if serving else None,
        "serving": serving,
        "batch_latency_ms": round(ms_step, 4),
        "gt_scan": {"kernel": "k_scan_int (MFMA i32_16x16x64_i8)", "ms": round(nn_ms, 3),
                    "tops": round(scan_tops, 1), "peak_tops": INT8_PEAK_TOPS,
                    "frac": round(scan_tops / INT8_PEAK_TOPS, 4)},
        "graph_build_s": round(build_s, 1) if build_s else None,
        "random_row_gather": gather,
        "greedy": {"phase_ms": round(float(np.mean(greedy_ms)), 4),
                   "kernel_ms": round(float(np.mean(gk_ms)), 4), "levels": st["greedy_levels"],
                   "items": st["greedy_items"], "tasks": st["expanded"],
                   "levels": st["levels"]},
        "curves": curves,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
