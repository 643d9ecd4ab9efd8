"""Benchmark: exact 1-NN queries/s on 10,000,000 x 256 float32 random walks (one MI355X).

A step answers the workload's query set through the plain per-query path (paris_query_exact:
prepare -> approximate-search seed -> lower-bound scan -> early-abandoning refine -> float64
resolve, one query at a time with its result back on the host), over an index built once before
the timed region (the build time is reported beside). Inputs are resident in HBM before timing.

Beside the headline the default run records: the scan cold (caches swept before every query);
the best-so-far sharing ablation on hard queries (with the refine kernel's bytes per second);
exact k-NN (k = 10 and 64) on 200 of the queries; the ADS+ tree leaf mode and the collection in
pinned host memory (out of core);
batches of 4096 through the batched pipeline (paris_query_batch) with a brute-force check of 64
of their answers; the CPU oracle (brute force over all host threads, and on one thread the
median latency of brute force and of the serial exact-search twin over 20 queries); the learned
seed on 50,000,000 x 256 with 4096 equal-count leaves; and the mixed-length workload
(100M x 128 + 20M x 512 + 5M x 1024 in one call per batch of 2048).

Prints one JSON line. Options: --gpus N (only 1 is supported: the benchmark measures one GPU),
--steps K, --warmup W, --queries Q, --series N, --length n, --fresh-queries (new random walks
as queries, the paper's workload), --no-cpu-baseline, --cpu-single S, --oracle-check C,
--no-knn, --no-tree, --no-batched, --batch B, --batch-steps K, --cold-queries C, --no-nb-ablation, --no-learned,
--learned-series N (0: the main collection), --train-queries T, --epochs E, --eval-queries V,
--learned-only, --multi (only the mixed-length workload), --no-multi, --multi-scale F.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E peak (8 TB/s)
SAX_BYTES_PER_SERIES = 16
ENV_BYTES_PER_SERIES = 1      # a run's symbol envelope (32 B per 32 series), read by the scan's run pass
SURVIVOR_BYTES = 12           # a survivor's series index (perm, 4 B) and its list entry (8 B)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_10Mx256.md")
KERNEL_SOURCES = {"k_lbscan": "paris_query.hip", "k_screen": "paris_batch.hip"}


def source_digest(kernel: str) -> str:
    """Digest of the source file that holds a kernel, comments and whitespace removed: the
    measured HBM traffic of a kernel is reported only while this digest is unchanged."""
    import hashlib
    import re
    path = os.path.join(ROOT, "paper_2009_00166_amd", "csrc", KERNEL_SOURCES[kernel])
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    txt = re.sub(r"//[^\n]*", "", txt)
    txt = re.sub(r"\s+", " ", txt).strip()
    return hashlib.sha256(txt.encode()).hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or
    None when it is absent or the kernel's source has changed since it was taken."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    vals = {}
    for ln in lines:
        if ln.startswith(f"{kernel}.") and "=" in ln:
            k, v = ln.split("=", 1)
            vals[k.strip()[len(kernel) + 1:]] = v.strip()
    if vals.get("source_digest") != source_digest(kernel) or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(X, Q, gpu_idx, n_queries: int, threads: int, single: int):
    """The C oracle on bounded samples of the same workload: brute force (float64, the
    definition) over all host threads, then on one thread the median latency of brute force and
    of the serial exact-search twin (ExactSearch with its lower-bound and distance workers,
    Section 3.3.3, run by one thread: approximate-search seed, float64 lower bound of every
    series, sorted candidates, early-abandoning distances), over ``single`` queries each."""
    import statistics
    import numpy as np
    from oracle import native
    native.build(force=False)
    sample = Q[:n_queries]
    t0 = time.perf_counter()
    ri, rd, used = native.nn_many(sample, X, threads=threads)
    dt = time.perf_counter() - t0
    agrees = bool(np.array_equal(ri, np.asarray(gpu_idx[:n_queries])))
    log(f"cpu oracle: {n_queries} brute-force queries in {dt:.1f}s on {used} threads")
    base = {"value": n_queries / dt, "unit": "queries/s", "cores": int(used), "kind": "oracle",
            "sample": f"first {n_queries} of the {Q.shape[0]} queries against the full "
                      f"{X.shape[0]}x{X.shape[1]} collection, brute-force float64 C oracle "
                      f"(-O2, no FMA), queries split over {used} threads",
            "seconds": dt, "answers_agree_with_gpu": agrees,
            "host": {"cpu_count": os.cpu_count(), "model": cpu_model(), "threads_used": int(used)}}
    if single <= 0:
        return base
    bf_ms, tw_ms, tw_ok = [], [], True
    for m in range(single):
        t1 = time.perf_counter()
        i, _, _ = native.nn_many(Q[m:m + 1], X, threads=1)
        bf_ms.append((time.perf_counter() - t1) * 1e3)
        tw_ok &= int(i[0]) == int(gpu_idx[m])
    log(f"cpu oracle: {single} single-thread brute-force queries, median {statistics.median(bf_ms):.0f} ms")
    t2 = time.perf_counter()
    ix = native.SearchIndex(X)
    prep_s = time.perf_counter() - t2
    counters = []
    for m in range(single):
        mem = ix.members(Q[m])     # leaf lookup (numpy), outside the timed call
        t1 = time.perf_counter()
        i, _, st = native.exact_search(Q[m], ix, members=mem)
        tw_ms.append((time.perf_counter() - t1) * 1e3)
        tw_ok &= i == int(gpu_idx[m])
        counters.append(st)
    log(f"cpu oracle: {single} single-thread exact-search twin queries, median {statistics.median(tw_ms):.0f} ms")
    mean = lambda k: float(np.mean([c[k] for c in counters]))
    return {**base, "single_thread": {
                "queries": single,
                "brute_force_median_ms": statistics.median(bf_ms),
                "exact_search_twin_median_ms": statistics.median(tw_ms),
                "twin_mean_lb_survivors": mean("lb_survivors"), "twin_mean_refined": mean("refined"),
                "twin_index_prep_s": prep_s,
                "answers_agree_with_gpu": bool(tw_ok),
                "note": "one thread each; brute force = the definition (every distance in float64); "
                        "twin = serial C ExactSearch (seed over the approximate search's leaf, float64 "
                        "lower bound of every series, candidates sorted by bound, early abandoning); "
                        "its words and leaf order are prepared once by the numpy oracle (twin_index_prep_s)"}}


def bsf_sharing_ablation(index, X, n: int, count: int = 200):
    """Hard queries (dataset series + N(0, 0.5) noise) through the plain path with the shared
    best-so-far of ParIS+ and with one private copy per distance worker, nb-ParIS+'s design
    (Section 3.3): answers, refined rows and queries/s of both (not part of the headline)."""
    import numpy as np
    import torch
    import synth
    Q, _, _ = synth.noisy_queries(X, count, seed=4, sigma=0.5)
    Qd = torch.from_numpy(Q).to("cuda:0")
    rows = [Qd[m] for m in range(count)]

    def run():
        index.query(rows[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        got = [index.query(r)[0] for r in rows]
        torch.cuda.synchronize()
        qps = count / (time.perf_counter() - t0)
        st = [index.query(r, with_stats=True)[2] for r in rows]
        mean = lambda k: float(np.mean([x[k] for x in st]))
        # one more pass with events between the phases: the refine + resolve kernel's time
        index.set_timing(True)
        for r in rows:
            index.query(r)
        ms, k = index.timing()
        index.set_timing(False)
        ref_ms = ms[2] / max(k, 1)
        # a refined row's first 64 points (256 B) are read with it; the rest only when those did
        # not abandon it: refined x 4n bounds the bytes from above, refined x 256 B from below
        row_bytes = 4 * n
        read = mean("refined") * row_bytes
        read_lo = mean("refined") * min(row_bytes, 256)
        return {"queries_per_s": qps, "mean_lb_survivors": mean("lb_survivors"),
                "mean_refined": mean("refined"), "mean_abandoned": mean("abandoned"),
                "mean_bsf_updates": mean("bsf_updates"),
                "mean_raw_bytes_read": read,
                "refine_roofline": {"bound": "hbm", "kernel": "k_refine_resolve",
                                    "bytes_per_launch": read, "avg_launch_ms": ref_ms,
                                    "achieved": read / (ref_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBPS,
                                    "unit": "GB/s", "frac": read / (ref_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                                    "note": "bytes = refined rows x 4n, an upper bound (a row abandoned within its first "
                                            "64 points reads 256 B: bytes_lower_bound); time from events recorded "
                                            "around the refine + resolve launch (includes its dispatch gap)",
                                    "bytes_lower_bound": read_lo,
                                    "achieved_lower_bound": read_lo / (ref_ms * 1e-3) / 1e9}}, got

    # alternate the modes twice and keep each one's faster pass, so neither gains from going last
    res = {True: [], False: []}
    try:
        for shared in (True, False, True, False):
            index.set_bsf_sharing(shared)
            res[shared].append(run())
    finally:
        index.set_bsf_sharing(False)    # the library's default
    best = lambda r: max(r, key=lambda x: x[0]["queries_per_s"])
    (shared, a), (private, b) = best(res[True]), best(res[False])
    return {"queries": f"{count} hard queries (dataset series + N(0,0.5) noise)", "shared": shared,
            "private": private, "answers_identical": bool(a == b),
            "passes": "two per mode, alternated; the faster of each mode's passes"}


def knn_section(index, X, Q, args, count: int = 200):
    """Exact k-NN (k = 10 and 64) through paris_query_knn on the first queries of the plain
    workload: queries/s, counters, and the answers of a few queries against the k-NN by
    definition (the C oracle's float64 distances ordered by (distance, index))."""
    import numpy as np
    import torch
    Qd = torch.from_numpy(np.ascontiguousarray(Q[:count])).to("cuda:0")
    rows = [Qd[m] for m in range(Qd.shape[0])]
    out = {"queries": f"first {len(rows)} queries of the plain workload"}
    for k in (10, 64):
        for r in rows[:10]:
            index.query_knn(r, k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        got = [index.query_knn(r, k) for r in rows]
        dt = time.perf_counter() - t0
        st = [index.query_knn(r, k, with_stats=True)[2] for r in rows[:50]]
        mean = lambda key: float(np.mean([x[key] for x in st]))
        rec = {"queries_per_s": len(rows) / dt, "mean_lb_survivors": mean("lb_survivors"),
               "mean_refined": mean("refined"), "mean_resolved": mean("resolved")}
        if not args.no_cpu_baseline:
            from concurrent.futures import ThreadPoolExecutor
            from oracle import native
            native.build(force=False)
            kk = 4
            with ThreadPoolExecutor(max_workers=kk) as ex:
                d2s = list(ex.map(lambda q: native.ed2(q, X), Q[:kk]))
            ok = True
            for m in range(kk):
                order = np.lexsort((np.arange(X.shape[0]), d2s[m]))[:k]
                ok &= bool(np.array_equal(got[m][0], order) and np.array_equal(got[m][1], np.sqrt(d2s[m][order])))
            rec["oracle_check"] = {"queries": kk, "answers_equal_oracle": ok}
        out[f"k{k}"] = rec
        log(f"k-NN k={k}: {rec['queries_per_s']:.0f} queries/s")
    return out


def tree_and_host_section(index, X, Q, answers, args):
    """The ADS+ tree leaf mode (Section 2.2 node splitting, bulk loaded on the GPU) and the
    out-of-core collection (raw series in pinned host memory, index in HBM, rows read over PCIe)
    on the main collection: build times, tree shape, per-query queries/s on the plain workload's
    queries and on hard ones (noise 0.5), batched queries/s, answers against the in-HBM root16
    index."""
    import numpy as np
    import torch
    import paper_2009_00166_amd as paris
    import synth
    N, n = X.shape
    M = min(1000, Q.shape[0])
    Qd = torch.from_numpy(np.ascontiguousarray(Q[:M])).to("cuda:0")
    rows = [Qd[m] for m in range(M)]
    Qh, _, _ = synth.noisy_queries(X, 200, seed=4, sigma=0.5)
    Qhd = torch.from_numpy(Qh).to("cuda:0")
    hrows = [Qhd[m] for m in range(Qh.shape[0])]
    ref_h = [index.query(r)[0] for r in hrows]

    def per_query(ix, rs):
        for r in rs[:20]:
            ix.query(r)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        got = [ix.query(r)[0] for r in rs]
        return len(rs) / (time.perf_counter() - t0), got

    def batched(ix):
        B = args.batch
        Qb, _, _ = synth.noisy_queries(X, B, seed=1, sigma=(0.01, 0.5))
        Qbd = torch.from_numpy(Qb).cuda()
        ix.attach_batch(max_batch=B)
        I, D = ix.query_batch(Qbd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            ix.query_batch(Qbd, out=(I, D))
        torch.cuda.synchronize()
        return B * args.batch_steps / (time.perf_counter() - t0), I.cpu().numpy(), Qbd

    out = {}
    Xd = index.series
    t0 = time.perf_counter()
    tree = paris.build(Xd, leaf_mode=paris.LEAF_ADS, leaf_cap=2048)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t = tree.tree_nodes()
    leaves = t["child0"] < 0
    sizes = (t["end"] - t["start"])[leaves]
    qps, got = per_query(tree, rows)
    hqps, hgot = per_query(tree, hrows)
    out["ads_tree"] = {"leaf_cap": 2048, "build_ms": tb * 1e3, "nodes": int(len(t["start"])),
                       "leaves_nonempty": int((sizes > 0).sum()), "largest_leaf": int(sizes.max()),
                       "mean_nonempty_leaf": float(sizes[sizes > 0].mean()),
                       "per_query_queries_per_s": qps, "hard_queries_per_s": hqps,
                       "answers_equal_root16": bool(np.array_equal(got, answers[:M]) and hgot == ref_h)}
    log(f"ADS+ tree: built in {tb * 1e3:.0f} ms, {len(t['start'])} nodes; {qps:.0f} q/s, hard {hqps:.0f} q/s")
    tree.close()
    # out of core: the same series in pinned host memory
    coll = paris.HostCollection(N, n)
    np.copyto(coll.array, X)
    t0 = time.perf_counter()
    host = paris.build(coll)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    qps, got = per_query(host, rows)
    hqps, hgot = per_query(host, hrows)
    bqps, bI, Qbd = batched(host)
    ref_b, _ = index.query_batch(Qbd)
    torch.cuda.synchronize()
    out["host_collection"] = {
        "where": f"{N} x {n} float32 ({X.nbytes / 1e9:.1f} GB) in pinned host memory mapped for the GPU; "
                 "index, iSAX words and the batched path's bfloat16 copy in HBM",
        "build_ms": tb * 1e3, "build_GBps_raw_over_pcie": X.nbytes / tb / 1e9,
        "per_query_queries_per_s": qps, "hard_queries_per_s": hqps, "batched_queries_per_s": bqps,
        "answers_equal_in_hbm": bool(np.array_equal(got, answers[:M]) and hgot == ref_h
                                     and np.array_equal(bI, ref_b.cpu().numpy()))}
    log(f"host collection: built in {tb * 1e3:.0f} ms; {qps:.0f} q/s, hard {hqps:.0f} q/s, batched {bqps:.0f} q/s")
    host.close()
    coll.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--queries", type=int, default=1000)
    ap.add_argument("--series", type=int, default=10_000_000)
    ap.add_argument("--length", type=int, default=256)
    ap.add_argument("--sigma", type=float, default=0.1)
    ap.add_argument("--fresh-queries", action="store_true",
                    help="plain path: queries are new random walks (the paper's query workload) "
                         "instead of dataset series plus noise")
    ap.add_argument("--no-nb-ablation", dest="nb_ablation", action="store_false",
                    help="skip the best-so-far sharing ablation (shared vs private copies, hard queries)")
    ap.add_argument("--cpu-queries", type=int, default=16)
    ap.add_argument("--cpu-threads", type=int, default=16)
    ap.add_argument("--cpu-single", type=int, default=20,
                    help="queries timed on one thread (brute force and the serial exact-search twin)")
    ap.add_argument("--oracle-check", type=int, default=64,
                    help="batched answers checked against the brute-force oracle per batch record")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-knn", action="store_true", help="skip the exact k-NN sub-record")
    ap.add_argument("--no-tree", action="store_true",
                    help="skip the ADS+ tree and host-resident collection sub-record")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--cold-queries", type=int, default=200)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--train-queries", type=int, default=200_000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--eval-queries", type=int, default=1000)
    ap.add_argument("--learned-series", type=int, default=50_000_000,
                    help="collection size of the learned-seed section (0: the main collection)")
    ap.add_argument("--learned-only", action="store_true", help="run only the learned-seed section")
    ap.add_argument("--multi", action="store_true",
                    help="only the mixed-length workload: 100M x 128 + 20M x 512 + 5M x 1024")
    ap.add_argument("--no-multi", action="store_true",
                    help="skip the mixed-length sub-record of the default run")
    ap.add_argument("--multi-scale", type=float, default=1.0,
                    help="fraction of the mixed-length collections' sizes (1.0 = full)")
    args = ap.parse_args()
    args._plain_qps = None

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the exact search is built and measured on a single "
              "MI355X (run with --gpus 1).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2009_00166_amd as paris
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    if args.multi:
        rec = multi_section(args)
        print(json.dumps(rec), flush=True)
        return 0
    if args.learned_only:
        args._plain_qps = None
        N = args.learned_series or args.series
        X = synth.random_walks(N, args.length, seed=0, threads=16)
        rec = {"metric": "learned best-so-far seed", "learned": learned_section(torch.from_numpy(X).to(dev), X, args)}
        print(json.dumps(rec), flush=True)
        return 0
    N, n, M = args.series, args.length, args.queries

    t0 = time.perf_counter()
    X = synth.random_walks(N, n, seed=0, threads=16)
    if args.fresh_queries:
        Q, src = synth.fresh_walk_queries(M, n, seed=0), None
        qdesc = "new z-normalised random walks"
    else:
        Q, src, _ = synth.noisy_queries(X, M, seed=0, sigma=args.sigma)
        qdesc = f"dataset series + N(0,{args.sigma}) noise"
    log(f"generated {N}x{n} + {M} queries in {time.perf_counter() - t0:.1f}s")
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    torch.cuda.synchronize()

    tb = time.perf_counter()
    index = paris.build(Xd)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - tb
    log(f"built index in {build_s * 1e3:.1f} ms")

    rows = [Qd[m] for m in range(M)]
    answers = np.empty(M, np.int64)

    def step(record: bool):
        for m in range(M):
            i, _ = index.query(rows[m])
            if record:
                answers[m] = i

    for w in range(args.warmup):
        step(record=(w == 0))
        log(f"warmup step {w + 1}/{args.warmup} done")

    # timed region: a start and a stop HIP event bound to the scan kernel's dispatch in every 8th
    # query (read back one timed query late; the other queries run without events)
    index.set_timing(True, scan_only=True, sampled=True)
    torch.cuda.synchronize()
    w0 = time.clock_gettime_ns(time.CLOCK_MONOTONIC)
    t1 = time.perf_counter()
    for k in range(args.steps):
        step(record=False)
        log(f"timed step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    # the window in CLOCK_MONOTONIC nanoseconds, to pick this region's launches out of a trace
    log(f"timed window monotonic ns {w0} {time.clock_gettime_ns(time.CLOCK_MONOTONIC)}")
    scan_ms, timed = index.timing()
    lay = index.layout()
    scan_shape = {"threads": lay.scan_threads, "blocks_per_cu": lay.scan_blocks_per_cu, "unroll": lay.scan_unroll}
    # one more pass, outside the timed region, with events around all three phases
    index.set_timing(True)
    step(record=False)
    phase_ms, phased = index.timing()
    index.set_timing(False)

    # the same queries queued on the stream: the per-query kernels of query m + 1 enqueued behind
    # those of query m without waiting for its answer on the host (answers to device arrays)
    Iq = torch.empty(M, dtype=torch.int64, device=dev)
    Dq = torch.empty(M, dtype=torch.float64, device=dev)
    index.query_batch(Qd, out=(Iq, Dq))
    torch.cuda.synchronize()
    tq = time.perf_counter()
    for k in range(args.steps):
        index.query_batch(Qd, out=(Iq, Dq))
    torch.cuda.synchronize()
    queued = {"queries_per_s": M * args.steps / (time.perf_counter() - tq),
              "answers_identical": bool(np.array_equal(Iq.cpu().numpy(), answers)),
              "note": "the same queries and kernels, each query's seed, scan and refine enqueued "
                      "behind the previous query's without its answer being read back in between "
                      "(paris_query_batch with no batch workspace attached); value answers one query "
                      "at a time, each answer read back before the next query is issued"}
    log(f"queued per-query path: {queued['queries_per_s']:.0f} queries/s")

    cold = cold_scan_section(index, rows, N, args) if args.cold_queries > 0 else None

    # counters of one pass (not timed)
    stats = [index.query(rows[m], with_stats=True)[2] for m in range(min(M, 200))]
    mean = lambda k: float(np.mean([s[k] for s in stats]))
    nb = bsf_sharing_ablation(index, X, n) if args.nb_ablation else None
    knn = knn_section(index, X, Q, args) if not args.no_knn else None

    total_q = M * args.steps
    args._plain_qps = total_q / elapsed
    lb_ms = scan_ms[1] / max(timed, 1)
    # algorithmic bytes of a scan launch: the symbol envelope of every run of 32 series (1 B per
    # series), the 8-bit word of every series of the runs that pass (16 B) and every survivor's
    # series index and entry (12 B)
    lb_bytes = (ENV_BYTES_PER_SERIES * N + SAX_BYTES_PER_SERIES * mean("words_read")
                + SURVIVOR_BYTES * mean("lb_survivors"))
    achieved = lb_bytes / (lb_ms * 1e-3) / 1e9
    single_pass_GBps = SAX_BYTES_PER_SERIES * N / (lb_ms * 1e-3) / 1e9
    if cold:
        cold["achieved_GBps"] = lb_bytes / (cold["avg_launch_ms"] * 1e-3) / 1e9
        cold["frac"] = cold["achieved_GBps"] / HBM_PEAK_GBPS
    rec = {
        "metric": (f"exact 1-NN queries/s @{N / 1e6:g}M x {n} fp32 (plain per-query path)"
                   + ("" if not args.fresh_queries else ", new random-walk queries")),
        "value": total_q / elapsed,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"plain exact 1-NN: {N} x {n} z-normalised random walks, {M} queries "
                               f"({qdesc}) answered one at a time, "
                               "root-subtree leaves, lower-bound-guided approximate-leaf seed (16384), LB scan + "
                               "early-abandon refine + float64 resolve",
                   "n_series": N, "length": n, "queries_per_step": M, "leaf_mode": "root16",
                   "seed_cap": 16384},
        "roofline": {"bound": "hbm", "kernel": "k_lbscan", "achieved": achieved,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "launch_shape": scan_shape,
                     "cache_resident": bool(ENV_BYTES_PER_SERIES * N < 256e6),
                     "achieved_cold": cold["achieved_GBps"] if cold else None,
                     "frac_cold": cold["frac"] if cold else None,
                     "single_pass_equivalent_GBps": single_pass_GBps,
                     "single_pass_equivalent_frac": single_pass_GBps / HBM_PEAK_GBPS,
                     # the committed counter summary covers the 10M x 256 launch only
                     "traffic": measured_traffic("k_lbscan") if (N, n) == (10_000_000, 256) else None,
                     "bytes_per_launch": lb_bytes, "avg_launch_ms": lb_ms,
                     "note": "bytes per launch = 1 B per series (the symbol envelopes of the runs of 32 "
                             "leaf-order series, read by the run pass) + 16 B per series of the runs that pass "
                             "(its 8-bit word) + 12 B per survivor (series index and list entry), the means over "
                             "200 queries; avg_launch_ms from HIP start/stop events bound to the scan kernel's "
                             "dispatch (every 8th query of the timed region); single_pass_equivalent_GBps = 16 B "
                             "per series / that time (the rate a scan of every 8-bit word would need); the "
                             f"{ENV_BYTES_PER_SERIES * N / 1e6:g} MB of envelopes "
                             + ("fit the 256 MB Infinity Cache (achieved_cold / frac_cold: the same kernel after "
                                "a 1 GiB read-only sweep before every query)" if ENV_BYTES_PER_SERIES * N < 256e6
                                else "exceed the 256 MB Infinity Cache (streamed from HBM)")},
        "lbscan_cold": cold,
        "queued": queued,
        "phases_ms_per_query": dict(zip(["prepare_seed", "lbscan", "refine_resolve"],
                                        [p / max(phased, 1) for p in phase_ms])),
        "build_ms": build_s * 1e3,
        "build_GBps_raw": X.nbytes / build_s / 1e9,
        "mean_counters": {k: mean(k) for k in ("words_read", "lb_survivors", "refined", "abandoned",
                                               "bsf_updates", "resolved")},
        "answers_match_source_frac": None if src is None else float(np.mean(answers == src)),
        "bsf_sharing_ablation": nb,
        "knn": knn,
    }
    if not args.no_batched:
        rec["batched"] = batched_section(index, X, args)
    if not args.no_tree:
        rec["tree_and_host_collection"] = tree_and_host_section(index, X, Q, answers, args)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        rec["cpu_baseline"] = cpu_baseline(X, Q, answers, min(args.cpu_queries, M), args.cpu_threads,
                                           min(args.cpu_single, M))
    if not args.no_learned:
        if args.learned_series and args.learned_series != N:
            index.close()   # frees the library state; the workspace goes with the object
            del index, Xd, rows, Qd
            torch.cuda.empty_cache()
            XL = synth.random_walks(args.learned_series, n, seed=0, threads=16)
            log(f"generated the {args.learned_series} x {n} learned-seed collection")
            XLd = torch.from_numpy(XL).to(dev)
            rec["learned"] = learned_section(XLd, XL, args)
            del XL, XLd
            torch.cuda.empty_cache()
        else:
            rec["learned"] = learned_section(Xd, X, args)
            index.close()
    else:
        index.close()
    if not args.no_multi and not args.fresh_queries and (N, n) == (10_000_000, 256):
        # the mixed-length workload as a sub-record of the default run
        index = None
        Xd = rows = Qd = None
        torch.cuda.empty_cache()
        rec["mixed_lengths"] = multi_section(args)
    print(json.dumps(rec), flush=True)
    return 0


def cold_scan_section(index, rows, N, args):
    """The lower-bound scan with nothing of the iSAX array left in any cache: before each query
    a 1 GiB buffer is read (one reduction kernel), which replaces the contents of the 256 MB
    Infinity Cache and of the L2s with clean lines of that buffer, as the refinement's row reads
    would in a long-running service. HIP events bound to the scan kernel's dispatch then time
    the scan straight from HBM. (A flush that writes leaves dirty lines behind, whose write-back the scan would then pay
    for.) The fill kernel (1 GiB written once) and the reduction (1 GiB read) are also the
    known-size references for the HBM byte counters."""
    import torch
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
    flush.fill_(1.0)
    K = min(args.cold_queries, len(rows))
    index.set_timing(True, scan_only=True)    # events bound to the scan kernel's dispatch
    for m in range(K):
        flush.sum()
        index.query(rows[m])
    torch.cuda.synchronize()
    phase_ms, timed = index.timing()
    index.set_timing(False)
    del flush
    lb_ms = phase_ms[1] / max(timed, 1)
    log(f"cold lbscan {lb_ms * 1e3:.1f} us over {timed} queries")
    return {"avg_launch_ms": lb_ms, "queries": timed, "flush": "1 GiB read (reduction kernel) before each query"}


def batched_section(index, X, args):
    """Batches of 4096 queries with noise sigma ~ U[0.01, 0.5] through paris_query_batch
    (per-query seeds, bfloat16 MFMA screen, float32 re-score, float64 resolve; one HIP graph
    per batch) over the same 10M x 256 collection."""
    import numpy as np
    import torch

    import synth
    B = args.batch
    N, n = X.shape
    t0 = time.perf_counter()
    ws_bytes = index.attach_batch(max_batch=B)
    attach_s = time.perf_counter() - t0
    Qb, src, sig = synth.noisy_queries(X, B, seed=1, sigma=(0.01, 0.5))
    Qd = torch.from_numpy(Qb).cuda()
    I = torch.empty(B, dtype=torch.int64, device="cuda")
    D = torch.empty(B, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        index.query_batch(Qd, out=(I, D))
    torch.cuda.synchronize()
    log(f"batched warmup done (attach {attach_s * 1e3:.0f} ms)")
    t1 = time.perf_counter()
    for k in range(args.batch_steps):
        index.query_batch(Qd, out=(I, D))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    log(f"batched timed {args.batch_steps} batches")
    answers = I.cpu().numpy()
    # one more batch, launched stage by stage with HIP events, for the per-stage times
    index.screen_tiles(reset=True)
    index.set_timing(True)
    _, _, st = index.query_batch(Qd, out=(I, D), with_stats=True)
    ms, chunks = index.batch_timing()
    index.set_timing(False)
    tiles_run, tiles_dense = index.screen_tiles(reset=True)
    stage = [m / max(chunks, 1) for m in ms]
    np_ = (n + 31) // 32 * 32
    dense_flops = 2.0 * B * N * np_
    keep = tiles_run / max(tiles_dense, 1)
    # MFMA work the screen ran: the (query tile, work item) pairs the block bound kept
    flops = dense_flops * keep
    achieved = flops / (stage[2] * 1e-3) / 1e12
    qps = B * args.batch_steps / elapsed
    return {
        "metric": "exact 1-NN queries/s @10M x 256 fp32 (batched)",
        "value": qps, "unit": "queries/s", "ms_per_batch": elapsed / args.batch_steps * 1e3,
        "steps": args.batch_steps, "dtype": "bf16 screen, f32 re-score, f64 resolve",
        "config": {"workload": f"batched exact 1-NN: {N} x {n} random walks, batches of {B} queries "
                               "(dataset series + N(0, sigma) noise, sigma ~ U[0.01, 0.5]), per-query "
                               "seeds, block lower bound over leaf-order runs, bfloat16 MFMA screen with "
                               "certified margin on the kept pairs, float32 re-score, float64 resolve, "
                               "one HIP graph per batch",
                   "batch": B, "n_series": N, "length": n},
        "vs_plain": qps / args._plain_qps if args._plain_qps else None,
        "roofline": {"bound": "mfma", "kernel": "k_screen32", "achieved": achieved, "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": achieved / 2500.0, "traffic": (measured_traffic("k_screen")     # counters cover 10M x 256, 4096-query batches
                                                 if (N, n, B) == (10_000_000, 256, 4096) else None),
                     "flops_per_launch": flops, "avg_launch_ms": stage[2],
                     "note": "flops = 2 x 256 per (query, series) pair of the query tiles the block "
                             "bound kept (tiles_kept_frac of a screen of every pair)"},
        "screen_tiles_kept_frac": keep,
        "dense_equivalent_TFLOPs": dense_flops / ((stage[1] + stage[2]) * 1e-3) / 1e12,
        "stages_ms_per_batch": dict(zip(["seeds", "block_bound", "screen", "rescore", "resolve"], stage)),
        "screen_survivors_per_query": st["lb_survivors"] / B,
        "fallback_queries": st["resolved"],
        "workspace_bytes": ws_bytes,
        "answers_match_source_frac": float(np.mean(answers == src)),
        "oracle_check": oracle_check(X, Qb, answers, D.cpu().numpy(), sig, args),
    }


def oracle_check(X, Q, I, D, sig, args, seed=0):
    """Brute-force check of a batch's answers on ``args.oracle_check`` of its queries (a quarter
    of them the noisiest, the rest at random): indices equal and distances bit-identical."""
    import numpy as np
    from oracle import native
    k = min(args.oracle_check, Q.shape[0])
    if k == 0 or args.no_cpu_baseline:
        return None
    native.build(force=False)
    order = np.argsort(-np.asarray(sig), kind="stable")
    hard = k // 4
    pick = np.sort(np.concatenate([order[:hard], np.random.default_rng(seed).choice(order[hard:], k - hard,
                                                                                    replace=False)]))
    t0 = time.perf_counter()
    ri, rd, used = native.nn_many_blocked(Q[pick], X, threads=args.cpu_threads)
    dt = time.perf_counter() - t0
    log(f"oracle check: {k} queries of {X.shape[0]} x {X.shape[1]} in {dt:.1f}s")
    return {"queries": k, "indices_equal": bool(np.array_equal(ri, np.asarray(I)[pick])),
            "distances_bit_identical": bool(np.array_equal(np.sqrt(rd), np.asarray(D)[pick])),
            "selection": f"{hard} noisiest + {k - hard} at random", "seconds": dt}


def learned_section(Xd, X, args):
    """The learned best-so-far seed on the same collection: an index with 4096 equal-count leaves,
    a 16-256-256-4096 network trained on exact (query, nearest-neighbour leaf) pairs from the
    training stream (noise sigma ~ U[0.05, 0.5]), then hard queries (sigma 0.5) through the
    per-query path with the plain one-leaf seed and with the learned 8-leaf seed, and one batch
    of the batched workload through the pipeline with the learned seed."""
    import numpy as np
    import torch

    import paper_2009_00166_amd as paris
    import synth
    N, n = X.shape
    n_leaves = 4096
    idx = paris.build(Xd, leaf_mode=1, n_leaves=n_leaves)
    idx.attach_batch(max_batch=args.batch)
    Qt, _, _ = synth.training_queries(X, args.train_queries, seed=0)
    Qtd = torch.from_numpy(Qt).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F, y, _ = paris.learned.exact_labels(idx, Qtd)
    torch.cuda.synchronize()
    label_s = time.perf_counter() - t0
    log(f"labelled {args.train_queries} training queries in {label_s:.1f}s")
    net = paris.SeedModel(n_leaves, max_rows=1024, params=paris.init_params(n_leaves, seed=0))
    t1 = time.perf_counter()
    hist = paris.train_seed_model(net, F, y, epochs=args.epochs, batch=1024, lr=2e-3, seed=0)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    steps = args.epochs * ((args.train_queries + 1023) // 1024)
    log(f"trained {args.epochs} epochs ({steps} steps) in {train_s:.1f}s, loss {hist[0]:.3f} -> {hist[-1]:.3f}")
    del Qtd, F, y

    Qe, _, _ = synth.noisy_queries(X, args.eval_queries, seed=2, sigma=0.5)
    Qed = torch.from_numpy(Qe).cuda()
    rows = [Qed[m] for m in range(Qe.shape[0])]

    def per_query(enabled):
        idx.set_seed_model(net, enabled)
        for m in range(min(50, len(rows))):
            idx.query(rows[m])
        torch.cuda.synchronize()
        ta = time.perf_counter()
        ans = [idx.query(r)[0] for r in rows]
        torch.cuda.synchronize()
        dt = time.perf_counter() - ta
        st = [idx.query(r, with_stats=True)[2] for r in rows[:300]]
        nn = np.array([idx.query(r)[1] for r in rows[:300]])
        seed = np.array([x["seed_dist"] for x in st])
        return ans, {"queries_per_s": len(rows) / dt,
                     "mean_lb_survivors": float(np.mean([x["lb_survivors"] for x in st])),
                     "mean_refined": float(np.mean([x["refined"] for x in st])),
                     "mean_seed_over_nn_distance": float(np.mean(seed / np.maximum(nn, 1e-30)))}

    a0, plain = per_query(False)
    a1, learned = per_query(True)
    log(f"hard queries: plain {plain['queries_per_s']:.0f} q/s, learned {learned['queries_per_s']:.0f} q/s")
    per_query_check = None
    if not args.no_cpu_baseline:
        from oracle import native
        native.build(force=False)
        k = min(32, len(rows))
        ri, _, _ = native.nn_many_blocked(Qe[:k], X, threads=args.cpu_threads)
        per_query_check = {"queries": k, "learned_answers_equal_oracle": bool(np.array_equal(ri, np.array(a1[:k]))),
                        "plain_answers_equal_oracle": bool(np.array_equal(ri, np.array(a0[:k])))}

    B = args.batch
    Qb, _, sigb = synth.noisy_queries(X, B, seed=1, sigma=(0.01, 0.5))
    Qbd = torch.from_numpy(Qb).cuda()
    I = torch.empty(B, dtype=torch.int64, device="cuda")
    D = torch.empty(B, dtype=torch.float64, device="cuda")
    res = {}
    for enabled in (False, True):
        idx.set_seed_model(net, enabled)
        idx.query_batch(Qbd, out=(I, D))
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for _ in range(args.batch_steps):
            idx.query_batch(Qbd, out=(I, D))
        torch.cuda.synchronize()
        el = time.perf_counter() - tb
        _, _, st = idx.query_batch(Qbd, out=(I, D), with_stats=True)
        res[enabled] = {"queries_per_s": B * args.batch_steps / el, "ms_per_batch": el / args.batch_steps * 1e3,
                        "screen_survivors_per_query": st["lb_survivors"] / B, "fallback_queries": st["resolved"],
                        "answers": I.cpu().numpy(), "dists": D.cpu().numpy()}
    same_batch = bool(np.array_equal(res[False].pop("answers"), res[True]["answers"]))
    res[False].pop("dists")
    learned_check = oracle_check(X, Qb, res[True].pop("answers"), res[True].pop("dists"), sigb, args, seed=5)
    idx.set_seed_model(None, False)
    net.close()
    idx.close()
    return {
        "workload": f"{N} x {n} random walks, {n_leaves} equal-count leaves; network 16-256-256-{n_leaves} "
                    f"(bfloat16 MFMA, float32 accumulate) trained {args.epochs} epochs on {args.train_queries} "
                    "exact labels (sigma ~ U[0.05, 0.5]); evaluation: hard queries (sigma 0.5) one at a time, "
                    f"and batches of {B} (sigma ~ U[0.01, 0.5])",
        "label_s": label_s, "train_s": train_s, "train_steps": steps, "loss_first_epoch": hist[0],
        "loss_last_epoch": hist[-1],
        "hard_queries": {"count": len(rows), "plain_seed": plain, "learned_seed": learned,
                         "answers_identical": bool(np.array_equal(np.array(a0), np.array(a1))),
                         "oracle_sample": per_query_check},
        "batched": {"plain_seed": res[False], "learned_seed": res[True], "answers_identical": same_batch,
                    "oracle_check": learned_check,
                    "learned_vs_plain_per_query_path": (res[True]["queries_per_s"] / args._plain_qps
                                                        if args._plain_qps else None)},
    }


def multi_section(args):
    """Mixed-length workload: three collections resident together (100M x 128, 20M x 512 and
    5M x 1024 random walks, ~113 GB of float32), batches of 2048 queries whose collection is drawn
    uniformly (noise sigma ~ U[0.05, 0.5]), answered by paris_query_batch_multi with a screen
    shape tuned per length; plus the per-query path's lower-bound scan over the 100M collection's
    1.6 GB iSAX array (too large for any cache) and the CPU oracle on a sample."""
    import numpy as np
    import torch

    import paper_2009_00166_amd as paris
    import synth
    B = 2048
    specs = [(int(100_000_000 * args.multi_scale), 128, 0), (int(20_000_000 * args.multi_scale), 512, 1),
             (int(5_000_000 * args.multi_scale), 1024, 2)]
    Xs, idxs = [], []
    for N, n, seed in specs:
        t0 = time.perf_counter()
        X = synth.random_walks(N, n, seed=seed, threads=16)
        Xd = torch.from_numpy(X).cuda()
        torch.cuda.synchronize()
        ix = paris.build(Xd)
        ix.attach_batch(max_batch=B)
        torch.cuda.synchronize()
        log(f"collection {N} x {n}: generated, copied, built and attached in {time.perf_counter() - t0:.1f}s")
        Xs.append((X, Xd))
        idxs.append(ix)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(7)))
    which = rng.integers(0, 3, size=B)
    counts = [int((which == c).sum()) for c in range(3)]
    Qs, srcs, sigs = [], [], []
    for c, (X, _) in enumerate(Xs):
        Q, src, sig = synth.noisy_queries(X, counts[c], seed=10 + c, sigma=(0.05, 0.5))
        Qs.append(torch.from_numpy(Q).cuda())
        srcs.append(src)
        sigs.append(sig)
    paris.query_batch_multi(idxs, Qs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.batch_steps):
        outs = paris.query_batch_multi(idxs, Qs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    _, st = paris.query_batch_multi(idxs, Qs, with_stats=True)
    log(f"mixed batches: {B * args.batch_steps / el:.0f} queries/s")
    per_coll = []
    for c, ix in enumerate(idxs):
        ix.set_timing(True)
        ix.query_batch(Qs[c])
        ms, k = ix.batch_timing()
        ix.set_timing(False)
        lay = ix.layout()
        per_coll.append({"n_series": specs[c][0], "length": specs[c][1], "queries_in_batch": counts[c],
                         "stages_ms": dict(zip(["seeds", "block_bound", "screen", "rescore", "resolve"],
                                               [m / max(k, 1) for m in ms])),
                         "scan_shape": [lay.scan_threads, lay.scan_blocks_per_cu, lay.scan_unroll]})
    # per-query path over the 100M collection: its scan reads the 1.6 GB iSAX array from HBM
    ix0 = idxs[0]
    rows = [Qs[0][m] for m in range(min(200, Qs[0].shape[0]))]
    for r in rows[:10]:
        ix0.query(r)
    ix0.set_timing(True, scan_only=True)
    for r in rows:
        ix0.query(r)
    scan_ms, timed = ix0.timing()
    ix0.set_timing(False)
    st0 = [ix0.query(r, with_stats=True)[2] for r in rows]
    lb_ms = scan_ms[1] / max(timed, 1)
    lb_bytes = (ENV_BYTES_PER_SERIES * specs[0][0] + SAX_BYTES_PER_SERIES * np.mean([x["words_read"] for x in st0])
                + SURVIVOR_BYTES * np.mean([x["lb_survivors"] for x in st0]))
    gbps = lb_bytes / (lb_ms * 1e-3) / 1e9
    rec = {
        "metric": "exact 1-NN queries/s, mixed batches over 100M x 128 + 20M x 512 + 5M x 1024 fp32",
        "value": B * args.batch_steps / el, "unit": "queries/s", "n_gpus": 1, "steps": args.batch_steps,
        "warmup": 1, "ms_per_step": el / args.batch_steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 screen, f32 re-score, f64 resolve", "data": "synthetic",
        "config": {"workload": f"three resident collections {specs[0][0]} x 128, {specs[1][0]} x 512, "
                               f"{specs[2][0]} x 1024 z-normalised random walks; batches of {B} queries, collection "
                               "drawn uniformly, dataset series + N(0, sigma) noise, sigma ~ U[0.05, 0.5]; "
                               "paris_query_batch_multi (per-length tuned screens; series longer than 256 screened "
                               "on segment means)", "batch": B, "collections": per_coll},
        "roofline": {"bound": "hbm", "kernel": "k_lbscan (per-query path, 100M x 128)", "achieved": gbps,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS, "traffic": None,
                     "bytes_per_launch": lb_bytes, "avg_launch_ms": lb_ms,
                     "single_pass_equivalent_GBps": SAX_BYTES_PER_SERIES * specs[0][0] / (lb_ms * 1e-3) / 1e9,
                     "single_pass_equivalent_frac": SAX_BYTES_PER_SERIES * specs[0][0] / (lb_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                     "note": "bytes = 1 B per series (run envelopes) + 16 B per series of the runs that pass + "
                             "12 B per survivor, means over the 200 timed queries"},
        "screen_survivors_per_query": st["lb_survivors"] / B, "fallback_queries": st["resolved"],
    }
    if not args.no_cpu_baseline:
        from oracle import native
        native.build(force=False)
        X0 = Xs[0][0]
        sample = Qs[0][:4].cpu().numpy()
        t2 = time.perf_counter()
        ri, _, used = native.nn_many(sample, X0, threads=args.cpu_threads)
        dt = time.perf_counter() - t2
        rec["cpu_baseline"] = {"value": len(sample) / dt, "unit": "queries/s", "cores": int(used), "kind": "oracle",
                               "sample": f"4 queries of the 100M x 128 collection, brute-force float64 C oracle",
                               "answers_agree_with_gpu": bool(np.array_equal(ri, outs[0][0][:4].cpu().numpy()))}
        rec["oracle_check"] = [oracle_check(Xs[c][0], Qs[c].cpu().numpy(), outs[c][0].cpu().numpy(),
                                            outs[c][1].cpu().numpy(), sigs[c], args, seed=20 + c)
                               for c in range(3)]
    for ix in idxs:
        ix.close()
    return rec


if __name__ == "__main__":
    sys.exit(main())
