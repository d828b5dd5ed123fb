#!/usr/bin/env python
"""Benchmark of the Extended RaBitQ hot path on one MI355X.

Workload (embed768): N = 1,000,000 x D = 768 FP32 rows of a 1024-component
Gaussian mixture with Zipf weights, sigma 0.3, every row rescaled to a
LogNormal(0, 0.2) norm; 10,000 queries from the same mixture; IVF with 4096
k-means lists; B = 4 codes (B = 8 reported beside it); k = 10.

A step is one search of the whole query batch through the C ABI
(erq_search: rotation, coarse probe, pair build, int8 matrix-core scan with
estimator and top-k, exact re-rank), with the index and the queries
resident in HBM.  The operating point (nprobe, re-rank depth) is the fastest
one whose recall@10 against exact FP32 brute force is >= 0.95.  Encode
throughput is the time of erq_index_build (residuals, rotation, Algorithm 1,
factors, packing) over the 1M rows.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
INT8_PEAK_TOPS = 5000.0        # dense int8 matrix cores


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def recall_at(ids, truth, k=10):
    ids = ids[:, :k]
    hit = 0
    for a, b in zip(ids, truth[:, :k]):
        hit += len(set(a.tolist()) & set(b.tolist()))
    return hit / (k * len(ids))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--nq", type=int, default=10_000)
    ap.add_argument("--nlist", type=int, default=4096)
    ap.add_argument("--bits", type=int, default=4)
    ap.add_argument("--bits2", type=int, default=8, help="second code width reported as context (0 = skip)")
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--kmeans-iters", type=int, default=10)
    ap.add_argument("--target-recall", type=float, default=0.95)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-queries", type=int, default=1000,
                    help="queries of the oracle's all-core run (the first ones)")
    ap.add_argument("--cpu-single-queries", type=int, default=40,
                    help="queries of the oracle's single-thread run")
    ap.add_argument("--est-queries", type=int, default=400,
                    help="queries of the float- vs int8-query recall table (0 = skip)")
    ap.add_argument("--flat", type=int, default=1, help="1: FP32 IVF-Flat comparator sweep on the same lists")
    ap.add_argument("--serve-n", type=int, default=5_000_000, help="rows of the serving workload")
    ap.add_argument("--serve-kmeans-iters", type=int, default=6, help="k-means rounds of the serving workload")
    ap.add_argument("--nprobe", type=int, default=0, help="fixed operating point (skips the sweep)")
    ap.add_argument("--rerank", type=int, default=-1, help="fixed re-rank depth (with --nprobe)")
    ap.add_argument("--tune", type=int, default=1, help="1: run the scan-schedule autotuner before timing")
    ap.add_argument("--schedule", type=str, default="",
                    help="nqt,pd,round1[,round2]: fixed scan schedule (with --tune 0), e.g. the tuner's choice")
    ap.add_argument("--graph", type=int, default=1,
                    help="1: the timed steps replay the search captured in a HIP graph; 0: eager calls")
    ap.add_argument("--serve", type=int, default=2000,
                    help="N > 0: also run N Poisson-arrival requests per rate through the batching server "
                         "(p50/p99); 0 skips it")
    ap.add_argument("--workload", type=str, default="embed768",
                    choices=("embed768", "batching", "serving", "two_stage", "precision"),
                    help="embed768 (the default line); batching: 2M x 960, 8192 uneven lists, B=3/5/7, batches "
                         "1..4096 with mixed nprobe; serving: 5M x 3072, 16384 lists, B=4, Poisson arrivals; "
                         "two_stage: embed768 with the MSB-first two-stage scan against the one-stage scan; "
                         "precision: 1M x 1536 unit vectors, FP32 vs BF16 rotation, B=2..8, errors against FP64")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (scale for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU and has no multi-GPU path; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        calib_copy()
        return
    if args.workload == "batching":
        run_batching(args)
        return
    if args.workload == "serving":
        run_serving(args)
        return
    if args.workload == "two_stage":
        run_two_stage(args)
        return
    if args.workload == "precision":
        run_precision(args)
        return

    import torch
    from paper_2409_09913_amd import erq, serve, synth

    dev = torch.device("cuda:0")
    erq.load()
    t0 = time.time()
    log("generating data", args.n, "x 768 and", args.nq, "queries")
    x_np, q_np = synth.embed768(args.n, args.nq)
    dp = x_np.shape[1]
    P_np = synth.haar_orthogonal(dp).astype(np.float32)
    x = torch.from_numpy(x_np).to(dev)
    q = torch.from_numpy(q_np).to(dev)
    P = torch.from_numpy(P_np).to(dev)
    log("data ready %.1fs" % (time.time() - t0))

    log("k-means", args.nlist, "lists,", args.kmeans_iters, "iterations")
    cent, assign = erq.kmeans(x, args.nlist, iters=args.kmeans_iters)
    torch.cuda.synchronize()
    sizes = torch.bincount(assign.long(), minlength=args.nlist).cpu().numpy()
    log("k-means done %.1fs; list sizes min %d mean %.1f max %d" % (time.time() - t0, sizes.min(), sizes.mean(),
                                                                    sizes.max()))

    # ---- warm the kernels on a small build, then time the encode ---------------------
    def build_index(B, keep_raw):
        ix = erq.Index(dp, B, args.nlist, P)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        ix.build(x, cent, assign, precision=0, keep_raw=False)
        torch.cuda.synchronize()
        te = time.perf_counter()
        if keep_raw:
            ix.set_raw(x)
        return ix, te - ts

    warm = erq.Index(dp, args.bits, args.nlist, P)
    warm.build(x[:20000].contiguous(), cent, assign[:20000].contiguous())
    if args.bits2:
        warm2 = erq.Index(dp, args.bits2, args.nlist, P)
        warm2.build(x[:4000].contiguous(), cent, assign[:4000].contiguous())
        warm2.close()
    warm.close()
    ix, t_enc = build_index(args.bits, keep_raw=True)
    enc_rate = args.n / t_enc
    log("encode B=%d: %.3fs -> %.3g codes/s" % (args.bits, t_enc, enc_rate))
    enc_rate2 = None
    if args.bits2:
        ix2, t_enc2 = build_index(args.bits2, keep_raw=True)
        enc_rate2 = args.n / t_enc2
        log("encode B=%d: %.3fs -> %.3g codes/s" % (args.bits2, t_enc2, enc_rate2))

    # ---- exact FP32 brute force (library GEMM) : ground truth and comparator -----------
    def brute(qb, k):
        xn = (x * x).sum(1)
        out = torch.empty((qb.shape[0], k), dtype=torch.int64, device=dev)
        for i in range(0, qb.shape[0], 1000):
            d = xn[None, :] - 2.0 * (qb[i:i + 1000] @ x.T)
            out[i:i + 1000] = torch.topk(d, k, dim=1, largest=False).indices
        return out

    truth = brute(q, args.k)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    truth = brute(q, args.k)
    torch.cuda.synchronize()
    flat_qps = args.nq / (time.perf_counter() - tb)
    truth_np = truth.cpu().numpy()
    log("FP32 brute force: %.0f QPS" % flat_qps)

    # ---- sweep the operating point ---------------------------------------------------
    def timed_search(index, nprobe, rr, reps):
        ws = torch.empty(index.search_workspace_size(args.nq, nprobe, args.k, rr), dtype=torch.uint8, device=dev)
        out = (torch.empty((args.nq, args.k), dtype=torch.int64, device=dev),
               torch.empty((args.nq, args.k), dtype=torch.float32, device=dev))
        index.search(q, nprobe, args.k, rr, ws=ws, out=out)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(reps):
            index.search(q, nprobe, args.k, rr, ws=ws, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - ts) / reps
        return out[0].cpu().numpy(), args.nq / dt

    def sweep(index, label):
        rows = []
        grid = [(args.nprobe, max(args.rerank, 0))] if args.nprobe > 0 else \
            [(n_, r_) for n_ in (16, 32, 64, 72, 80, 84, 88, 92, 96, 104, 112, 128, 160, 256)
             for r_ in (0, 16, 18, 20, 22, 24, 32, 50, 100)]
        for nprobe, rr in grid:
            if True:
                ids, qps = timed_search(index, nprobe, rr, 3)
                rec = recall_at(ids, truth_np, args.k)
                rows.append((nprobe, rr, rec, qps))
                log("%s nprobe %3d rerank %2d recall@10 %.4f QPS %.0f" % (label, nprobe, rr, rec, qps))
        ok = [r for r in rows if r[2] >= args.target_recall]
        if not ok:
            return max(rows, key=lambda r: r[2]), rows
        # the few fastest points that reach the recall target, timed again over more calls
        top = sorted(ok, key=lambda r: -r[3])[:4]
        if len(top) > 1:
            again = []
            for nprobe, rr, rec, _ in top:
                _, qps = timed_search(index, nprobe, rr, 12)
                again.append((nprobe, rr, rec, qps))
                log("%s refine nprobe %3d rerank %2d QPS %.0f" % (label, nprobe, rr, qps))
            top = again
        return max(top, key=lambda r: r[3]), rows

    best, rows = sweep(ix, "B=%d" % args.bits)
    nprobe, rr, rec, _ = best
    best2 = None
    best2_lo = None
    if args.bits2:
        best2, _ = sweep(ix2, "B=%d" % args.bits2)
        if args.bits2 >= 5:                     # the same sweep with the int8 query in two planes
            ix2.set_query_planes(2)
            best2_lo, _ = sweep(ix2, "B=%d two query planes" % args.bits2)
            ix2.set_query_planes(1)

    # ---- scan schedule: the library's autotuner at the operating point ------------------
    tuned = None
    if args.schedule:
        ix.set_tune(*(int(v) for v in args.schedule.split(",")))
        tuned = dict(ix.get_tune(), ms=None, fixed=True)
        log("fixed scan schedule", tuned)
    if args.tune and not args.schedule:
        tuned = ix.tune(q, nprobe, args.k, rr, reps=2)
        log("autotune: nqt %d, ring depth %d, round-1 ranks %d, middle round to %d (%.3f ms per search)" %
            (tuned["nqt"], tuned["pd"], tuned["round1"], tuned["round2"], tuned["ms"]))

    # ---- timed region -----------------------------------------------------------------
    ws = torch.empty(ix.search_workspace_size(args.nq, nprobe, args.k, rr), dtype=torch.uint8, device=dev)
    out = (torch.empty((args.nq, args.k), dtype=torch.int64, device=dev),
           torch.empty((args.nq, args.k), dtype=torch.float32, device=dev))
    for _ in range(args.warmup):
        ix.search(q, nprobe, args.k, rr, ws=ws, out=out)
    torch.cuda.synchronize()
    graph_dt, graph_rec = None, None
    if args.graph:
        # the whole search (rotation, probe, scan rounds, selects, re-rank) as one
        # graph; queries already sit in its static input when the clock starts
        g = serve.SearchGraph(ix, args.nq, nprobe, args.k, rr)
        with torch.cuda.stream(g.stream):
            g.q.copy_(q)
            for _ in range(args.warmup):
                g.graph.replay()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        with torch.cuda.stream(g.stream):
            for _ in range(args.steps):
                g.graph.replay()
        torch.cuda.synchronize()
        graph_dt = time.perf_counter() - ts
        graph_rec = recall_at(g.ids.cpu().numpy(), truth_np, args.k)
        log("graph replay: %.3f ms/step, recall %.4f" % (1000 * graph_dt / args.steps, graph_rec))
    # eager steps with the library's HIP events around every kernel (per-launch durations)
    erq.profile_enable(True)
    erq.profile_read("scan", reset=True)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        ix.search(q, nprobe, args.k, rr, ws=ws, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - ts
    scan_ms, scan_n = erq.profile_read("scan")
    tot, raw = {}, {}
    for kname in ("rotate", "probe", "scan", "scan_a", "scan_b", "scan_c", "rerank"):
        ms, nl = erq.profile_read(kname)
        tot[kname] = ms / max(nl, 1)
        raw[kname] = (ms, nl)
    erq.profile_read("scan", reset=True)
    erq.profile_enable(2)                       # one extra search: count the pairs re-scanned in pass C
    erq.profile_read("scan_redo_pairs", reset=True)
    ix.search(q, nprobe, args.k, rr, ws=ws, out=out)
    torch.cuda.synchronize()
    redo, _ = erq.profile_read("scan_redo_pairs", reset=True)
    tot["redo_pairs"] = redo
    erq.profile_read("scan", reset=True)
    erq.profile_enable(False)
    eager_ms = 1000 * dt / args.steps
    rec_final = recall_at(out[0].cpu().numpy(), truth_np, args.k)
    if graph_dt is not None:
        if graph_rec != rec_final:
            log("WARNING: graph replay recall %.4f differs from the eager call's %.4f" % (graph_rec, rec_final))
        dt = graph_dt
    qps = args.steps * args.nq / dt
    ms_per_step = 1000 * dt / args.steps
    log("timed: %.0f QPS, %.3f ms/step (eager %.3f), recall %.4f; per-launch ms %s" % (qps, ms_per_step, eager_ms,
                                                                                   rec_final, tot))

    # ---- roofline of the scan kernel ------------------------------------------------------
    probes = erq.coarse_probe(q, cent, nprobe).cpu().numpy()
    lists, pair_cnt = np.unique(probes, return_counts=True)
    nb = args.bits * dp // 8 + 8
    bytes_alg = float(sizes[lists].sum()) * nb
    # pass-B work: every probed (query, member) pair but those the first bound
    # estimates (the first 256 members of each query's 4 nearest lists)
    ops_alg = float((sizes[lists] * pair_cnt).sum() - dense_covered(probes, sizes)) * 2 * dp
    # dominant kernel: the pass-B scan (scanB_kernel), launched once per round of
    # probe ranks; over one search its launches cover every (query, list) pair once
    sb_ms, sb_n = raw["scan_b"]
    per_search = sb_n / max(args.steps, 1)
    avg_s = sb_ms / max(sb_n, 1) / 1000.0
    bytes_alg /= per_search                     # algorithmic bytes and ops per launch
    ops_alg /= per_search
    hbm_t = bytes_alg / (HBM_PEAK_GBS * 1e9)
    mma_t = ops_alg / (INT8_PEAK_TOPS * 1e12)
    src = open(os.path.join(ROOT, "paper_2409_09913_amd", "csrc", "scan.hip"), "rb").read()
    sha = hashlib.sha256(src).hexdigest()[:16]
    # HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE counters
    # (profiles/scan_traffic.json, one entry per operating point), used only
    # when the entry was taken on this scan source at this nprobe and B
    traffic = None
    tf = os.path.join(ROOT, "profiles", "scan_traffic.json")
    if os.path.exists(tf):
        try:
            for t in json.load(open(tf)).get("entries", []):
                if t.get("scan_hip_sha256_16") == sha and t.get("nprobe") == nprobe and t.get("bits") == args.bits:
                    traffic = t.get("hbm_bytes_per_launch")
        except Exception:
            traffic = None
    if hbm_t >= mma_t:
        roof = {"bound": "hbm", "achieved": bytes_alg / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "mfma", "achieved": ops_alg / avg_s / 1e12, "peak": INT8_PEAK_TOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic
    roof.update({"kernel": "scanB_kernel (int8 MFMA scan + estimator + bound test)", "avg_launch_ms": avg_s * 1e3,
                 "launches_per_search": per_search, "scan_ms_per_search": scan_ms / max(scan_n, 1),
                 "alg_bytes_per_launch": bytes_alg, "alg_int8_ops_per_launch": ops_alg,
                 "mfma_frac": ops_alg / avg_s / 1e12 / INT8_PEAK_TOPS,
                 "hbm_frac": bytes_alg / avg_s / 1e9 / HBM_PEAK_GBS, "scan_hip_sha256_16": sha})
    log("roofline", roof)

    # ---- serving: Poisson arrivals through the continuous-batching server ----------------
    serving = None
    if args.serve:
        srv = serve.Server(ix, max_batch=1024, max_nprobe=max(nprobe, 64), max_k=args.k, max_rerank=max(rr, 20),
                           slots=4)
        # untimed pass first: the slots' streams and output blocks are set up on first use
        serve.poisson_run(srv, q, rate=10000.0, n_requests=200, per_request=1, k=args.k, nprobes=(16, 64),
                          rerank_k=rr, seed=1)
        res_s = {}
        for rate in (1000.0, 10000.0, 50000.0):
            reqs, p50, p99, sq = serve.poisson_run(srv, q, rate=rate, n_requests=args.serve, per_request=1,
                                                   k=args.k, nprobes=(16, 64), rerank_k=rr, seed=7)
            res_s["%d_rps" % rate] = {"p50_ms": p50, "p99_ms": p99, "qps": sq}
            log("serving at %d req/s: p50 %.3f ms p99 %.3f ms, %.0f QPS" % (rate, p50, p99, sq))
        serving = {"slots": srv.slots_admitted, "request": "1 query, nprobe 16 or 64, k=%d, rerank %d" % (args.k, rr),
                   "by_rate": res_s}

    # ---- FP32 IVF-Flat on the same lists and probes: the metric's FP32 scan ---------------
    flat = None
    if args.flat:
        rows_f = []
        for npf in (16, 32, 64, 88, 128, 192):
            run = ivf_flat_fp32(x, q, cent, assign.cpu().numpy(), npf, args.k)
            ids_f = run()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            ids_f = run()
            torch.cuda.synchronize()
            dtf = time.perf_counter() - ts
            rec_f = recall_at(ids_f.cpu().numpy(), truth_np, args.k)
            rows_f.append({"nprobe": npf, "recall@10": rec_f, "qps": args.nq / dtf})
            log("IVF-Flat FP32 nprobe %3d recall@10 %.4f QPS %.0f" % (npf, rec_f, args.nq / dtf))
            del run
        ok_f = [r for r in rows_f if r["recall@10"] >= args.target_recall]
        flat = {"kind": "FP32 IVF-Flat, same lists and probe lists, exact distances by torch.bmm (library GEMM)",
                "best": max(ok_f, key=lambda r: r["qps"]) if ok_f else None, "sweep": rows_f}

    # ---- accuracy of the int8 query (reading C-13): float- vs int8-query recall ------------
    est_tab = []
    if args.est_queries:
        for index, B, npr in ((ix, args.bits, nprobe),) + (((ix2, args.bits2, best2[0]),) if args.bits2 else ()):
            r = estimator_recall(index, cent, q_np, P_np, truth_np, npr, args.k, B, args.est_queries)
            est_tab.append(r)
            log("estimator recall B=%d nprobe %d (%d queries, no re-rank): int8 query %.4f, float query %.4f%s" %
                (B, npr, r["queries"], r["recall_int8_query"], r["recall_float_query"],
                 ", int8 two planes %.4f" % r["recall_int8_two_planes"] if "recall_int8_two_planes" in r else ""))

    # ---- CPU baseline: the oracle on a bounded sample ------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, x_np, q_np, P_np, cent.cpu().numpy(), assign.cpu().numpy(), nprobe, rr)

    res = {
        "metric": "QPS at recall@10>=0.95 (int8-MFMA scan vs FP32 scan), encode codes/s",
        "value": qps, "unit": "QPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8", "data": "synthetic",
        "config": {"workload": "embed768: N=%d x D=768 GMM(1024 comps, Zipf, sigma 0.3, LogNormal(0,0.2) norms), "
                               "IVF %d k-means lists, B=%d, %d queries, k=%d" % (args.n, args.nlist, args.bits,
                                                                                args.nq, args.k),
                   "global_batch": args.nq, "nprobe": nprobe, "rerank_k": rr, "recall@10": rec_final,
                   "parallelism": "single GPU"},
        "encode_codes_per_s": enc_rate,
        "fp32_bruteforce_qps": flat_qps,
        "fp32_ivf_flat": flat,
        "estimator_recall": est_tab,
        "per_launch_ms": tot,
        "timed_mode": "hip_graph_replay" if graph_dt is not None else "eager",
        "autotune": tuned,
        "eager_ms_per_step": eager_ms,
        "serving": serving,
        "roofline": roof,
        "cpu_baseline": cpu,
        "sweep": [{"nprobe": a, "rerank_k": b, "recall@10": c, "qps": d} for a, b, c, d in rows],
    }
    if args.bits2:
        res["bits2"] = {"bits": args.bits2, "encode_codes_per_s": enc_rate2,
                        "best": {"nprobe": best2[0], "rerank_k": best2[1], "recall@10": best2[2], "qps": best2[3]}}
        if best2_lo is not None:
            res["bits2"]["best_two_query_planes"] = {"nprobe": best2_lo[0], "rerank_k": best2_lo[1],
                                                     "recall@10": best2_lo[2], "qps": best2_lo[3]}
    log("total %.1fs" % (time.time() - t0))
    print(json.dumps(res), flush=True)


def brute_topk(x, qb, k, chunk=256):
    """Exact FP32 k-NN (library GEMM + top-k), the ground truth of a workload."""
    import torch
    xn = (x * x).sum(1)
    out = torch.empty((qb.shape[0], k), dtype=torch.int64, device=qb.device)
    for i in range(0, qb.shape[0], chunk):
        d = xn[None, :] - 2.0 * (qb[i:i + chunk] @ x.T)
        out[i:i + chunk] = torch.topk(d, k, dim=1, largest=False).indices
    return out


def dense_covered(probes_np, sizes, ranks=4, members=256):
    """(query, member) pairs the scan's first bound estimates and pass B then
    skips: the first `members` members of each query's `ranks` nearest lists."""
    p = probes_np[:, :ranks]
    return float(np.minimum(sizes[p[p >= 0]], members).sum())


def scan_roofline(ix, nq, dp, B, sizes, probes_np, launches_ms):
    """Algorithmic int8 ops and code bytes of one search over the probed pairs,
    against the pass-B launch time."""
    lists, cnt = np.unique(probes_np[probes_np >= 0], return_counts=True)
    ops = float((sizes[lists] * cnt).sum() - dense_covered(probes_np, sizes)) * 2 * dp
    byt = float(sizes[lists].sum()) * (B * dp / 8 + 8)
    ms, nl = launches_ms
    t = ms / 1000.0
    return {"int8_tops": ops / t / 1e12, "mfma_frac": ops / t / 1e12 / INT8_PEAK_TOPS,
            "code_gbs": byt / t / 1e9, "hbm_frac": byt / t / 1e9 / HBM_PEAK_GBS, "scan_b_ms_per_search": ms,
            "launches": nl}


def run_batching(args):
    """Batching workload: N = 2,000,000 x D = 960 clusters of an anisotropic
    Gaussian (variance i^-0.5), 8192 lists of 20..5000 members (power law,
    mean about 244), B = 3, 5, 7; 4096 queries with per-query nprobe uniform in
    {8, ..., 256}; each batch size of 1..4096 captured as one HIP graph with
    per-query parameters, scan schedule autotuned at the full batch."""
    import torch
    from paper_2409_09913_amd import erq, serve, synth
    dev = torch.device("cuda:0")
    erq.load()
    t0 = time.time()
    nl, dp, nq, k = 8192, 960, 4096, args.k
    sizes = synth.power_law_sizes(nl, 20, 5000, 0.76)
    x, lab, cent = synth.clustered_anisotropic_device(sizes, dp, device=dev)
    n = x.shape[0]
    g = np.random.default_rng(7)
    qsz = np.zeros(nl, np.int64)
    qlab = g.integers(0, nl, nq)
    sd = torch.from_numpy((np.arange(1, dp + 1, dtype=np.float64) ** -0.25).astype(np.float32)).to(dev)
    gq = torch.Generator(device=dev).manual_seed(11)
    q = (cent[torch.from_numpy(qlab).to(dev)] + 0.5 * torch.randn((nq, dp), device=dev, generator=gq) * sd).contiguous()
    own = g.choice([8, 16, 32, 64, 128, 256], nq).astype(np.int32)
    npq = torch.from_numpy(own).to(dev)
    truth = brute_topk(x, q, k).cpu().numpy()
    log("batching workload: %d x %d, %d lists (%d..%d), data %.1fs" % (n, dp, nl, sizes.min(), sizes.max(),
                                                                      time.time() - t0))
    out = {"metric": "QPS per batch size, per-query nprobe 8..256 (batching workload)", "unit": "QPS",
           "config": {"workload": "batching: N=%d x D=960 anisotropic clusters, 8192 lists 20..5000, %d queries, "
                                  "nprobe uniform in {8..256} per query, k=%d" % (n, nq, k)}, "by_bits": []}
    for B in (3, 5, 7):
        ix = erq.Index(dp, B, nl, None, seed=240909913)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        ix.build(x, cent, lab, keep_raw=False)
        torch.cuda.synchronize()
        enc = n / (time.perf_counter() - ts)
        ix.set_raw(x)
        small_default = ix.small_batch()
        tuned = ix.tune(q, 128, k, 2 * k, reps=2)
        rows = []
        for rr in (0, 2 * k):
            ids, _ = ix.search(q, 256, k, rr, nprobe_q=npq)
            rec = recall_at(ids.cpu().numpy(), truth, k)
            for bs in (1, 4, 16, 32, 64, 256, 1024, 4096):
                row = {"rerank_k": rr, "batch": bs, "recall@10_full_batch": rec}
                # the index's default path, then (up to the small path's limit of 1024
                # queries) the small-batch path and the pair-grouped pipeline forced
                paths = (("", None), ("_small", 1024), ("_pipeline", 0)) if bs <= 1024 else (("", None),)
                for label, sq in paths:
                    ix.set_small_batch(small_default if sq is None else sq)
                    gph = serve.SearchGraph(ix, bs, 256, k, rr, per_query=True)
                    gph.q.copy_(q[:bs])
                    gph.params[0].copy_(npq[:bs])
                    with torch.cuda.stream(gph.stream):
                        gph.graph.replay()
                    torch.cuda.synchronize()
                    reps = max(3, min(200, 8192 // bs))
                    ts = time.perf_counter()
                    with torch.cuda.stream(gph.stream):
                        for _ in range(reps):
                            gph.graph.replay()
                    torch.cuda.synchronize()
                    dt = (time.perf_counter() - ts) / reps
                    row["qps" + label] = bs / dt
                    row["ms_per_batch" + label] = dt * 1e3
                    del gph
                ix.set_small_batch(small_default)
                rows.append(row)
            log("batching B=%d rerank %d recall@10 %.4f; QPS by batch %s; pipeline path at small batches %s" %
                (B, rr, rec, {r["batch"]: round(r["qps"]) for r in rows if r["rerank_k"] == rr},
                 {r["batch"]: round(r["qps_pipeline"]) for r in rows if r["rerank_k"] == rr and "qps_pipeline" in r}))
        # pass-B launch time of the full batch for the roofline
        erq.profile_enable(True)
        erq.profile_read("scan_b", reset=True)
        ix.search(q, 256, k, 0, nprobe_q=npq)
        torch.cuda.synchronize()
        sb = erq.profile_read("scan_b", reset=True)
        erq.profile_read("scan", reset=True)
        erq.profile_enable(False)
        probes = erq.coarse_probe(q, cent, 256).cpu().numpy()
        probes[np.arange(256)[None, :] >= own[:, None]] = -1
        roof = scan_roofline(ix, nq, dp, B, sizes, probes, sb)
        out["by_bits"].append({"bits": B, "encode_codes_per_s": enc, "autotune": tuned, "rows": rows,
                               "scan_full_batch": roof})
        log("batching B=%d encode %.3g codes/s, scan %s" % (B, enc, roof))
        ix.close()
        torch.cuda.empty_cache()
    log("total %.1fs" % (time.time() - t0))
    print(json.dumps(out), flush=True)


def run_two_stage(args):
    """MSB-first two-stage scan (Sec. 4.2) against the one-stage scan on the
    embed768 workload (N = 1,000,000 x 768, 4096 k-means lists), B = 4 and 8:
    QPS at recall@10 >= the target for eps0 in {0 (one-stage), 1.9, 3} at the
    full 10,000-query batch, and QPS by batch size (1, 16, 256, 4096) at the
    one-stage operating point, each batch size captured as a HIP graph."""
    import torch
    from paper_2409_09913_amd import erq, serve, synth
    dev = torch.device("cuda:0")
    erq.load()
    t0 = time.time()
    x_np, q_np = synth.embed768(args.n, args.nq)
    dp = x_np.shape[1]
    x = torch.from_numpy(x_np).to(dev)
    q = torch.from_numpy(q_np).to(dev)
    P = torch.from_numpy(synth.haar_orthogonal(dp).astype(np.float32)).to(dev)
    cent, assign = erq.kmeans(x, args.nlist, iters=args.kmeans_iters)
    truth = brute_topk(x, q, args.k).cpu().numpy()
    log("two-stage workload ready %.1fs" % (time.time() - t0))
    eps_list = (0.0, 1.9, 3.0)
    out = {"metric": "QPS at recall@10>=%.2f, two-stage (MSB-first) vs one-stage scan" % args.target_recall,
           "unit": "QPS", "config": {"workload": "embed768: N=%d x 768, %d lists, %d queries, k=%d" %
                                     (args.n, args.nlist, args.nq, args.k)}, "by_bits": []}
    for B in (4, 8):
        ix = erq.Index(dp, B, args.nlist, P)
        ix.set_two_stage(1.0)                      # the build stores the 1-bit data
        ix.build(x, cent, assign, keep_raw=False)
        ix.set_raw(x)
        res = {"bits": B, "best": {}, "by_batch": {}}

        def timed(nq_b, nprobe, rr, reps, qb):
            ws = torch.empty(ix.search_workspace_size(nq_b, nprobe, args.k, rr), dtype=torch.uint8, device=dev)
            o = (torch.empty((nq_b, args.k), dtype=torch.int64, device=dev),
                 torch.empty((nq_b, args.k), dtype=torch.float32, device=dev))
            ix.search(qb, nprobe, args.k, rr, ws=ws, out=o)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            for _ in range(reps):
                ix.search(qb, nprobe, args.k, rr, ws=ws, out=o)
            torch.cuda.synchronize()
            return o[0].cpu().numpy(), nq_b * reps / (time.perf_counter() - ts)

        ix.set_small_batch(0)                          # the two-stage scan lives in the pair-grouped pipeline
        for eps in eps_list:
            ix.set_two_stage(eps)
            rows = []
            for nprobe in (64, 80, 96, 112, 128):
                for rr in (0, 16, 24, 32):
                    ids, qps = timed(args.nq, nprobe, rr, 3, q)
                    rows.append((nprobe, rr, recall_at(ids, truth, args.k), qps))
            ok = [r for r in rows if r[2] >= args.target_recall] or [max(rows, key=lambda r: r[2])]
            b = max(ok, key=lambda r: r[3])
            res["best"][str(eps)] = {"nprobe": b[0], "rerank_k": b[1], "recall@10": b[2], "qps": b[3]}
            if eps > 0:                                # share of 64-member groups whose full codes were skipped
                erq.profile_enable(2)
                erq.profile_read("scan2_groups", reset=True)
                ix.search(q, b[0], args.k, b[1])
                torch.cuda.synchronize()
                sk, ng = erq.profile_read("scan2_groups", reset=True)
                erq.profile_read("scan", reset=True)
                erq.profile_enable(False)
                res["best"][str(eps)]["groups_skipped_frac"] = sk / max(ng, 1)
            log("two-stage B=%d eps0 %.1f: best nprobe %d rerank %d recall %.4f QPS %.0f, groups skipped %.3f" %
                ((B, eps) + b + (res["best"][str(eps)].get("groups_skipped_frac", 0.0),)))
        op = res["best"]["0.0"]
        for bs in (1, 16, 256, 4096):
            row = {}
            for eps in eps_list:
                ix.set_two_stage(eps)
                gph = serve.SearchGraph(ix, bs, op["nprobe"], args.k, op["rerank_k"])
                nb = max(1, min(256, 4096 // bs))
                got = torch.empty((nb * bs, args.k), dtype=torch.int64, device=dev)
                with torch.cuda.stream(gph.stream):       # warm-up replay
                    gph.q.copy_(q[:bs])
                    gph.graph.replay()
                torch.cuda.synchronize()
                ts = time.perf_counter()
                with torch.cuda.stream(gph.stream):       # consecutive batches, results kept on the device
                    for it in range(nb):
                        gph.q.copy_(q[it * bs:(it + 1) * bs])
                        gph.graph.replay()
                        got[it * bs:(it + 1) * bs].copy_(gph.ids)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - ts) / nb
                rec = recall_at(got.cpu().numpy(), truth[:nb * bs], args.k)
                row[str(eps)] = {"qps": bs / dt, "ms_per_batch": dt * 1e3, "recall@10": rec}
                if eps > 0:
                    erq.profile_enable(2)
                    erq.profile_read("scan2_groups", reset=True)
                    ix.search(q[:bs].contiguous(), op["nprobe"], args.k, op["rerank_k"])
                    torch.cuda.synchronize()
                    sk, ng = erq.profile_read("scan2_groups", reset=True)
                    erq.profile_read("scan", reset=True)
                    erq.profile_enable(False)
                    row[str(eps)]["groups_skipped_frac"] = sk / max(ng, 1)
                del gph
            res["by_batch"][str(bs)] = row
            log("two-stage B=%d batch %d: %s" % (B, bs, {e: (round(v["qps"]), round(v["recall@10"], 4),
                                                            round(v.get("groups_skipped_frac", 0), 3))
                                                        for e, v in row.items()}))
        out["by_bits"].append(res)
        ix.close()
        torch.cuda.empty_cache()
    log("total %.1fs" % (time.time() - t0))
    print(json.dumps(out), flush=True)


def run_serving(args):
    """Serving workload: N = 5,000,000 x D = 3072 Gaussian mixture (2048
    components, Zipf weights, sigma 0.3), 16384 k-means lists, B = 4 codes
    and raw vectors resident in HBM; requests of one query with k in {10, 100}
    and nprobe in {16, 64}, Poisson arrivals, admitted by memory."""
    import torch
    from paper_2409_09913_amd import erq, serve, synth
    dev = torch.device("cuda:0")
    erq.load()
    t0 = time.time()
    n, dp, nl, nq = args.serve_n, 3072, 16384, 2000
    x, _ = synth.gmm_device(n, dp, 2048, 0.3, zipf=True, device=dev)
    q = torch.from_numpy(synth.gmm(nq, dp, 2048, 0.3, zipf=True, stream=synth.S_QUERY)).to(dev)
    log("serving workload: %d x %d data in %.1fs" % (n, dp, time.time() - t0))
    ts = time.perf_counter()
    cent, assign = erq.kmeans(x, nl, iters=args.serve_kmeans_iters)
    torch.cuda.synchronize()
    t_km = time.perf_counter() - ts
    sizes = torch.bincount(assign.long(), minlength=nl).cpu().numpy()
    log("k-means %d lists, %d rounds: %.1fs; sizes %d..%d" % (nl, args.serve_kmeans_iters, t_km, sizes.min(),
                                                            sizes.max()))
    ix = erq.Index(dp, 4, nl, None, seed=240909913)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    ix.build(x, cent, assign, keep_raw=False)
    torch.cuda.synchronize()
    enc = n / (time.perf_counter() - ts)
    ix.set_raw(x)
    truth = brute_topk(x, q, 100).cpu().numpy()
    log("encode %.3g codes/s; ground truth done %.1fs" % (enc, time.time() - t0))
    sweep = []
    # isotropic clusters in 3072 dimensions: a query's neighbours spread over all the lists k-means cut its
    # cluster into (up to a few thousand for the Zipf-heavy clusters), so the recall target needs a wide probe
    for kq, rrs in ((10, (0, 50, 200, 1000)), (100, (0, 200, 1000))):
        for npr in (16, 64, 128, 256, 512, 1024):
            for rr in rrs:
                ids, _ = ix.search(q, npr, kq, rr)
                torch.cuda.synchronize()
                tt = time.perf_counter()
                for _ in range(3):
                    ids, _ = ix.search(q, npr, kq, rr)
                torch.cuda.synchronize()
                qps = 3 * nq / (time.perf_counter() - tt)
                rec = recall_at(ids.cpu().numpy(), truth, kq)
                sweep.append({"k": kq, "nprobe": npr, "rerank_k": rr, "recall": rec, "qps": qps})
                log("serving sweep k=%d nprobe %d rerank %d recall@%d %.4f QPS %.0f" % (kq, npr, rr, kq, rec, qps))
    # the recall-target operating point per k: the fastest sweep point reaching it (else the best recall)
    op = {}
    for kq in (10, 100):
        rows = [r for r in sweep if r["k"] == kq]
        ok = [r for r in rows if r["recall"] >= args.target_recall]
        if not ok:      # target out of reach: the fastest point within 0.005 of the best recall
            top = max(r["recall"] for r in rows)
            ok = [r for r in rows if r["recall"] >= top - 0.005]
        op[kq] = max(ok, key=lambda r: r["qps"])
        log("serving k=%d operating point: nprobe %d rerank %d recall %.4f QPS %.0f" %
            (kq, op[kq]["nprobe"], op[kq]["rerank_k"], op[kq]["recall"], op[kq]["qps"]))
    by_rate = {}
    # two request mixes: the workload's nprobe in {16, 64} (re-rank 20 / 200), and each k at its
    # recall-target operating point
    mixes = {"nprobe_16_64": ((16, 64), {10: 20, 100: 200}, 64),
             "recall_target": (None, {kq: op[kq]["rerank_k"] for kq in op}, max(op[kq]["nprobe"] for kq in op))}
    for mix, (nps, rr_of, max_np) in mixes.items():
        np_of = nps if nps is not None else {kq: op[kq]["nprobe"] for kq in op}
        srv = serve.Server(ix, max_batch=256, max_nprobe=max_np, max_k=100,
                           max_rerank=max(max(rr_of.values()), 1), slots=4, mem_budget=4 << 30)
        serve.poisson_run(srv, q, rate=2000.0, n_requests=200, per_request=1, k=(10, 100), nprobes=np_of,
                          rerank_k=rr_of, seed=1)
        by_rate[mix] = {}
        for rate in (1000.0, 2000.0, 5000.0, 10000.0, 20000.0, 50000.0):
            reqs, p50, p99, sq = serve.poisson_run(srv, q, rate=rate, n_requests=args.serve, per_request=1,
                                                   k=(10, 100), nprobes=np_of, rerank_k=rr_of, seed=7)
            hit = [len(set(r.ids[0].cpu().numpy().tolist()) & set(truth[(r.rid * 1) % (nq - 1)][:r.k].tolist()))
                   / r.k for r in reqs[:400]]
            by_rate[mix]["%d_rps" % rate] = {"p50_ms": p50, "p99_ms": p99, "qps": sq,
                                             "recall_mixed_k": float(np.mean(hit)), "batches": srv.batches}
            log("serving [%s] %d req/s: p50 %.3f ms p99 %.3f ms, %.0f QPS, recall (k 10/100 mix) %.4f" %
                (mix, rate, p50, p99, sq, np.mean(hit)))
            if p50 > 200.0:                        # far past capacity: higher rates only queue longer
                break
        del srv
        torch.cuda.empty_cache()
    # scan roofline of a 256-query batch at nprobe 64 (lists rarely shared: the HBM-bound regime)
    erq.profile_enable(True)
    erq.profile_read("scan_b", reset=True)
    ix.search(q[:256].contiguous(), 64, 10, 0)
    torch.cuda.synchronize()
    sb = erq.profile_read("scan_b", reset=True)
    erq.profile_read("scan", reset=True)
    erq.profile_enable(False)
    probes = erq.coarse_probe(q[:256].contiguous(), cent, 64).cpu().numpy()
    roof = scan_roofline(ix, 256, dp, 4, sizes, probes, sb)
    log("scan at batch 256, nprobe 64: %s" % roof)
    out = {"metric": "serving: p50/p99 latency and sustained QPS under Poisson arrivals; QPS at recall@10>=0.95",
           "unit": "QPS", "config": {"workload": "serving: N=%d x D=3072 GMM(2048, Zipf, sigma 0.3), IVF 16384, B=4, "
                                                  "raw resident; requests: 1 query, k in {10,100}, nprobe in "
                                                  "{16,64}" % n},
           "encode_codes_per_s": enc, "kmeans_s": t_km, "sweep": sweep, "operating_points": op,
           "serving": {"by_rate": by_rate},
           "scan_batch256_np64": roof}
    log("total %.1fs" % (time.time() - t0))
    print(json.dumps(out), flush=True)


def run_precision(args):
    """Precision workload: N = 1,000,000 x D = 1536 unit vectors (256
    clusters normalize(mu + g / sqrt(D)), mu uniform on the sphere); one
    k-means of 4096 lists shared by every index; per rotation precision
    (FP32, BF16 matrix cores) and B = 2..8 an index is built from the same
    lists, and 1000 queries of the same mixture are searched at nprobe 256
    without re-rank.  Reported against FP64 exact squared distances (torch
    float64 on the device): recall@10 of the estimated top-10 against the
    exact top-10 over all N, and the relative error |est - d| / d of the
    estimates of each query's 100 returned candidates (mean, 99th
    percentile, maximum); for B >= 5 also with the two-plane int8 query."""
    import torch
    from paper_2409_09913_amd import erq, synth
    dev = torch.device("cuda:0")
    erq.load()
    t0 = time.time()
    n, dp, nl, nq, nprobe = 1_000_000, 1536, 4096, 1000, 256
    x = synth.spherical_clusters_device(n, dp, 256, 1.0, device=dev)
    q = synth.spherical_clusters_device(nq, dp, 256, 1.0, stream=synth.S_QUERY, device=dev)
    cent, assign = erq.kmeans(x, nl, iters=6)
    torch.cuda.synchronize()
    log("precision workload: %d x %d data and k-means in %.1fs" % (n, dp, time.time() - t0))
    # FP64 exact squared distances: the top-10 over all rows per query
    q64 = q.double()
    best_d = torch.full((nq, 10), float("inf"), dtype=torch.float64, device=dev)
    best_i = torch.zeros((nq, 10), dtype=torch.int64, device=dev)
    for lo in range(0, n, 1 << 17):
        xb = x[lo:lo + (1 << 17)].double()
        d = (q64 * q64).sum(1, keepdim=True) + (xb * xb).sum(1)[None, :] - 2.0 * (q64 @ xb.T)
        dd, ii = torch.topk(torch.cat([best_d, d], 1), 10, dim=1, largest=False)
        best_i = torch.gather(torch.cat([best_i, torch.arange(lo, lo + xb.shape[0], device=dev)[None, :].expand(nq, -1)],
                                        1), 1, ii)
        best_d = dd
    truth = best_i.cpu().numpy()
    log("FP64 ground truth %.1fs" % (time.time() - t0))

    def errors(ids, est):
        """|est - d| / d over the returned candidates, d the FP64 exact squared distance."""
        ok = ids >= 0
        idx = torch.where(ok, ids, torch.zeros_like(ids))
        xr = x[idx.reshape(-1)].double().reshape(nq, ids.shape[1], dp)
        d = ((xr - q64[:, None, :]) ** 2).sum(-1)
        rel = ((est.double() - d).abs() / d.clamp_min(1e-12))[ok]
        return float(rel.mean()), float(torch.quantile(rel.float(), 0.99)), float(rel.max())

    out = {"metric": "estimated-distance error and recall@10 against FP64, by rotation precision and B "
                     "(precision workload)", "unit": "relative error",
           "config": {"workload": "precision: N=%d x D=1536 unit vectors, 256 clusters, IVF %d lists, %d queries, "
                                  "nprobe %d, no re-rank" % (n, nl, nq, nprobe)}, "rows": []}
    for prec, pname in ((0, "fp32"), (1, "bf16")):
        for B in range(2, 9):
            ix = erq.Index(dp, B, nl, None, seed=240909913)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            ix.build(x, cent, assign, precision=prec, keep_raw=False)
            torch.cuda.synchronize()
            enc = n / (time.perf_counter() - ts)
            planes = (1, 2) if B >= 5 else (1,)
            for pl in planes:
                ix.set_query_planes(pl)
                ids10, _ = ix.search(q, nprobe, 10, 0)
                ids, est = ix.search(q, nprobe, 100, 0)
                torch.cuda.synchronize()
                rec = recall_at(ids10.cpu().numpy(), truth, 10)
                mean_e, p99_e, max_e = errors(ids, est)
                row = {"rotation": pname, "bits": B, "query_planes": pl, "recall@10": rec,
                       "rel_err_mean": mean_e, "rel_err_p99": p99_e, "rel_err_max": max_e,
                       "encode_codes_per_s": enc}
                out["rows"].append(row)
                log("precision %s B=%d planes %d: recall@10 %.4f, rel. error mean %.3g p99 %.3g max %.3g, "
                    "encode %.3g/s" % (pname, B, pl, rec, mean_e, p99_e, max_e, enc))
            ix.close()
            torch.cuda.empty_cache()
    log("total %.1fs" % (time.time() - t0))
    print(json.dumps(out), flush=True)


def calib_copy():
    """A plain device-to-device copy of 1 GiB, five times: under a counter
    profiler its read and write byte counts per dispatch calibrate the
    counters against a known number of bytes."""
    import torch
    n = 1 << 28                                 # 2^28 float32 = 1 GiB
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy calibration: 5 copies of %d bytes" % (4 * n))
    print(json.dumps({"copy_bytes": 4 * n, "copies": 5}), flush=True)


def host_cores() -> int:
    """Cores this process may run on (the affinity mask, as nproc reports)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(args, x_np, q_np, P_np, cent_np, assign_np, nprobe, rr):
    """The oracle as it stands, on the host cores: the first S queries
    (default 1,000) are probed over all centroids (FP64), the lists they probe
    are encoded by the oracle (untimed: the search needs codes), scanned with
    the int8 estimator and re-ranked exactly; the whole query path is timed
    with every core and again with one thread (the paper's single-thread
    convention) on the first S1 queries.  The oracle's encode rate is timed on
    the first 100,000 rows."""
    import oracle
    cores = host_cores()
    oracle.set_threads(cores)
    S, S1 = min(args.cpu_sample_queries, len(q_np)), min(args.cpu_single_queries, len(q_np))
    sizes = np.bincount(assign_np, minlength=cent_np.shape[0])
    # encode rate: the first 100k rows, each centred on its own list
    ne = min(100_000, len(x_np))
    t1 = time.perf_counter()
    oracle.encode(x_np[:ne], cent_np.astype(np.float64), assign_np[:ne], P_np.astype(np.float64), args.bits)
    enc_rate = ne / (time.perf_counter() - t1)
    log("cpu baseline: oracle encode %.0f codes/s on %d threads (first %d rows)" % (enc_rate, cores, ne))
    probes_all, _ = oracle.probe(q_np[:S], cent_np, nprobe)
    lists = np.unique(probes_all)
    remap = -np.ones(cent_np.shape[0], np.int64)
    remap[lists] = np.arange(len(lists))
    members = [np.nonzero(assign_np == l)[0] for l in lists]
    ids = np.concatenate(members).astype(np.int64)
    off = np.zeros(len(lists) + 1, np.int64)
    off[1:] = np.cumsum([len(m) for m in members])
    asg_local = np.repeat(np.arange(len(lists), dtype=np.int32), [len(m) for m in members])
    log("cpu baseline: encoding %d rows of the %d lists the first %d queries probe" % (len(ids), len(lists), S))
    codes, fa, fr, co, _ = oracle.encode(x_np[ids], cent_np[lists].astype(np.float64), asg_local,
                                         P_np.astype(np.float64), args.bits)
    crot = oracle.rotate(cent_np[lists], P_np).astype(np.float32)
    kk = rr if rr > 0 else args.k
    fa32, fr32 = fa.astype(np.float32), fr.astype(np.float32)

    def path(qs):
        pr, _ = oracle.probe(qs, cent_np, nprobe)
        qrot = oracle.rotate(qs, P_np).astype(np.float32)
        oi, od = oracle.search(off, ids, codes, fa32, fr32, crot, qrot, remap[pr].astype(np.int32), args.bits, kk)
        if rr > 0:
            oi, od = oracle.rerank(x_np, qs, oi, args.k)
        return oi

    t2 = time.perf_counter()
    path(q_np[:S])
    t_all = time.perf_counter() - t2
    oracle.set_threads(1)
    t3 = time.perf_counter()
    path(q_np[:S1])
    t_one = time.perf_counter() - t3
    oracle.set_threads(cores)
    qps, qps1 = S / t_all, S1 / t_one
    log("cpu baseline: %.1f QPS on %d threads (%d queries, %.1f s); %.2f QPS on 1 thread (%d queries, %.1f s)" %
        (qps, cores, S, t_all, qps1, S1, t_one))
    return {"value": qps, "unit": "QPS", "cores": cores, "kind": "oracle",
            "sample": "first %d queries, whole query path once (%.1f s): FP64 probe over %d centroids, rotation, "
                      "int8-estimator scan of nprobe=%d lists, re-rank %d; lists encoded by the oracle first "
                      "(%d rows, untimed)" % (S, t_all, cent_np.shape[0], nprobe, rr, len(ids)),
            "single_thread": {"value": qps1, "unit": "QPS", "cores": 1, "queries": S1, "seconds": t_one},
            "encode_codes_per_s": enc_rate, "encode_sample_rows": ne}


def ivf_flat_fp32(x, q, cent, assign_np, nprobe, k, budget=1 << 27, xbudget=1 << 28):
    """FP32 IVF-Flat on the same lists and the same probe lists (erq's coarse
    probe): exact squared distances ||q||^2 + ||x||^2 - 2 q.x of every member
    of the probed lists as batched FP32 products (torch.bmm, the library
    GEMM), padded groups of lists, top-k per (query, list), then per query.
    Returns a function running the search (timed by the caller) and the
    host-side group tables (built once, outside the timing)."""
    import torch
    from paper_2409_09913_amd import erq
    dev = q.device
    nq, dp = q.shape
    nl = cent.shape[0]
    probes = erq.coarse_probe(q, cent, nprobe).cpu().numpy().astype(np.int64)
    order = np.argsort(assign_np, kind="stable")
    sizes = np.bincount(assign_np, minlength=nl)
    loff = np.zeros(nl + 1, np.int64)
    loff[1:] = np.cumsum(sizes)
    pl = probes.reshape(-1)
    pslot = np.arange(nq * nprobe)
    po = np.argsort(pl, kind="stable")
    pcnt = np.bincount(pl, minlength=nl)
    poff = np.zeros(nl + 1, np.int64)
    poff[1:] = np.cumsum(pcnt)
    lists = [l for l in np.argsort(-sizes, kind="stable") if pcnt[l] > 0 and sizes[l] > 0]
    groups, cur, mq, mm = [], [], 0, 0
    for l in lists:
        nmq, nmm = max(mq, pcnt[l]), max(mm, sizes[l])
        if cur and ((len(cur) + 1) * nmq * nmm > budget or (len(cur) + 1) * nmm * dp > xbudget):
            groups.append(cur)
            cur, nmq, nmm = [], pcnt[l], sizes[l]
        cur.append(l)
        mq, mm = nmq, nmm
    if cur:
        groups.append(cur)
    tabs = []
    for gl in groups:
        G = len(gl)
        mq = int(max(pcnt[l] for l in gl))
        mm = int(max(sizes[l] for l in gl))
        mem = np.zeros((G, mm), np.int64)
        mval = np.zeros((G, mm), bool)
        qs = np.zeros((G, mq), np.int64)
        sl = np.full((G, mq), -1, np.int64)
        for i, l in enumerate(gl):
            m = order[loff[l]:loff[l + 1]]
            mem[i, :len(m)] = m
            mval[i, :len(m)] = True
            ps = pslot[po[poff[l]:poff[l + 1]]]
            qs[i, :len(ps)] = ps // nprobe
            sl[i, :len(ps)] = ps
        tabs.append(tuple(torch.from_numpy(a).to(dev) for a in (mem, mval, qs, sl)))
    xn = (x * x).sum(1)
    qn = (q * q).sum(1)
    kk = k

    def run():
        best_d = torch.full((nq * nprobe, kk), float("inf"), device=dev)
        best_i = torch.full((nq * nprobe, kk), -1, dtype=torch.int64, device=dev)
        for mem, mval, qs, sl in tabs:
            X = x[mem]                                       # G x mm x dp
            Q = q[qs]                                        # G x mq x dp
            d = qn[qs][:, :, None] + xn[mem][:, None, :] - 2.0 * torch.bmm(Q, X.transpose(1, 2).contiguous())
            d = d.masked_fill(~mval[:, None, :], float("inf"))
            kt = min(kk, d.shape[2])
            tv, ti = torch.topk(d, kt, dim=2, largest=False)
            ids = torch.gather(mem[:, None, :].expand(-1, d.shape[1], -1), 2, ti)
            ok = sl >= 0
            best_d[sl[ok], :kt] = tv[ok]
            best_i[sl[ok], :kt] = ids[ok]
        bd = best_d.view(nq, nprobe * kk)
        bi = best_i.view(nq, nprobe * kk)
        tv, ti = torch.topk(bd, kk, dim=1, largest=False)
        return torch.gather(bi, 1, ti)

    return run


def estimator_recall(ix, cent, q_np, P_np, truth_np, nprobe, k, B, S):
    """Recall@k without re-rank of the paper's float-query estimator (the
    oracle in FP64, factor form with the index's stored codes and factors)
    beside the int8-query estimator of the GPU scan, on the first S queries
    with the same probe lists."""
    import torch
    import oracle
    from paper_2409_09913_amd import erq
    dev = torch.device("cuda:0")
    off, ids, codes, fa, fr, crot = [t.cpu().numpy() for t in ix.export()]
    qs = torch.from_numpy(np.ascontiguousarray(q_np[:S])).to(dev)
    probes = erq.coarse_probe(qs, cent, nprobe).cpu().numpy()
    gi, _ = ix.search(qs, nprobe, k, 0)
    gi = gi.cpu().numpy()
    qrot = oracle.rotate(q_np[:S], P_np).astype(np.float32)
    fi, _ = oracle.search(off, ids, codes, fa, fr, crot, qrot, probes, B, k, est_mode=2)
    out = {"bits": B, "nprobe": nprobe, "queries": S, "recall_int8_query": recall_at(gi, truth_np[:S], k),
           "recall_float_query": recall_at(fi, truth_np[:S], k)}
    if B >= 5:                                  # the int8 query in two planes (GPU)
        ix.set_query_planes(2)
        g2, _ = ix.search(qs, nprobe, k, 0)
        ix.set_query_planes(1)
        out["recall_int8_two_planes"] = recall_at(g2.cpu().numpy(), truth_np[:S], k)
    return out


if __name__ == "__main__":
    main()
