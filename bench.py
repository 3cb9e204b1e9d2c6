#!/usr/bin/env python3
"""LIDER batched search on one MI355X: queries/s at recall@10 >= 0.9.

Workload (synthetic, generated on the GPU): N=1,000,000 fp32 vectors, d=768,
from a 1,000-component Gaussian mixture (component norms U[8, 12], sigma 0.5),
stand-in for the paper's 768-d passage corpora; 10,000 queries = corpus points
+ N(0, 0.1^2) noise.  Index: 1,000 k-means clusters (farthest-first seeds, 20
Lloyd iterations, on the GPU), E2LSH m=8, w=2.0, RMI fanout 64.

A step is one lider_search of the whole 10,000-query batch (hashing, layer-1
routing, layer-2 windows, rerank, top-k) with queries already in HBM.  The
operating point (c clusters, r rows per cluster window, r1 centroids in the
layer-1 window) is the fastest of a small sweep whose recall@10 against exact
search is >= 0.9; the literal point (c=8, r=256) is reported beside it.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per rerank launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading for a
    plain copy of known size), or None if the kernel source changed since."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "rerank_1M_hbm_traffic.json")
    src = os.path.join(root, "paper_2205_00970_amd", "csrc", "search.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    return rec["bytes_per_launch"] if rec.get("search_hip_sha256") == digest else None


def exact_topk(torch, X, Q, k, chunk=1000):
    """Exact inner-product top-k (fp32 GEMM on the GPU) for recall."""
    ids, scs = [], []
    for a in range(0, Q.shape[0], chunk):
        s = Q[a:a + chunk] @ X.T
        v, i = torch.topk(s, k, dim=1)
        ids.append(i)
        scs.append(v)
        del s
    return torch.cat(ids), torch.cat(scs)


def recall_at(torch, X, Q, ids, gt_scores, k, tol=1e-4, chunk=1000):
    """Fraction of returned ids (first k) whose exact score reaches the k-th
    exact score (ties within tol*|q|*|x| count)."""
    hits = 0
    for a in range(0, Q.shape[0], chunk):
        ii = ids[a:a + chunk, :k]
        q = Q[a:a + chunk]
        valid = ii >= 0
        rows = X[ii.clamp(min=0)]
        xs = (rows * q[:, None, :]).sum(-1)
        thr = gt_scores[a:a + chunk, k - 1:k] - tol * q.norm(dim=1, keepdim=True) * rows.norm(dim=2)
        hits += int(((xs >= thr) & valid).sum().item())
    return hits / float(ids.shape[0] * k)


def pair_unions(torch, gi, dbg, c):
    """Per (query, routed cluster) pair: the number of distinct window rows
    (the union of its H windows, in the stored corpus order), and the set of
    distinct rows over all pairs.  Returns (per-pair counts [nq*c] int64 with
    0 for pads, union row count, hull rows summed over pairs)."""
    dev = dbg["routed"].device
    H = gi.H
    routed = dbg["routed"].reshape(-1).long()
    pr = dbg["pairs"].reshape(routed.shape[0], H, 3)
    off = torch.from_numpy(gi.export("offsets")).to(dev)
    perm = torch.from_numpy(gi.export("perm")).to(dev).reshape(H, -1)
    n = perm.shape[1]
    inv0 = torch.empty_like(perm[0])
    inv0[perm[0]] = torch.arange(n, device=dev)
    seen = torch.zeros(n, dtype=torch.bool, device=dev)
    counts = torch.zeros(routed.shape[0], dtype=torch.int64, device=dev)
    hull = 0
    valid = torch.nonzero(routed >= 0).reshape(-1)
    rmax = int(pr[..., 2].max().item()) if valid.numel() else 0
    ar = torch.arange(max(rmax, 1), device=dev)
    for a in range(0, valid.numel(), 4096):
        v = valid[a:a + 4096]
        j = routed[v]
        st = pr[v, :, 1]
        ln = pr[v, :, 2]
        gpos = off[j][:, None, None] + st[..., None] + ar[None, None, :]  # [P, H, rmax]
        ok = ar[None, None, :] < ln[..., None]
        hidx = torch.arange(H, device=dev)[None, :, None].expand_as(gpos)
        ids = perm[hidx, gpos.clamp(max=n - 1)]
        p0 = torch.where(ok, inv0[ids], torch.full_like(ids, -1)).reshape(v.numel(), -1)
        p0s, _ = torch.sort(p0, dim=1)
        distinct = ((p0s[:, 1:] != p0s[:, :-1]) & (p0s[:, 1:] >= 0)).sum(1) + (p0s[:, 0] >= 0).long()
        counts[v] = distinct
        seen[p0s[p0s >= 0]] = True
        mx = torch.where(p0 >= 0, p0, torch.full_like(p0, -1)).max(1).values
        mn = torch.where(p0 >= 0, p0, torch.full_like(p0, n)).min(1).values
        hull += int((mx - mn + 1).clamp(min=0).sum().item())
    return counts, int(seen.sum().item()), hull


def rerank_roofline(torch, gi, Q, k, c, r, r1, rr_ms, **kw):
    """Roofline of one rerank launch.  Algorithmic bytes = the distinct window
    rows U times 4d (each row of the union read once); algorithmic flops = 2d
    per (pair, distinct row of the pair's union).  The bound is whichever of
    HBM (8 TB/s) and fp32 MFMA (157.3 TFLOP/s) takes longer for these amounts;
    `achieved` / `frac` are for that bound.  Query and score bytes are
    reported separately (not part of the algorithmic figure)."""
    _, _, dbg = gi.search(Q, k, c, r, r1=r1, debug=True, **kw)
    if gi.H == 1:
        dbg = dict(routed=dbg["routed"], pairs=dbg["pairs"][:, :, None, :])
    counts, U, hull = pair_unions(torch, gi, dbg, c)
    d = gi.d
    t = rr_ms * 1e-3
    alg_bytes = U * 4 * d
    flops = int(counts.sum().item()) * 2 * d
    pairs_rows = int(counts.sum().item())
    t_hbm, t_mfma = alg_bytes / 8.0e12, flops / 157.3e12
    hbm = dict(bound="hbm", achieved=round(alg_bytes / t / 1e9, 1), peak=8000.0, unit="GB/s",
               frac=round(alg_bytes / t / 8.0e12, 4))
    mf = dict(bound="mfma", achieved=round(flops / t / 1e12, 2), peak=157.3, unit="TFLOP/s",
              frac=round(flops / t / 157.3e12, 4))
    main_b, other = (hbm, mf) if t_hbm >= t_mfma else (mf, hbm)
    out = dict(main_b)
    out.update(traffic=None,
               traffic_unit="HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
               kernel="rerank_wg_kernel (fp32 operand-ordered feed, a workgroup of 4 waves per 128-row tile)",
               kernel_ms=round(rr_ms, 4), union_rows=U, hull_rows=hull, pair_rows=pairs_rows,
               algorithmic_bytes=alg_bytes, algorithmic_flops=flops,
               query_bytes=Q.shape[0] * 4 * d, score_bytes=hull * 4,
               other_bound={kk: other[kk] for kk in ("bound", "achieved", "peak", "unit", "frac")})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--nq", type=int, default=10_000)
    ap.add_argument("--clusters", type=int, default=1000)
    ap.add_argument("--point", default="", help="c,r,r1: skip the sweep")
    ap.add_argument("--quick", action="store_true",
                    help="profiling run: no sweep, no side measurements, no CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--streams", type=int, default=1,
                    help="consecutive batches alternate over this many streams, each with its own "
                         "workspace and outputs (1: every step on one stream, the kernels' isolated "
                         "durations; the other setting of 1 / 2 is timed after it and reported too)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--workload", default="search", choices=["search", "batching", "serving"],
                    help="search: the 1M x 768 headline; batching: 4M x 768 Zipf clusters, "
                         "65,536 queries in batches of 1-4096; serving: see serving.py")
    ap.add_argument("--serve-n", dest="serve_n", type=int, default=0,
                    help="serving workload corpus size (default 21,000,000)")
    ap.add_argument("--serve-queries", dest="serve_queries", type=int, default=0,
                    help="queries per arrival rate in the serving workload (default 110,000)")
    ap.add_argument("--calib", action="store_true",
                    help="also run a plain 1 GiB fp32 copy kernel (HBM counter calibration)")
    ap.add_argument("--labels", action="store_true",
                    help="cluster by the generator's component labels instead of k-means")
    ap.add_argument("--arrays", type=int, default=0,
                    help="H hashkey arrays per core model (implies --labels; E2LSH draws of seed 31, "
                         "the same as the bench line's several-arrays measurements)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2205_00970_amd import datagen, lider

    torch.backends.cuda.matmul.allow_tf32 = False
    if args.workload == "batching":
        return run_batching(args, torch, datagen, lider)
    if args.workload == "serving":
        from paper_2205_00970_amd import serving
        return serving.bench_main(args, exact_topk, recall_at)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, d, C, m, w, F = args.n, 768, args.clusters, 8, 2.0, 64
    t0 = time.time()
    X, lab = datagen.mixture(n, d, ncomp=C, seed=0, device="cuda")
    Q, src = datagen.queries_from(X, args.nq, 0.1, seed=1)
    A, b = datagen.lsh_params(m, d, w, seed=2)
    init = datagen.kmeans_init(n, C, seed=3)
    torch.cuda.synchronize()
    log(f"data {n}x{d} + {args.nq} queries in {time.time() - t0:.1f}s")
    t0 = time.time()
    H = max(1, args.arrays)
    if args.labels or args.arrays:
        if args.arrays:
            A, b = datagen.lsh_params(m, d, w, seed=31, n_arrays=H)
        gi = lider.Index(X, C, m, w, F, (A, b), assignment=lab, storage="bf16",
                         centroid_storage="fp8", n_arrays=H)
    else:
        gi = lider.Index(X, C, m, w, F, (A, b), kmeans_init=init, kmeans_iters=20, storage="bf16",
                         centroid_storage="fp8", seeding="farthest")
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log(f"build {build_s:.2f}s, k-means iterations {gi.iters_run}, largest cluster {gi.max_cluster}")
    Lmax = int(gi.max_cluster)

    gt_ids, gt_sc = exact_topk(torch, X, Q, 100)
    torch.cuda.synchronize()

    def run(k, c, r, r1, **kw):
        return gi.search(Q, k, c, r, r1=r1, **kw)

    def timed(k, c, r, r1, reps=5, **kw):
        ids = torch.empty((args.nq, k), dtype=torch.int64, device=dev)
        sc = torch.empty((args.nq, k), dtype=torch.float32, device=dev)
        run(k, c, r, r1, out=(ids, sc), **kw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            run(k, c, r, r1, out=(ids, sc), **kw)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps, ids, sc

    # ---- operating point: fastest sweep point with recall@10 >= 0.9
    sweep = []
    if args.point:
        c, r, r1 = (int(v) for v in args.point.split(","))
        point = (c, r, r1)
    else:
        cands = [(1, Lmax, C), (2, Lmax, C), (3, Lmax, C), (4, Lmax, C), (2, 512, C),
                 (4, 512, C), (8, 512, C), (8, 256, C), (16, 256, C), (8, 256, 256)]
        best = None
        for (c, r, r1) in cands:
            dt, ids, _ = timed(10, c, r, r1, reps=3)
            rec = recall_at(torch, X, Q, ids, gt_sc, 10)
            qps = args.nq / dt
            sweep.append(dict(c=c, r=r, r1=r1, recall10=round(rec, 4), qps=round(qps)))
            log(f"sweep c={c} r={r} r1={r1}: recall@10={rec:.4f} {qps:,.0f} q/s")
            if rec >= 0.9 and (best is None or qps > best[0]):
                best = (qps, (c, r, r1))
        point = best[1] if best else (8, Lmax, C)
    c, r, r1 = point

    # ---- timed region: W warmup steps, then exactly K steps.  Step i runs on
    # stream i mod S with that stream's workspace and output buffers; with
    # S = 2 one batch's short latency-bound stages (hashing, routing, work
    # list, selection) overlap the previous batch's HBM-bound rerank.  Every
    # step is one whole pass of the path over one 10,000-query batch.
    k = 10
    nst = max(1, args.streams)
    need = gi.workspace_bytes(args.nq, k, c, r, r1=r1)
    streams = [torch.cuda.Stream() for _ in range(max(nst, 2))]
    wss = [torch.empty(max(need, 256), dtype=torch.uint8, device=dev) for _ in streams]
    outs = [(torch.empty((args.nq, k), dtype=torch.int64, device=dev),
             torch.empty((args.nq, k), dtype=torch.float32, device=dev)) for _ in streams]
    torch.cuda.synchronize()

    def steps_on(ns, count):
        for i in range(count):
            run(k, c, r, r1, out=outs[i % ns], stream=streams[i % ns], ws=wss[i % ns])

    steps_on(nst, args.warmup)
    torch.cuda.synchronize()
    t = time.perf_counter()
    steps_on(nst, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    # the other stream setting (2 when the timed steps used 1), for reference;
    # not under --quick, whose kernel traces then hold isolated launches only
    alt_nst = 2 if nst == 1 else 1
    alt_qps = None
    if not args.quick:
        steps_on(alt_nst, args.warmup)
        torch.cuda.synchronize()
        t = time.perf_counter()
        steps_on(alt_nst, args.steps)
        torch.cuda.synchronize()
        alt_qps = args.nq / ((time.perf_counter() - t) / args.steps)
    ids, sc = outs[0]
    used = max(nst, alt_nst) if alt_qps else nst  # output buffers written
    if not all(torch.equal(ids, o[0]) and torch.equal(sc, o[1]) for o in outs[1:used]):
        raise RuntimeError("batches on different streams gave different results")
    # stage times: the same steps again with HIP events between the stages
    # (recording them costs a few microseconds each, so they stay out of the
    # timed region above)
    lider.profile_begin(args.steps)
    for _ in range(args.steps):
        run(k, c, r, r1, out=(ids, sc))
    torch.cuda.synchronize()
    stages, calls = lider.profile_end()
    ms_per_step = elapsed * 1e3 / args.steps
    value = args.nq / (elapsed / args.steps)
    rec = recall_at(torch, X, Q, ids, gt_sc, 10)
    stage_avg = {s: v / calls for s, v in stages.items()}
    log(f"point c={c} r={r} r1={r1}: {value:,.0f} q/s, {ms_per_step:.3f} ms/step, recall@10 {rec:.4f} "
        f"({nst} stream(s)" + (f"; {alt_nst} stream(s): {alt_qps:,.0f} q/s)" if alt_qps else ")"))
    log("stage ms/step: " + ", ".join(f"{s}={v:.3f}" for s, v in stage_avg.items()))

    # ---- roofline of the rerank kernel (algorithmic bytes / measured duration)
    rr_ms = stage_avg["rerank"]
    roofline = rerank_roofline(torch, gi, Q, k, c, r, r1, rr_ms)
    roofline["traffic"] = measured_traffic() if H == 1 and not args.labels else None
    log(f"rerank: union rows {roofline['union_rows']:,}, {rr_ms:.3f} ms -> "
        f"{roofline['achieved']:,.1f} {roofline['unit']} ({roofline['frac']:.1%} of peak, "
        f"bound {roofline['bound']})")

    extra = {}
    if args.calib:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).uniform_()
        bcopy = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=bcopy)
        torch.cuda.synchronize()
        del a, bcopy
        log("calibration copy: 3 x (1 GiB read + 1 GiB write)")
    if not args.quick:
        # literal point (c=8, r=256, r1=r) for k=10 and k=100, with its stages
        # and the rerank's roofline
        for kk in (10, 100):
            dt, li, _ = timed(kk, 8, 256, 0, reps=5)
            lider.profile_begin(5)
            for _ in range(5):
                run(kk, 8, 256, 256)
            torch.cuda.synchronize()
            lst, lcalls = lider.profile_end()
            rl = rerank_roofline(torch, gi, Q, kk, 8, 256, 256, lst["rerank"] / lcalls)
            extra[f"literal_k{kk}"] = dict(
                c=8, r=256, r1=256, qps=round(args.nq / dt),
                recall10=round(recall_at(torch, X, Q, li, gt_sc, 10), 4),
                stage_ms={s2: round(v / lcalls, 4) for s2, v in lst.items()},
                roofline={kk2: rl[kk2] for kk2 in ("bound", "achieved", "unit", "frac", "union_rows",
                                                  "pair_rows", "other_bound")})
            log(f"literal c=8 r=256 k={kk}: {args.nq / dt:,.0f} q/s, recall@10 "
                f"{extra[f'literal_k{kk}']['recall10']}, rerank {rl['frac']:.1%} of {rl['bound']} peak")
        # k=100 at the operating point
        dt, li, _ = timed(100, c, r, r1, reps=5)
        extra["point_k100"] = dict(qps=round(args.nq / dt),
                                   recall100=round(recall_at(torch, X, Q, li, gt_sc, 100), 4))
        # precision form: bf16 windows, exact routing from the bf16 layer-1
        # product, the certified shortlist (every candidate within the bf16
        # error margin of the k-th best) reranked in fp32: the fp32 top k
        def precision_entry(kk, cc, rr, rr1):
            dt, pi, ps = timed(kk, cc, rr, rr1, reps=5, precision="bf16")
            fi, _ = run(kk, cc, rr, rr1)
            rows = X[pi.clamp(min=0)]
            xs = (rows.double() * Q.double()[:, None, :]).sum(-1)
            err = ((ps.double() - xs).abs()
                   / (Q.double().norm(dim=1, keepdim=True) * rows.double().norm(dim=2)))[pi >= 0]
            e = err.cpu().numpy()
            out = dict(c=cc, r=rr, r1=rr1, k=kk, shortlist="certified", qps=round(args.nq / dt),
                       recall10=round(recall_at(torch, X, Q, pi, gt_sc, 10), 4),
                       ids_equal_fp32_path=round(float((pi == fi).float().mean().item()), 6),
                       rel_score_err={"p50": float(np.percentile(e, 50)),
                                      "p99": float(np.percentile(e, 99)), "max": float(e.max())})
            del rows, xs, err
            return out
        extra["precision_bf16"] = precision_entry(10, c, r, r1)
        log(f"precision form (certified): {extra['precision_bf16']['qps']:,} q/s, recall@10 "
            f"{extra['precision_bf16']['recall10']}")
        extra["precision_bf16_literal"] = precision_entry(10, 8, 256, 256)
        log(f"precision form (certified), literal point: "
            f"{extra['precision_bf16_literal']['qps']:,} q/s")
        # fixed-length shortlists (the mult*k best bf16 scores): approximate
        extra["precision_bf16_shortlist"] = []
        for mult in (4, 2):
            dt, pi, _ = timed(10, c, r, r1, reps=5, precision="bf16", shortlist_mult=mult)
            rec_s = round(recall_at(torch, X, Q, pi, gt_sc, 10), 4)
            extra["precision_bf16_shortlist"].append(dict(shortlist=f"{mult}k", qps=round(args.nq / dt),
                                                          recall10=rec_s))
            log(f"precision form, shortlist {mult}k: {args.nq / dt:,.0f} q/s, recall@10 {rec_s}")
        extra["persistent_qps"] = round(args.nq / timed(10, c, r, r1, reps=5, persistent=True)[0])
        extra["cosine"] = cosine_variant(args, torch, datagen, lider, X, lab, Q, C, F, log)
        extra["arrays"] = arrays_variant(args, torch, datagen, lider, X, lab, Q, C, F, log, gt_sc)

    cpu = None
    if not args.quick and not args.no_cpu_baseline:
        # the oracle indexes the same partition as the timed index (its k-means
        # assignment, or the labels with --labels)
        assign = torch.from_numpy(gi.export("assign").astype(np.int64))
        cpu = cpu_baseline(X, assign, Q, A, b, C, m, w, F, c, r, r1, args.cpu_seconds)

    line = {
        "metric": "queries/s at recall@10>=0.9 (1Mx768)",
        "value": round(value, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"gaussian-mixture N={n} d={d} fp32, {C} "
                               + ("clusters = the generator's labels" if args.labels or args.arrays
                                  else "k-means clusters")
                               + (f", H={H} hashkey arrays" if H > 1 else "")
                               + f", m={m} w={w} rmi_fanout={F}, {args.nq} queries (noise 0.1)",
                   "global_batch": args.nq, "k": k, "c": c, "r": r, "r1": r1,
                   "recall10": round(rec, 4), "parallelism": "single-gpu", "streams": nst},
        f"qps_{alt_nst}_stream{'s' if alt_nst > 1 else ''}": round(alt_qps) if alt_qps else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stage_ms": {s: round(v, 4) for s, v in stage_avg.items()},
        "build_s": round(build_s, 2),
        "sweep": sweep,
        **extra,
    }
    print(json.dumps(line), flush=True)


def run_batching(args, torch, datagen, lider):
    """Batching form: N=4,000,000 d=768 (bf16 copy + fp32 master), 4,096 clusters
    with Zipf(1.1) sizes in [50, 200,000] (the generator's components, given as
    the clustering), 65,536 queries in batches of U[1, 4096]; c=16, r=512,
    k=100.  Plain schedule vs the autotuned (possibly persistent) one."""
    from paper_2205_00970_amd import autotune
    dev = torch.device("cuda:0")
    n, d, C, m, w, F = 4_000_000, 768, 4096, 8, 2.0, 64
    k, c, r = 100, 16, 512
    t0 = time.time()
    sizes = datagen.zipf_sizes(n, C, 1.1, 50, 200_000)
    X, lab = datagen.mixture(n, d, ncomp=C, seed=10, device="cuda", sizes=sizes)
    Q, _ = datagen.queries_from(X, 65536, 0.1, seed=11)
    A, b = datagen.lsh_params(m, d, w, seed=12)
    torch.cuda.synchronize()
    log(f"data {n}x{d}, cluster sizes {sizes.max()}..{sizes.min()}, in {time.time() - t0:.1f}s")
    t0 = time.time()
    gi = lider.Index(X, C, m, w, F, (A, b), assignment=lab, storage="bf16", centroid_storage="fp8")
    torch.cuda.synchronize()
    log(f"build {time.time() - t0:.2f}s")
    g = np.random.default_rng(13)
    bs = []
    tot = 0
    while tot < Q.shape[0]:
        bsz = int(min(g.integers(1, 4097), Q.shape[0] - tot))
        bs.append((tot, bsz))
        tot += bsz
    sample = Q[:2048].contiguous()
    gt_ids, gt_sc = exact_topk(torch, X, sample, k)
    tuner = autotune.Autotuner(gi)
    res = {"workload": f"gaussian-mixture N={n} d={d}, {C} Zipf(1.1) clusters "
                       f"({int(sizes.min())}..{int(sizes.max())} rows), 65,536 queries in "
                       f"{len(bs)} batches of U[1,4096]", "k": k, "c": c, "r": r}
    for prec in ("f32", "bf16"):
        for r1 in (r, C):
            ids, _ = gi.search(sample, k, c, r, r1=r1, precision=prec)
            rec = recall_at(torch, X, sample, ids, gt_sc, 10)
            # tune every batch-size bucket on a representative batch
            buckets = sorted({autotune.bucket(bsz) for _, bsz in bs})
            for bk in buckets:
                tuner.tune(Q[:min(bk, Q.shape[0])].contiguous(), k, c, r, r1, prec)
            for mode in ("plain", "tuned"):
                outs = []
                for a, bsz in bs:  # warm (and allocate workspaces)
                    gi.search(Q[a:a + bsz], k, c, r, r1=r1, precision=prec)
                torch.cuda.synchronize()
                t = time.perf_counter()
                for a, bsz in bs:
                    sch = tuner.schedule(bsz, k, c, r, r1, prec) if mode == "tuned" else {}
                    gi.search(Q[a:a + bsz], k, c, r, r1=r1, precision=prec, **sch)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                res[f"{prec}_r1_{r1}_{mode}_qps"] = round(Q.shape[0] / dt)
                log(f"{prec} r1={r1} {mode}: {Q.shape[0] / dt:,.0f} q/s (recall@10 {rec:.4f})")
            res[f"{prec}_r1_{r1}_recall10"] = round(rec, 4)
    res["schedules"] = tuner.cache
    print(json.dumps(res), flush=True)


def cosine_variant(args, torch, datagen, lider, X, lab, Q, C, F, log):
    """The cosine variant on the same mixture, rows and queries normalised:
    random-hyperplane bits (m = 10 = ceil(log2 of the ~1,000-row clusters)),
    key = Decimal(bits), clusters = the generator's labels.  Recall@10 and q/s
    at the literal point (c=8, r=r1=256) with the fixed window and with the
    dist_e-guided expansion (B = 3), and at whole-cluster windows."""
    Xn = datagen.normalize_rows(X)
    Qn = datagen.normalize_rows(Q)
    m = 10
    A, _ = datagen.lsh_params(m, X.shape[1], 1.0, seed=12)
    gi = lider.Index(Xn, C, m, 1.0, F, (A, None), assignment=lab.to(torch.int32),
                     hash_kind="sign")
    _, gt_sc = exact_topk(torch, Xn, Qn, 10)
    out = {"m": m}
    for name, (c, r, r1, B) in {"literal_fixed": (8, 256, 256, 0),
                                "literal_expand_B3": (8, 256, 256, 3),
                                "whole_cluster": (1, int(gi.max_cluster), C, 0)}.items():
        ids = torch.empty((Qn.shape[0], 10), dtype=torch.int64, device=Qn.device)
        sc = torch.empty((Qn.shape[0], 10), dtype=torch.float32, device=Qn.device)
        gi.search(Qn, 10, c, r, r1=r1, expand_bits=B, out=(ids, sc))
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            gi.search(Qn, 10, c, r, r1=r1, expand_bits=B, out=(ids, sc))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / 5
        rec = recall_at(torch, Xn, Qn, ids, gt_sc, 10)
        out[name] = dict(c=c, r=r, r1=r1, expand_bits=B, qps=round(Qn.shape[0] / dt),
                         recall10=round(rec, 4))
        log(f"cosine {name}: {Qn.shape[0] / dt:,.0f} q/s, recall@10 {rec:.4f}")
    del gi, Xn
    torch.cuda.empty_cache()
    return out


def arrays_variant(args, torch, datagen, lider, X, lab, Q, C, F, log, gt_sc, H_list=(1, 4, 10)):
    """Multi-array core models (Section 3.3.1) on the same mixture, clusters =
    the generator's labels, E2LSH m=8 w=2 per array: recall@10 and q/s at the
    literal window (c=8, r=r1=256) and at c=4, r=128, r1=C for H = 1, 4, 10
    (H=10 is the paper's setting), with the per-stage times of each."""
    m, w = 8, 2.0
    out = {"m": m, "w": w}
    for H in H_list:
        A, b = datagen.lsh_params(m, X.shape[1], w, seed=31, n_arrays=H)
        t0 = time.time()
        gi = lider.Index(X, C, m, w, F, (A, b), assignment=lab.to(torch.int32), n_arrays=H,
                         storage="bf16" if H > 1 else "f32")
        torch.cuda.synchronize()
        bs = time.time() - t0
        res = {"build_s": round(bs, 2)}
        for name, (c, r, r1) in {"literal": (8, 256, 256), "c4_r128": (4, 128, C)}.items():
            ids = torch.empty((Q.shape[0], 10), dtype=torch.int64, device=Q.device)
            sc = torch.empty((Q.shape[0], 10), dtype=torch.float32, device=Q.device)
            gi.search(Q, 10, c, r, r1=r1, out=(ids, sc))
            torch.cuda.synchronize()
            lider.profile_begin(5)
            t = time.perf_counter()
            for _ in range(5):
                gi.search(Q, 10, c, r, r1=r1, out=(ids, sc))
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / 5
            stages, calls = lider.profile_end()
            rec = recall_at(torch, X, Q, ids, gt_sc, 10)
            res[name] = dict(c=c, r=r, r1=r1, qps=round(Q.shape[0] / dt), recall10=round(rec, 4),
                             stage_ms={s: round(v / calls, 4) for s, v in stages.items()})
            rl = rerank_roofline(torch, gi, Q, 10, c, r, r1, stages["rerank"] / calls)
            if H > 1 and name == "literal":  # the precision form (certified shortlist) beside it
                gi.search(Q, 10, c, r, r1=r1, precision="bf16", out=(ids, sc))
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(5):
                    gi.search(Q, 10, c, r, r1=r1, precision="bf16", out=(ids, sc))
                torch.cuda.synchronize()
                dtp = (time.perf_counter() - t) / 5
                res["precision_bf16_literal"] = dict(
                    qps=round(Q.shape[0] / dtp), recall10=round(recall_at(torch, X, Q, ids, gt_sc, 10), 4))
                log(f"arrays H={H} literal, precision form: {Q.shape[0] / dtp:,.0f} q/s")
            res[name]["roofline"] = {kk: rl[kk] for kk in ("bound", "achieved", "unit", "frac",
                                                          "union_rows", "hull_rows", "pair_rows",
                                                          "other_bound")}
            log(f"arrays H={H} {name}: {Q.shape[0] / dt:,.0f} q/s, recall@10 {rec:.4f}, "
                + ", ".join(f"{s}={v / calls:.3f}" for s, v in stages.items()))
        out[f"H{H}"] = res
        gi.close()
        del gi
        torch.cuda.empty_cache()
    return out


def cpu_baseline(X, lab, Q, A, b, C, m, w, F, c, r, r1, seconds):
    """The FP64 oracle's search, timed on this host's cores on a sample of the
    queries.  The oracle index is built over the same corpus with the timed GPU
    index's cluster assignment (`lab`; the oracle's own FP64 k-means at this
    size would take hours); the build is not timed."""
    import oracle
    import torch
    t0 = time.time()
    Xh = X.cpu().numpy()
    Qh = Q.cpu().numpy()
    oi = oracle.Index(Xh, C, A, b, m, w, F, assignment=lab.cpu().numpy())
    log(f"oracle index built in {time.time() - t0:.1f}s")
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    probe = 64
    t = time.perf_counter()
    oi.search(Qh[:probe], 10, c, r, r1)
    per_q = (time.perf_counter() - t) / probe
    nsamp = int(min(Qh.shape[0], max(probe, seconds / max(per_q, 1e-6))))
    t = time.perf_counter()
    oi.search(Qh[:nsamp], 10, c, r, r1)
    dt = time.perf_counter() - t
    log(f"oracle: {nsamp} queries in {dt:.2f}s on {threads} threads")
    del torch
    return {"value": round(nsamp / dt, 2), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"first {nsamp} of the queries at c={c} r={r} r1={r1} k=10, FP64, "
                      f"oracle index over the timed index's cluster assignment"}


if __name__ == "__main__":
    main()
