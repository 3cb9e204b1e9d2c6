"""Serving form: continuous batching of LIDER search requests on one GPU.

The index stays resident in HBM.  Requests (a batch of 1-256 query rows and a
k) arrive open-loop.  A scheduler admits pending requests FIFO into the next
batch while (a) an execution slot is free and (b) the batch's search
workspace fits the memory budget left by the batches in flight; requests of
one k share a batch.  Each batch runs on its slot's own HIP stream (default
priority), so batches launched at different ticks overlap on the device;
completion is detected by polling the slot's event.  Per-query results do not
depend on batch composition (every score and selection is computed per
query), so a request's answer is the same alone and in the mix.

The executor is an interface: GpuExecutor runs lider_search through the C ABI;
FakeExecutor (tests) completes batches after a deterministic simulated delay
on the CPU and can inject failures.
"""
from __future__ import annotations

import collections
import time

import numpy as np


class Request:
    __slots__ = ("rid", "arrival", "rows", "k", "status", "launch", "done", "ids", "scores",
                 "error")

    def __init__(self, rid, arrival, rows, k):
        self.rid, self.arrival, self.rows, self.k = rid, float(arrival), rows, int(k)
        self.status = "new"  # new -> pending -> running -> done | failed | rejected
        self.launch = self.done = None
        self.ids = self.scores = None
        self.error = None

    @property
    def nq(self):
        return int(self.rows.shape[0])


class Batch:
    def __init__(self, bid, slot, k, reqs, ws_bytes):
        self.bid, self.slot, self.k, self.reqs, self.ws_bytes = bid, slot, k, reqs, ws_bytes
        self.handle = None


# ----------------------------------------------------------------- executors
class GpuExecutor:
    """Runs batches with lider_search_ex on `slots` HIP streams."""

    def __init__(self, index, queries, c, r, r1=0, precision="f32", slots=4, max_batch=4096,
                 max_k=100, schedule=None):
        import torch
        self.torch = torch
        self.schedule = dict(schedule or {})
        self.index, self.Q = index, queries
        self.c, self.r, self.r1, self.precision = c, r, r1, precision
        self.max_batch, self.max_k = max_batch, max_k
        dev = queries.device
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(slots)]
        cap = index.workspace_bytes(max_batch, max_k, c, r, r1=r1, precision=precision,
                                    **self.schedule)
        self.ws = [torch.empty(cap, dtype=torch.uint8, device=dev) for _ in range(slots)]
        self.qbuf = [torch.empty((max_batch, queries.shape[1]), dtype=torch.float32, device=dev)
                     for _ in range(slots)]
        self.ids = [torch.empty(max_batch * max_k, dtype=torch.int64, device=dev)
                    for _ in range(slots)]
        self.sc = [torch.empty(max_batch * max_k, dtype=torch.float32, device=dev)
                   for _ in range(slots)]
        self.ev = [torch.cuda.Event() for _ in range(slots)]
        self.slot_bytes = cap

    def workspace_bytes(self, nq, k):
        return self.index.workspace_bytes(nq, k, self.c, self.r, r1=self.r1,
                                          precision=self.precision, **self.schedule)

    def launch(self, batch):
        torch = self.torch
        s = batch.slot
        rows = np.concatenate([q.rows for q in batch.reqs])
        nq = rows.shape[0]
        with torch.cuda.stream(self.streams[s]):
            idx = torch.from_numpy(rows).to(self.Q.device)
            q = self.qbuf[s][:nq]
            torch.index_select(self.Q, 0, idx, out=q)
            ids = self.ids[s][:nq * batch.k].view(nq, batch.k)
            sc = self.sc[s][:nq * batch.k].view(nq, batch.k)
            self.index.search(q, batch.k, self.c, self.r, r1=self.r1, precision=self.precision,
                              stream=self.streams[s], ws=self.ws[s], out=(ids, sc),
                              **self.schedule)
            self.ev[s].record(self.streams[s])
        batch.handle = (ids, sc)

    def poll(self, batch):
        return self.ev[batch.slot].query()

    def finish(self, batch):
        ids, sc = batch.handle
        ids, sc = ids.cpu().numpy(), sc.cpu().numpy()
        a = 0
        for q in batch.reqs:
            q.ids, q.scores = ids[a:a + q.nq], sc[a:a + q.nq]
            a += q.nq


class FakeExecutor:
    """CPU stand-in: a batch of nq queries completes `base + per_query * nq`
    seconds after launch (simulated clock); results are a deterministic
    function of each query row and k.  fail_batches: batch ids that fail."""

    def __init__(self, clock, base=1e-4, per_query=1e-6, ws_per_query=1000, fail_batches=()):
        self.clock, self.base, self.per_query = clock, base, per_query
        self.ws_per_query = ws_per_query
        self.fail = set(fail_batches)
        self.slot_bytes = None

    def workspace_bytes(self, nq, k):
        return self.ws_per_query * nq + 10 * k

    def launch(self, batch):
        if batch.bid in self.fail:
            raise RuntimeError(f"injected failure in batch {batch.bid}")
        nq = sum(q.nq for q in batch.reqs)
        batch.handle = self.clock() + self.base + self.per_query * nq

    def poll(self, batch):
        return self.clock() >= batch.handle

    def finish(self, batch):
        for q in batch.reqs:
            q.ids = (q.rows[:, None] * 7 + np.arange(q.k)[None, :]) % 1000003
            q.scores = -np.arange(q.k, dtype=np.float32)[None, :].repeat(q.nq, 0)


# ----------------------------------------------------------------- scheduler
class Scheduler:
    """Continuous batching with memory-based admission over `slots` slots.
    poll_interval: seconds slept between completion polls while batches are
    in flight; 0 polls without sleeping (an OS sleep lasts tens of
    microseconds at least, which light-load latency would otherwise pay)."""

    def __init__(self, executor, slots=4, mem_budget=None, max_batch=4096, clock=None,
                 sleep=None, poll_interval=2e-5):
        self.poll_interval = poll_interval
        self.ex = executor
        self.slots = slots
        self.mem_budget = mem_budget
        self.max_batch = max_batch
        self.clock = clock or time.perf_counter
        self.sleep = sleep or (lambda s: time.sleep(s))
        self.batches = []
        self.max_used = 0      # most workspace bytes in flight at once
        self.mem_limited = 0   # batch formations cut short by the memory budget

    def run(self, requests, t0=None):
        """Serve `requests` (arrival offsets in seconds, sorted); returns them."""
        reqs = sorted(requests, key=lambda q: q.arrival)
        t0 = self.clock() if t0 is None else t0
        nxt = 0
        pending = collections.deque()
        free = list(range(self.slots))
        inflight = []
        used = 0
        bid = 0
        done = 0
        while done < len(reqs):
            now = self.clock() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                q = reqs[nxt]
                nxt += 1
                need = self.ex.workspace_bytes(q.nq, q.k)
                if q.nq > self.max_batch or (self.mem_budget is not None and need > self.mem_budget):
                    q.status, q.done = "rejected", now
                    done += 1
                else:
                    q.status = "pending"
                    pending.append(q)
            # completions (any order)
            for b in list(inflight):
                if self.ex.poll(b):
                    inflight.remove(b)
                    self.ex.finish(b)
                    t = self.clock() - t0
                    for q in b.reqs:
                        q.status, q.done = "done", t
                    done += len(b.reqs)
                    used -= b.ws_bytes
                    free.append(b.slot)
            # form and launch batches while slots and memory allow
            while free and pending:
                k = pending[0].k
                take, nq = [], 0
                for q in pending:
                    if q.k != k:
                        continue
                    if nq + q.nq > self.max_batch:
                        break
                    ws = self.ex.workspace_bytes(nq + q.nq, k)
                    if self.mem_budget is not None and used + ws > self.mem_budget:
                        self.mem_limited += 1
                        break
                    if self.ex.slot_bytes is not None and ws > self.ex.slot_bytes:
                        break
                    take.append(q)
                    nq += q.nq
                if not take:
                    break
                for q in take:
                    pending.remove(q)
                ws = self.ex.workspace_bytes(nq, k)
                b = Batch(bid, free.pop(0), k, take, ws)
                bid += 1
                t = self.clock() - t0
                try:
                    self.ex.launch(b)
                except Exception as e:  # the batch fails, later ones still run
                    for q in take:
                        q.status, q.done, q.error = "failed", t, str(e)
                    done += len(take)
                    free.append(b.slot)
                    continue
                for q in take:
                    q.status, q.launch = "running", t
                used += ws
                self.max_used = max(self.max_used, used)
                inflight.append(b)
                self.batches.append(b)
            if done < len(reqs):
                # idle until the next arrival or the next poll of work in flight
                wait = reqs[nxt].arrival - (self.clock() - t0) if nxt < len(reqs) else 1.0
                if inflight:
                    wait = min(wait, self.poll_interval)
                if wait > 0:
                    self.sleep(min(wait, 1e-3))
        return reqs


def make_requests(rate_qps, n_queries, pool_rows, seed=4, ks=(10, 100), bmin=1, bmax=256):
    """Open-loop Poisson request stream over a pool of query rows."""
    g = np.random.default_rng(seed)
    lam = rate_qps / ((bmin + bmax) / 2.0)
    t, tot, rid, out = 0.0, 0, 0, []
    while tot < n_queries:
        t += g.exponential(1.0 / lam)
        b = int(g.integers(bmin, bmax + 1))
        rows = (np.arange(tot, tot + b) % pool_rows).astype(np.int64)
        out.append(Request(rid, t, rows, ks[int(g.integers(0, len(ks)))]))
        rid += 1
        tot += b
    return out


def latency_stats(reqs, warm_frac=0.1):
    """p50 / p99 request latency (ms) and achieved queries/s after warm-up."""
    done = [q for q in reqs if q.status == "done"]
    done = done[int(len(done) * warm_frac):]
    if not done:
        return dict(p50_ms=None, p99_ms=None, qps=0.0, requests=0)
    lat = np.array([q.done - q.arrival for q in done]) * 1e3
    span = max(q.done for q in done) - min(q.arrival for q in done)
    nq = sum(q.nq for q in done)
    return dict(p50_ms=round(float(np.percentile(lat, 50)), 3),
                p99_ms=round(float(np.percentile(lat, 99)), 3),
                qps=round(nq / span, 1), requests=len(done))


# ----------------------------------------------------------------- benchmark
def run_plain(ex, reqs, clock=time.perf_counter, sleep=time.sleep):
    """Baseline: every request searched alone, in arrival order, on one stream,
    each waited for before the next starts (no batching, no overlap)."""
    t0 = clock()
    for i, q in enumerate(reqs):
        now = clock() - t0
        if q.arrival > now:
            sleep(q.arrival - now)
        b = Batch(i, 0, q.k, [q], 0)
        q.launch = clock() - t0
        ex.launch(b)
        while not ex.poll(b):
            pass
        ex.finish(b)
        q.status, q.done = "done", clock() - t0
    return reqs


def fresh(reqs):
    return [Request(q.rid, q.arrival, q.rows, q.k) for q in reqs]


def bench_main(args, exact_topk, recall_at):
    """Serving benchmark: N=21,000,000 d=768 (bf16 copy + fp32 master), 8,192
    clusters (the generator's components), m=8; Poisson arrivals at 5k-1M
    queries/s, request size U[1, 256], k in {10, 100}.  The same continuous-
    batching scheduler (4 streams, a memory budget of two full-size batches'
    workspaces) runs the precision form (bf16 windows, certified shortlist,
    fp32 rerank) and the plain fp32 search; one request at a time on one
    stream is reported as a third reference at the lowest and highest rate.
    Per-result score errors against FP64 are reported as percentiles."""
    import json
    import sys

    import torch

    from . import datagen, lider

    def log(*a):
        print("[serving]", *a, file=sys.stderr, flush=True)

    n = int(getattr(args, "serve_n", 0) or 21_000_000)
    d, C, m, w, F = 768, 8192, 8, 2.0, 64
    t0 = time.time()
    X, lab = datagen.mixture(n, d, ncomp=C, seed=20, device="cuda")
    pool = 200_000
    Q, _ = datagen.queries_from(X, pool, 0.1, seed=21)
    A, b = datagen.lsh_params(m, d, w, seed=22)
    torch.cuda.synchronize()
    log(f"data {n}x{d} in {time.time() - t0:.1f}s")
    t0 = time.time()
    gi = lider.Index(X, C, m, w, F, (A, b), assignment=lab, storage="bf16",
                     centroid_storage="fp8")
    torch.cuda.synchronize()
    log(f"build {time.time() - t0:.1f}s, largest cluster {gi.max_cluster}")
    c, r, r1 = 1, int(gi.max_cluster), C
    sample = Q[:512].contiguous()
    gt_ids, gt_sc = exact_topk(torch, X, sample, 10, chunk=64)
    out = {"workload": f"gaussian-mixture N={n} d={d}, {C} clusters, m={m}; Poisson "
                       f"arrivals, request size U[1,256], k in {{10,100}}", "c": c, "r": r,
           "r1": r1}
    for prec in ("f32", "bf16"):
        ids, sc = gi.search(sample, 10, c, r, r1=r1, precision=prec)
        out[f"recall10_{prec}"] = round(recall_at(torch, X, sample, ids, gt_sc, 10), 4)
        # per-result error of the returned score against the FP64 inner product,
        # relative to |q| |x|
        rows = X[ids.clamp(min=0)].double()
        s64 = (rows * sample.double()[:, None, :]).sum(-1)
        rel = ((sc.double() - s64).abs() / (sample.double().norm(dim=1, keepdim=True)
                                            * rows.norm(dim=2)))[ids >= 0].cpu().numpy()
        out[f"score_err_{prec}"] = {f"p{p}": float(np.percentile(rel, p)) for p in (50, 90, 99)}
        out[f"score_err_{prec}"]["max"] = float(rel.max())
        del rows, s64
    del X, gt_ids, gt_sc
    torch.cuda.empty_cache()
    nq_total = int(getattr(args, "serve_queries", 0) or 110_000)
    # Small batches touch few of the index's row tiles: the executors pull
    # only the overlapped tiles from a device-built work list.
    sched = dict(persistent=2, grid_mult=4)
    out["schedule"] = sched
    exs = {p: GpuExecutor(gi, Q, c, r, r1, precision=p, slots=4, max_batch=4096, schedule=sched)
           for p in ("bf16", "f32")}
    budget = {p: 2 * e.workspace_bytes(4096, 100) for p, e in exs.items()}
    out["mem_budget_bytes"] = budget
    plain_ex = GpuExecutor(gi, Q, c, r, r1, precision="f32", slots=1, max_batch=256,
                           schedule=sched)
    for lam in (5_000, 10_000, 20_000, 50_000, 200_000, 1_000_000):
        reqs = make_requests(lam, nq_total, pool, seed=4)
        for p, ex in exs.items():
            t = time.time()
            sch = Scheduler(ex, slots=4, mem_budget=budget[p], max_batch=4096, poll_interval=0)
            res = sch.run(fresh(reqs))
            st = latency_stats(res)
            st.update(batches=len(sch.batches), max_inflight_bytes=sch.max_used,
                      memory_limited=sch.mem_limited)
            out[f"continuous_{p}_{lam}"] = st
            log(f"lambda={lam} continuous {p}, 4 streams: {st} ({time.time() - t:.1f}s)")
        if lam in (5_000, 1_000_000):
            t = time.time()
            res = run_plain(plain_ex, fresh(reqs))
            st = latency_stats(res)
            out[f"one_at_a_time_f32_{lam}"] = st
            log(f"lambda={lam} fp32, one request at a time: {st} ({time.time() - t:.1f}s)")
    print(json.dumps(out), flush=True)
