"""Serving scheduler on the CPU with a fake executor and a simulated clock:
continuous batching, memory admission, rejection, injected failures,
out-of-order completion, latency accounting."""
import numpy as np

from paper_2205_00970_amd import serving


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-7)


def _sched(clock, **kw):
    ex_kw = {k: kw.pop(k) for k in list(kw) if k in ("base", "per_query", "ws_per_query",
                                                        "fail_batches")}
    ex = serving.FakeExecutor(clock, **ex_kw)
    return serving.Scheduler(ex, clock=clock, sleep=clock.sleep, **kw), ex


def test_all_requests_complete_with_correct_results():
    clock = SimClock()
    sch, ex = _sched(clock, slots=3, max_batch=512)
    reqs = serving.make_requests(20000, 5000, pool_rows=100000, seed=1)
    out = sch.run(reqs, t0=0.0)
    assert all(q.status == "done" for q in out)
    for q in out:
        ref = (q.rows[:, None] * 7 + np.arange(q.k)[None, :]) % 1000003
        assert np.array_equal(q.ids, ref)
        assert q.done >= q.arrival and q.launch >= q.arrival
    # batches are homogeneous in k and within the size cap
    for b in sch.batches:
        assert len({q.k for q in b.reqs}) == 1
        assert sum(q.nq for q in b.reqs) <= 512


def test_continuous_batching_merges_requests_under_load():
    clock = SimClock()
    sch, ex = _sched(clock, slots=1, max_batch=4096, base=5e-3, per_query=1e-6)
    reqs = serving.make_requests(50000, 20000, pool_rows=100000, seed=2)
    sch.run(reqs, t0=0.0)
    sizes = [len(b.reqs) for b in sch.batches]
    assert max(sizes) > 5  # requests that arrive while a batch runs are merged
    assert sum(sizes) == len(reqs)


def test_memory_admission_limits_batches_and_rejects_oversized():
    clock = SimClock()
    sch, ex = _sched(clock, slots=4, mem_budget=600_000, ws_per_query=1000, max_batch=4096,
                     base=2e-3)
    reqs = serving.make_requests(50000, 8000, pool_rows=100000, seed=3, bmax=256)
    big = serving.Request(10**6, 0.0005, np.arange(700), 10)  # needs 701,000 bytes > budget
    out = sch.run(reqs + [big], t0=0.0)
    assert big.status == "rejected"
    assert all(q.status == "done" for q in out if q is not big)
    assert all(b.ws_bytes <= 600_000 for b in sch.batches)
    # memory in flight never exceeded the budget: replay launch / completion times
    events = sorted([(b.reqs[0].launch, b.ws_bytes) for b in sch.batches] +
                    [(b.reqs[0].done, -b.ws_bytes) for b in sch.batches],
                    key=lambda e: (e[0], e[1]))
    used = 0
    for _, dlt in events:
        used += dlt
        assert used <= 600_000


def test_injected_failure_fails_one_batch_only():
    clock = SimClock()
    sch, ex = _sched(clock, slots=2, fail_batches=(3,))
    reqs = serving.make_requests(10000, 4000, pool_rows=100000, seed=5)
    out = sch.run(reqs, t0=0.0)
    failed = [q for q in out if q.status == "failed"]
    assert failed and all("injected" in q.error for q in failed)
    assert len({id(b) for b in sch.batches}) == len(sch.batches)
    assert all(q.status == "done" for q in out if q.status != "failed")
    assert any(q.arrival > max(f.arrival for f in failed) and q.status == "done" for q in out)


def test_out_of_order_completion():
    clock = SimClock()
    ex = serving.FakeExecutor(clock, base=1e-4, per_query=1e-4)
    sch = serving.Scheduler(ex, slots=2, max_batch=4096, clock=clock, sleep=clock.sleep)
    big = serving.Request(0, 0.0, np.arange(200), 10)    # long batch
    small = serving.Request(1, 1e-6, np.arange(2), 100)  # short batch, other k
    sch.run([big, small], t0=0.0)
    assert small.done < big.done


def test_latency_stats():
    reqs = [serving.Request(i, i * 0.001, np.arange(10), 10) for i in range(100)]
    for i, q in enumerate(reqs):
        q.status, q.done = "done", q.arrival + (0.002 if i < 99 else 0.05)
    st = serving.latency_stats(reqs, warm_frac=0.0)
    assert abs(st["p50_ms"] - 2.0) < 1e-6 and st["p99_ms"] > 2.0 and st["requests"] == 100
