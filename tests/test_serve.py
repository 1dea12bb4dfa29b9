"""The continuous-batching scheduler, driven on the CPU by executors that stand in for
the GPU (no kernels): admission by memory footprint, overlap of batches on several
slots, admission of later arrivals while batches run, and per-job results."""
import threading
import time

import numpy as np
import pytest

import graphgen
import oracle
from paper_2312_04876_amd.serve import Job, Server, latency_stats


class OracleExecutor:
    """Runs each job of a batch with the oracle (sync mode) and records the memory in use."""

    def __init__(self, pool, delay=0.0):
        self.pool = pool
        self.delay = delay
        self.lock = threading.Lock()
        self.running = 0
        self.in_use = 0
        self.peak_in_use = 0
        self.max_running = 0
        self.spans = []

    def footprint(self, job):
        return 100 + 10 * job.n + 20 * job.nnz

    def run(self, jobs, slot):
        mem = sum(self.footprint(j) for j in jobs)
        with self.lock:
            self.running += 1
            self.in_use += mem
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            self.max_running = max(self.max_running, self.running)
        t0 = time.perf_counter()
        out = []
        for j in jobs:
            g = self.pool[j.key]
            memb, q, _ = oracle.louvain(oracle.as_graph(g.offsets, g.targets, g.weights),
                                        oracle.Params(mode="sync"))
            out.append((memb, q))
        time.sleep(self.delay)
        with self.lock:
            self.running -= 1
            self.in_use -= mem
            self.spans.append((t0, time.perf_counter(), slot, len(jobs)))
        return out


@pytest.fixture(scope="module")
def pool():
    return {k: graphgen.sbm(60 + 7 * k, 3 + k % 4, 0.3, 0.01, seed=100 + k, name="p%d" % k)
            for k in range(8)}


def job_of(pool, k):
    g = pool[k]
    return Job(key=k, nnz=g.nnz, n=g.n)


def test_every_job_gets_its_own_result(pool):
    ex = OracleExecutor(pool)
    srv = Server(ex, memory_budget=10 ** 9, slots=3)
    jobs = [srv.submit(job_of(pool, k % 8)) for k in range(40)]
    assert srv.drain(timeout=120)
    srv.close()
    for j in jobs:
        assert j.error is None and j.done.is_set()
        g = pool[j.key]
        memb, q, _ = oracle.louvain(oracle.as_graph(g.offsets, g.targets, g.weights),
                                    oracle.Params(mode="sync"))
        assert np.array_equal(j.membership, memb) and j.modularity == q
    st = latency_stats(jobs)
    assert st["count"] == 40 and st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]


def test_memory_budget_is_never_exceeded(pool):
    ex = OracleExecutor(pool, delay=0.02)
    budget = 3 * max(ex.footprint(job_of(pool, k)) for k in pool)
    srv = Server(ex, memory_budget=budget, slots=4)
    jobs = [srv.submit(job_of(pool, k % 8)) for k in range(30)]
    assert srv.drain(timeout=120)
    srv.close()
    assert all(j.error is None for j in jobs)
    assert ex.peak_in_use <= budget and srv.peak_memory <= budget
    assert srv.batches >= 6  # the budget forces small batches


def test_batches_overlap_and_later_arrivals_join(pool):
    ex = OracleExecutor(pool, delay=0.15)
    srv = Server(ex, memory_budget=10 ** 9, slots=2)
    first = [srv.submit(job_of(pool, k)) for k in range(3)]
    time.sleep(0.05)          # the first batch is running on one slot
    late = [srv.submit(job_of(pool, k)) for k in range(3, 6)]
    assert srv.drain(timeout=60)
    srv.close()
    assert ex.max_running == 2  # the late jobs ran beside the first batch
    assert max(j.admitted for j in late) < min(j.finished for j in first)
    assert {j.batch for j in first}.isdisjoint({j.batch for j in late})


def test_oversized_job_is_rejected_not_queued(pool):
    ex = OracleExecutor(pool)
    srv = Server(ex, memory_budget=50, slots=1)
    j = srv.submit(job_of(pool, 0))
    assert j.done.is_set() and j.error is not None
    assert srv.drain(timeout=10)
    srv.close()


def test_failed_batch_reports_errors_and_server_goes_on(pool):
    class Flaky(OracleExecutor):
        calls = 0

        def run(self, jobs, slot):
            Flaky.calls += 1
            if Flaky.calls == 1:
                raise RuntimeError("device lost")
            return super().run(jobs, slot)

    srv = Server(Flaky(pool), memory_budget=10 ** 9, slots=1, max_jobs=1)
    a = srv.submit(job_of(pool, 0))
    b = srv.submit(job_of(pool, 1))
    assert srv.drain(timeout=60)
    srv.close()
    assert a.error and "device lost" in a.error
    assert b.error is None and b.membership is not None
