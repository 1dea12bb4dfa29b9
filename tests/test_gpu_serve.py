"""Serving on the GPU: jobs that arrive while others run are batched into union runs
on several streams; each job's result equals the same graph run alone (deterministic
mode, bit for bit)."""
import random
import threading
import time

import numpy as np
import pytest

import graphgen
from gpu_util import to_device

pytestmark = pytest.mark.gpu


def test_each_job_is_the_same_alone_and_in_the_mix():
    import paper_2312_04876_amd as P
    from paper_2312_04876_amd.serve import GpuExecutor, Job, Server, latency_stats
    pool = {k: g for k, g in enumerate(graphgen.serving_pool(12, seed=5, median=2e4, cap=3e5))}
    alone = {}
    for k, g in pool.items():
        m, q, _ = P.louvain(*to_device(g), mode="deterministic")
        alone[k] = (m.cpu().numpy()[:g.n], q)
    ex = GpuExecutor(pool, slots=3, mode="deterministic")
    srv = Server(ex, memory_budget=8 << 30, slots=3)
    rng = random.Random(7)
    jobs = []

    def feed():
        for _ in range(36):
            k = rng.randrange(len(pool))
            jobs.append(srv.submit(Job(key=k, nnz=pool[k].nnz, n=pool[k].n)))
            time.sleep(rng.random() * 0.01)

    t = threading.Thread(target=feed)
    t.start()
    t.join()
    assert srv.drain(timeout=300)
    srv.close()
    print("batches", srv.batches, latency_stats(jobs), flush=True)
    assert srv.batches > 1
    for j in jobs:
        assert j.error is None, j.error
        m, q = alone[j.key]
        assert np.array_equal(j.membership, m), j.key
        assert j.modularity == q, j.key
