"""R-MAT scale 24 (2.0e9 entries, total weight past 2^31): parity checks at full size.

Fast mode: a valid partition whose reported modularity is the oracle's modularity of
that membership, bit for bit.  Deterministic mode: the first synchronous iteration
(one round, from singletons) checked vertex by vertex on a sample that includes the
hundred longest rows, each against the oracle on a local replica (tests/replica.py).
"""
import time

import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import is_valid_partition, to_device
from replica import first_iteration_decision

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rmat24():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    t0 = time.time()
    print("generating rmat24 ...", flush=True)
    csr = graphgen.workload("rmat24", threads=16)
    print("rmat24: n=%d nnz=%d in %.0f s" % (csr.n, csr.nnz, time.time() - t0), flush=True)
    g = oracle.as_graph(csr.offsets, csr.targets, csr.weights)
    K, W = oracle.vertex_weights(g)
    print("oracle graph and weights ready, W=%d" % W, flush=True)
    return csr, g, K, W


def test_rmat24_fast_full_size(rmat24):
    import paper_2312_04876_amd as P
    csr, g, K, W = rmat24
    off, tgt, w = to_device(csr)
    memb, q, st = P.louvain(off, tgt, w, mode="fast")
    memb = memb.cpu().numpy()
    del off, tgt, w
    print("rmat24 fast: Q=%.6f passes=%d" % (q, st["passes"]), flush=True)
    assert is_valid_partition(memb)
    assert q == oracle.modularity(g, memb)


def test_rmat24_det_first_iteration_sampled(rmat24):
    import paper_2312_04876_amd as P
    csr, g, K, W = rmat24
    off, tgt, w = to_device(csr)
    ctx = P.Louvain(off, tgt, w, mode="deterministic", round_bits=0, max_iterations=1,
                    max_passes=1)
    try:
        ctx.move()
        labels = ctx.level_labels().cpu().numpy()
    finally:
        ctx.close()
    del off, tgt, w
    deg = np.diff(g.offsets)
    rng = np.random.default_rng(24)
    live = np.nonzero(deg > 0)[0]
    sample = np.unique(np.concatenate((rng.choice(live, size=900, replace=False),
                                       np.argsort(-deg)[:100])))
    t0 = time.time()
    for k, i in enumerate(sample):
        assert labels[i] == first_iteration_decision(g, K, W, int(i)), int(i)
        if k % 200 == 0:
            print("checked %d of %d vertices (%.0f s)" % (k, len(sample), time.time() - t0), flush=True)
