"""R-MAT scale 24 (2.0e9 entries, total weight past 2^31): parity at full size.

Deterministic mode, pass by pass against the oracle's synchronous run (records written
by tests/golden/make_golden.py --full rmat24, which calls only the oracle): iterations,
exact per-iteration gain sums, moves, vertex visits, a digest of the raw labels,
communities and an order-free digest of the aggregated level graph, then the
membership digest and Q.  Fast mode: a valid partition whose reported Q is the
oracle's Q of that membership bit for bit, within 0.01 of the oracle's sequential Q.
"""
import json
import os
import sys
import time

import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import is_valid_partition, to_device

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from digest import graph_digest, labels_digest  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "reference.json")


@pytest.fixture(scope="module")
def rmat24():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    ref = json.load(open(GOLDEN))["rmat24"]
    t0 = time.time()
    print("generating rmat24 ...", flush=True)
    csr = graphgen.workload("rmat24", threads=16)
    print("rmat24: n=%d nnz=%d in %.0f s" % (csr.n, csr.nnz, time.time() - t0), flush=True)
    assert (csr.n, csr.nnz, int(csr.weights.sum(dtype=np.int64))) == (ref["n"], ref["nnz"], ref["W"])
    dev = to_device(csr)
    iso0 = int((np.diff(csr.offsets) == 0).sum())
    return csr, dev, ref, iso0


def test_rmat24_det_pass_by_pass(rmat24):
    import paper_2312_04876_amd as P
    csr, (off, tgt, w), ref, iso0 = rmat24
    rec = ref["sync"]
    ctx = P.Louvain(off, tgt, w, mode="deterministic", seed=rec["seed"], round_bits=rec["round_bits"])
    iso = iso0
    try:
        for k, pr in enumerate(rec["per_pass"]):
            t0 = time.time()
            it, _ = ctx.move()
            tr = ctx.move_trace()
            print("pass %d: %d iterations (%.1f s)" % (k, it, time.time() - t0), flush=True)
            assert it == pr["iterations"], ("iterations", k)
            assert [str(x) for x in tr["sumN"]] == pr["sumN"], ("gain sums", k)
            assert tr["moves"] == pr["moves"], ("moves", k)
            # isolated vertices are never queued on the GPU; the oracle visits them in the
            # first iteration
            assert tr["processed"] == [p - (iso if j == 0 else 0)
                                       for j, p in enumerate(pr["processed"])], ("processed", k)
            assert labels_digest(ctx.level_labels().cpu().numpy()) == pr["labels"], ("labels", k)
            nc, stop = ctx.aggregate()
            assert nc == pr["communities"], ("communities", k)
            if "next_level" not in pr:
                assert stop
                break
            t0 = time.time()
            o, d, t, ww = ctx.level_graph()
            o, d, t, ww = o.cpu().numpy(), d.cpu().numpy(), t.cpu().numpy(), ww.cpu().numpy()
            dg = graph_digest(o[:-1], d, t, ww)
            print("level graph after pass %d: %d vertices, %d entries (%.1f s)" %
                  (k, dg["n"], dg["entries"], time.time() - t0), flush=True)
            assert dg == pr["next_level"], ("level graph", k)
            iso = int((d == 0).sum())
            del o, d, t, ww
        memb, q, st = ctx.run()
        memb = memb.cpu().numpy()
    finally:
        ctx.close()
    print("rmat24 deterministic: Q=%.6f (oracle %.6f)" % (q, rec["Q"]), flush=True)
    assert labels_digest(memb) == rec["digest"]
    assert q == rec["Q"]
    assert st["iterations"] == rec["iterations"] and st["communities"] == rec["communities"]


def test_rmat24_fast_full_size(rmat24):
    import paper_2312_04876_amd as P
    csr, (off, tgt, w), ref, _ = rmat24
    memb, q, st = P.louvain(off, tgt, w, mode="fast")
    memb = memb.cpu().numpy()
    print("rmat24 fast: Q=%.6f passes=%d, sequential oracle %.6f" % (q, st["passes"],
                                                                      ref["seq"]["Q"]), flush=True)
    assert is_valid_partition(memb)
    g = oracle.as_graph(csr.offsets, csr.targets, csr.weights)
    assert q == oracle.modularity(g, memb)
    assert abs(q - ref["seq"]["Q"]) <= 0.01
