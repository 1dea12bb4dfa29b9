"""The CPU-baseline build of the oracle (-O3 -march=native, OpenMP over the decisions of
a synchronous round) gives exactly the serial build's results: the timed baseline
computes what the parity oracle computes."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import heavy


def _og(csr):
    return oracle.as_graph(csr.offsets, csr.targets, csr.weights)


GRAPHS = {
    "sbm10k": lambda: graphgen.workload("sbm10k"),
    "rmat14-16": lambda: graphgen.workload("rmat14-16"),
    "rmat13-8-heavy": lambda: heavy(graphgen.rmat(13, 8, seed=43), 5),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("mode,bits", [("sync", 0), ("sync", 1), ("sync", 2), ("colour", 0)])
def test_timing_build_equals_serial_build(name, mode, bits):
    g = _og(GRAPHS[name]())
    fast = oracle.timing_library()
    prm = oracle.Params(mode=mode, sample_bits=bits, seed=3)
    m1, q1, r1 = oracle.louvain(g, prm)
    m2, q2, r2 = oracle.louvain(g, prm, lib=fast)
    assert np.array_equal(m1, m2) and q1 == q2 and r1 == r2
    # one local-moving phase: exact gain sums, moves and visits per sweep
    s1, s2 = oracle.MoveState.fresh(g), oracle.MoveState.fresh(g)
    t1 = oracle.move(g, s1, mode, 0.0, 6, True, 3, 0, bits)
    t2 = oracle.move(g, s2, mode, 0.0, 6, True, 3, 0, bits, lib=fast)
    assert t1 == t2
    for a, b in ((s1.C, s2.C), (s1.Sigma, s2.Sigma), (s1.size, s2.size), (s1.active, s2.active)):
        assert np.array_equal(a, b)
