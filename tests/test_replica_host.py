"""The local-replica decisions equal the oracle's own first synchronous iteration on
the whole graph (the reference the full-size GPU check samples)."""
import numpy as np
import pytest

import graphgen
import oracle
from replica import first_iteration_decision


@pytest.mark.parametrize("csr", [graphgen.rmat(11, 8, seed=61), graphgen.rmat(10, 8, wmax=9, seed=62),
                                 graphgen.sbm(1500, 15, 0.03, 0.002, seed=63)],
                         ids=["rmat11", "rmat10w", "sbm1500"])
def test_replica_decisions_equal_the_whole_graph_iteration(csr):
    g = oracle.as_graph(csr.offsets, csr.targets, csr.weights)
    K, W = oracle.vertex_weights(g)
    st = oracle.MoveState.fresh(g)
    oracle.move(g, st, mode="sync", tau=0.0, max_iter=1, prune=False, seed=0, pass_index=0,
                sample_bits=0)
    rng = np.random.default_rng(7)
    deg = np.diff(g.offsets)
    sample = np.concatenate((rng.choice(g.n, size=min(g.n, 300), replace=False), np.argsort(-deg)[:20]))
    for i in sample:
        assert first_iteration_decision(g, K, W, int(i)) == int(st.C[i]), int(i)
