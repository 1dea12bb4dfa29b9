"""Pins for the oracle's warm start (a first pass that starts from a given partition,
the dynamic re-run the paper names as future work)."""
from fractions import Fraction

import numpy as np
import pytest

import graphgen
import oracle
from refs import entries, q_pairwise, random_graph


def _og(csr):
    return oracle.as_graph(csr.offsets, csr.targets, csr.weights)


def _exact(g, C):
    num, den = oracle.modularity_exact(g, C)
    return Fraction(0) if den == 0 else Fraction(num, den)


@pytest.mark.parametrize("mode", ["seq", "sync"])
def test_warm_start_from_singletons_is_the_cold_run(mode):
    g = _og(graphgen.rmat(10, 8, seed=31))
    m0, q0, r0 = oracle.louvain(g, oracle.Params(mode=mode))
    m1, q1, r1 = oracle.louvain(g, oracle.Params(mode=mode), initial=np.arange(g.n))
    assert np.array_equal(m0, m1) and q0 == q1 and r0 == r1


def test_warm_state_holds_the_partitions_totals():
    g = _og(graphgen.sbm(200, 5, 0.2, 0.01, seed=32))
    labels = (np.arange(g.n) * 7) % 13
    st = oracle.MoveState.warm(g, labels)
    sig = np.zeros(g.n, dtype=np.int64)
    np.add.at(sig, labels, st.K)
    assert (st.Sigma == sig).all() and (st.size == np.bincount(labels, minlength=g.n)).all()
    assert int(st.Sigma.sum()) == st.W
    with pytest.raises(ValueError):
        oracle.MoveState.warm(g, np.full(g.n, g.n))


@pytest.mark.parametrize("seed", range(6))
def test_warm_sequential_run_never_lowers_q(seed):
    # sequential moves all have positive exact gain and aggregation keeps Q, so the
    # final Q is at least the Q of the starting partition
    rng = np.random.default_rng(300 + seed)
    g = _og(graphgen.rmat(9, 8, seed=40 + seed, wmax=3))
    start = rng.integers(0, max(g.n // 8, 1), size=g.n)
    memb, q, _ = oracle.louvain(g, oracle.Params(mode="seq"), initial=start)
    assert _exact(g, memb) >= _exact(g, start)
    assert q == oracle.modularity(g, memb)


@pytest.mark.parametrize("seed", range(6))
def test_warm_first_pass_ends_in_a_local_optimum(seed):
    # with tau = 0 and no pruning, the first pass's moving from any start stops only
    # when no single move has a positive gain (brute force); pruning would skip
    # vertices whose community lost a member that is not their neighbour
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(6, 25))
    edges, w = random_graph(rng, n, 0.3, wmax=4, self_loops=True)
    if not edges:
        return
    g = _og(graphgen.from_edges(n, edges, w))
    A = entries(g)
    st = oracle.MoveState.warm(g, rng.integers(0, n, size=n))
    tr = oracle.move(g, st, "seq", tau=0.0, max_iter=10000, prune=False)
    assert tr.sumN[-1] == 0
    base = q_pairwise(n, A, st.C)
    for i in range(n):
        for c in set(st.C[[j for (a, j) in A if a == i and j != i]].tolist()):
            C2 = st.C.copy()
            C2[i] = c
            assert q_pairwise(n, A, C2) <= base


def test_warm_trace_matches_the_c_driver():
    g = _og(graphgen.sbm(600, 6, 0.1, 0.004, seed=33))
    start = (np.arange(g.n) // 50).astype(np.int32)
    for mode in ("seq", "sync"):
        prm = oracle.Params(mode=mode)
        m0, q0, recs = oracle.louvain_trace(g, prm, initial=start)
        m1, q1, r1 = oracle.louvain(g, prm, initial=start)
        assert np.array_equal(m0, m1) and q0 == q1
        assert [r.trace.iterations for r in recs] == r1["iterations"]
