"""Pins for the oracle's local-moving phase (Alg. 2): sequential and synchronous sweeps."""
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


def _check_state(g, st):
    # Sigma' is the per-community sum of K', size the member count, labels valid
    sig = np.zeros(g.n, dtype=np.int64)
    np.add.at(sig, st.C, st.K)
    assert (sig == st.Sigma).all()
    assert (np.bincount(st.C, minlength=g.n) == st.size).all()
    assert int(st.Sigma.sum()) == st.W


@pytest.mark.parametrize("seed", range(10))
def test_seq_sweep_gain_is_exact_modularity_change(seed):
    # each sequential move's N is its exact gain, so a sweep changes Q by exactly 2*sumN/W^2
    rng = np.random.default_rng(seed)
    csr = graphgen.rmat(8, 6, seed=seed, wmax=3) if seed % 2 else None
    if csr is None:
        edges, w = random_graph(rng, 40, 0.12, wmax=4, self_loops=True)
        csr = graphgen.from_edges(40, edges, w)
    g = _og(csr)
    st = oracle.MoveState.fresh(g)
    for _ in range(12):
        q0 = _exact(g, st.C)
        tr = oracle.move(g, st, "seq", tau=-1.0, max_iter=1)
        assert _exact(g, st.C) - q0 == Fraction(2 * tr.sumN[0], st.W * st.W)
        _check_state(g, st)


@pytest.mark.parametrize("seed", range(8))
def test_seq_converges_to_local_optimum(seed):
    # with tau = 0 and no sweep cap the sequential phase stops only when no single move
    # has a positive gain (brute force over every vertex and neighbour community)
    rng = np.random.default_rng(50 + seed)
    n = int(rng.integers(5, 30))
    edges, w = random_graph(rng, n, 0.25, wmax=5, self_loops=True)
    if not edges:
        return
    g = _og(graphgen.from_edges(n, edges, w))
    A = entries(g)
    st = oracle.MoveState.fresh(g)
    tr = oracle.move(g, st, "seq", tau=0.0, max_iter=10000, prune=bool(seed % 2))
    assert tr.sumN[-1] == 0
    base = q_pairwise(n, A, st.C)
    for i in range(n):
        for c in set(st.C[[j for (a, j) in A if a == i and j != i]].tolist()):
            C2 = st.C.copy()
            C2[i] = c
            assert q_pairwise(n, A, C2) <= base


def test_seq_path_trace():
    # hand trace on the path 0-1-2-3 (W = 6): sweep 1 moves 0->1 (N=4) and 2->3 (N=4);
    # sweep 2 processes only vertex 1 and stays
    g = _og(graphgen.from_edges(4, [(0, 1), (1, 2), (2, 3)]))
    st = oracle.MoveState.fresh(g)
    tr = oracle.move(g, st, "seq", tau=0.01, max_iter=20)
    assert tr.iterations == 2
    assert tr.sumN == [8, 0]
    assert tr.moves == [2, 0]
    assert tr.processed == [4, 1]
    assert st.C.tolist() == [1, 1, 3, 3]


def test_sync_path_trace():
    # hand trace of the synchronous sweep with every vertex processed (sample_bits = 0) on
    # the path 0-1-2 (K = 1,2,1, W = 4): sweep 1 decides against the start state -- 0 is
    # blocked by the min-label rule, 1 joins 0 (tie 0/2 -> lowest), 2 joins 1's old label;
    # sweep 2 moves 2 into 0; sweep 3 moves nothing
    g = _og(graphgen.from_edges(3, [(0, 1), (1, 2)]))
    st = oracle.MoveState.fresh(g)
    tr = oracle.move(g, st, "sync", tau=0.01, max_iter=20, sample_bits=0)
    assert tr.iterations == 3
    assert tr.sumN == [4, 1, 0]
    assert tr.moves == [2, 1, 0]
    assert tr.processed == [3, 3, 1]
    assert st.C.tolist() == [0, 0, 0]
    _check_state(g, st)


def test_sync_min_label_singletons():
    # K_s from singletons: every vertex but 0 joins community 0 in sweep 1, 0 stays
    s = 6
    g = _og(graphgen.cliques(1, s))
    st = oracle.MoveState.fresh(g)
    tr = oracle.move(g, st, "sync", tau=0.01, max_iter=1, sample_bits=0)
    assert st.C.tolist() == [0] * s
    assert tr.moves == [s - 1]
    # two mutually-best singletons: only the higher id moves
    g2 = _og(graphgen.from_edges(2, [(0, 1)]))
    st2 = oracle.MoveState.fresh(g2)
    tr2 = oracle.move(g2, st2, "sync", tau=0.01, max_iter=20, sample_bits=0)
    assert st2.C.tolist() == [0, 0]
    assert tr2.moves == [1, 0]


def _round(seed, p, l, i, bits):
    # the synchronous iteration's round, computed with the generator module's SplitMix64
    ctr = (p << 40) | ((l & 0xFF) << 32) | i
    return graphgen.splitmix_draw(seed, ctr) >> (64 - bits)


@pytest.mark.parametrize("bits,seed", [(1, 0), (1, 99), (2, 5)])
def test_sync_rounds_partition_the_active_set(bits, seed):
    # every active vertex is processed once per iteration; on K_s the round-0 vertices
    # decide against all-singletons, so each of them other than 0 joins label 0
    s = 40
    g = _og(graphgen.cliques(1, s))
    st = oracle.MoveState.fresh(g)
    tr = oracle.move(g, st, "sync", tau=-1.0, max_iter=1, seed=seed, pass_index=3,
                     sample_bits=bits)
    assert tr.processed == [s]
    first = [i for i in range(s) if _round(seed, 3, 0, i, bits) == 0]
    assert len(first) > 1
    for i in first:
        assert st.C[i] == 0
    _check_state(g, st)


def test_sync_rounds_see_earlier_rounds():
    # single edge 0-1 with one vertex per round: whichever round comes first moves its
    # vertex only if the min-label rule allows it, and the second round then sees the move
    g = _og(graphgen.from_edges(2, [(0, 1)]))
    for seed in range(8):
        r0, r1 = _round(seed, 0, 0, 0, 1), _round(seed, 0, 0, 1, 1)
        st = oracle.MoveState.fresh(g)
        tr = oracle.move(g, st, "sync", tau=0.01, max_iter=20, seed=seed, sample_bits=1)
        assert st.C.tolist() == [0, 0]
        # 1 joins 0 in whichever round it runs; 0 never moves (blocked, then already joined)
        assert tr.moves[0] == 1
        assert r0 in (0, 1) and r1 in (0, 1)


@pytest.mark.parametrize("seed", range(6))
def test_sync_state_invariants(seed):
    g = _og(graphgen.rmat(9, 8, seed=seed))
    st = oracle.MoveState.fresh(g)
    tr = oracle.move(g, st, "sync", tau=0.0, max_iter=30, seed=seed)
    _check_state(g, st)
    assert all(x >= 0 for x in tr.sumN)
    assert tr.moves[0] > 0


def test_no_prune_processes_every_vertex():
    g = _og(graphgen.rmat(8, 4, seed=1))
    st = oracle.MoveState.fresh(g)
    tr = oracle.move(g, st, "seq", tau=0.0, max_iter=5, prune=False)
    assert all(p == g.n for p in tr.processed)
