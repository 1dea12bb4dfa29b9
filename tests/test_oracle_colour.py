"""Pins for the oracle's colouring and its colour-ordered iteration (the vertex
colouring alternative of Section 2: neighbours never decide in the same round)."""
import numpy as np
import pytest

import graphgen
import oracle
from refs import random_graph


def _og(csr):
    return oracle.as_graph(csr.offsets, csr.targets, csr.weights)


def _priority(seed, p, v):
    # SplitMix64 output for counter 1 << 63 | p << 40 | v under key seed (the
    # seeded-input module's own implementation of the published generator)
    return graphgen.splitmix_draw(seed, (1 << 63) | (p << 40) | v)


def _greedy(g, seed, p):
    # brute force: visit vertices by decreasing priority, take the smallest colour
    # no earlier neighbour holds
    order = sorted(range(g.n), key=lambda v: -_priority(seed, p, v))
    col = [-1] * g.n
    for v in order:
        taken = {col[int(u)] for u in g.targets[g.offsets[v]:g.offsets[v + 1]] if int(u) != v}
        c = 0
        while c in taken:
            c += 1
        col[v] = c
    return np.array(col, dtype=np.int32)


@pytest.mark.parametrize("seed", range(8))
def test_colouring_is_the_greedy_colouring_in_priority_order(seed):
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(1, 40))
    g = _og(graphgen.from_edges(n, *random_graph(rng, n, float(rng.uniform(0.05, 0.6)))))
    col, k = oracle.colour(g, seed=seed * 977, pass_index=seed % 3)
    assert np.array_equal(col, _greedy(g, seed * 977, seed % 3))
    assert k == int(col.max()) + 1


@pytest.mark.parametrize("seed", range(4))
def test_colouring_is_proper_and_greedy_minimal(seed):
    g = _og(graphgen.rmat(11, 8, seed=50 + seed))
    col, k = oracle.colour(g, seed=seed, pass_index=1)
    src = np.repeat(np.arange(g.n), np.diff(g.offsets))
    loop = src == g.targets
    assert not (col[src] == col[g.targets])[~loop].any()
    pr = np.array([_priority(seed, 1, v) for v in range(g.n)], dtype=np.uint64)
    for v in range(g.n):
        nb = g.targets[g.offsets[v]:g.offsets[v + 1]]
        nb = nb[nb != v]
        earlier = set(col[nb[pr[nb] > pr[v]]].tolist())
        assert set(range(col[v])) <= earlier and col[v] not in earlier
    # at most max degree + 1 colours
    deg = np.diff(g.offsets) - np.bincount(src[loop], minlength=g.n)
    assert k <= int(deg.max()) + 1


def test_colouring_special_cases():
    empty = oracle.as_graph(np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32),
                            np.zeros(0, dtype=np.int64))
    assert oracle.colour(empty)[1] == 0
    iso = _og(graphgen.from_edges(5, [(1, 1), (3, 3)]))
    col, k = oracle.colour(iso)
    assert k == 1 and (col == 0).all()
    kn = _og(graphgen.cliques(1, 7))
    col, k = oracle.colour(kn, seed=3)
    # a clique: the colours are the ranks in decreasing priority
    order = sorted(range(7), key=lambda v: -_priority(3, 0, v))
    assert k == 7 and [int(col[v]) for v in order] == list(range(7))


def test_coloured_rounds_on_disjoint_pairs():
    # each pair's higher-priority end (colour 0) joins its partner's singleton in
    # round 0; the partner then has nothing better, so the pair carries its label
    n = 40
    g = _og(graphgen.from_edges(n, [(2 * q, 2 * q + 1) for q in range(n // 2)]))
    col, _ = oracle.colour(g, seed=11)
    st = oracle.MoveState.fresh(g)
    tr = oracle.move(g, st, mode="colour", tau=0.0, max_iter=5, prune=False, seed=11)
    for q in range(n // 2):
        u, v = 2 * q, 2 * q + 1
        low = v if col[u] == 0 else u
        assert st.C[u] == st.C[v] == low
    assert tr.moves[0] == n // 2 and tr.moves[1] == 0


def _seed_with_id_order(n, passes=1):
    # a key whose priorities fall with the vertex id in every pass of the run
    for s in range(1, 200000):
        if all(all(_priority(s, p, v) > _priority(s, p, v + 1) for v in range(n - 1))
               for p in range(passes)):
            return s
    raise AssertionError("no key found")


@pytest.mark.parametrize("case", range(3))
def test_coloured_rounds_on_a_clique_are_the_sequential_sweep(case):
    # on a clique every colour class is one vertex; with priorities falling with the
    # id, class r is vertex r, so the rounds replay the ascending sequential sweep
    n = 6
    seed = _seed_with_id_order(n)
    rng = np.random.default_rng(900 + case)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n)]
    w = rng.integers(1, 9, size=len(edges)).tolist()
    g = _og(graphgen.from_edges(n, edges, w))
    col, k = oracle.colour(g, seed=seed)
    assert col.tolist() == list(range(n)) and k == n
    a, b = oracle.MoveState.fresh(g), oracle.MoveState.fresh(g)
    ta = oracle.move(g, a, mode="colour", tau=0.0, max_iter=10, prune=False, seed=seed)
    tb = oracle.move(g, b, mode="seq", tau=0.0, max_iter=10, prune=False)
    assert np.array_equal(a.C, b.C) and np.array_equal(a.Sigma, b.Sigma)
    assert ta.iterations == tb.iterations and ta.sumN == tb.sumN and ta.moves == tb.moves


@pytest.mark.parametrize("seed", range(4))
def test_coloured_run_state_and_quality(seed):
    g = _og(graphgen.sbm(3000, 8, 0.04, 0.002, seed=60 + seed))
    st = oracle.MoveState.fresh(g)
    oracle.move(g, st, mode="colour", seed=seed)
    sig = np.zeros(g.n, dtype=np.int64)
    np.add.at(sig, st.C, st.K)
    assert (st.Sigma == sig).all() and (st.size == np.bincount(st.C, minlength=g.n)).all()
    mc, qc, rc = oracle.louvain(g, oracle.Params(mode="colour", seed=seed))
    # eight dense blocks with sparse links between them: the planted partition is
    # what a good run finds
    planted = oracle.modularity(g, graphgen.sbm_blocks(3000, 8))
    assert qc == oracle.modularity(g, mc) and qc > planted - 0.002
    # the pass loop in C and the Python driver over single steps agree
    mt, qt, _ = oracle.louvain_trace(g, oracle.Params(mode="colour", seed=seed))
    assert np.array_equal(mt, mc) and qt == qc
