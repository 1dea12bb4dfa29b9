"""Pins for the oracle's whole pass loop (Alg. 1)."""
from fractions import Fraction

import numpy as np
import pytest

import graphgen
import oracle
from refs import entries, q_optimum, random_graph


def _og(csr):
    return oracle.as_graph(csr.offsets, csr.targets, csr.weights)


def _exact(g, C):
    num, den = oracle.modularity_exact(g, C)
    return Fraction(0) if den == 0 else Fraction(num, den)


MODES = ["seq", "sync"]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("k,s", [(2, 3), (4, 4), (8, 5), (16, 3), (3, 12)])
def test_disjoint_cliques_reach_closed_form(mode, k, s):
    # k equal disjoint cliques: Louvain finds them and Q = (k-1)/k
    g = _og(graphgen.cliques(k, s))
    memb, q, _ = oracle.louvain(g, oracle.Params(mode=mode))
    assert q == (k - 1) / k
    assert (memb == np.arange(k * s) // s).all()


def test_path_p4_trace():
    # two K_2 joined by one edge: W = 6, Q = 2[2/6 - (3/6)^2] = 1/6 (sequential mode)
    g = _og(graphgen.from_edges(4, [(0, 1), (1, 2), (2, 3)]))
    memb, q, rec = oracle.louvain(g, oracle.Params(mode="seq"))
    assert memb.tolist() == [0, 0, 1, 1]
    assert _exact(g, memb) == Fraction(1, 6)
    assert q == 1 / 6
    assert rec["iterations"] == [2, 1]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", range(10))
def test_never_beats_exhaustive_optimum(mode, seed):
    # a heuristic cannot exceed the best partition (exhaustive search, n <= 9)
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(3, 10))
    edges, w = random_graph(rng, n, 0.35, wmax=4, self_loops=bool(seed % 3 == 0))
    if not edges:
        return
    g = _og(graphgen.from_edges(n, edges, w))
    memb, q, _ = oracle.louvain(g, oracle.Params(mode=mode))
    opt = q_optimum(n, entries(g))
    assert _exact(g, memb) <= opt


def test_reaches_optimum_on_curated_graphs():
    # cases traced by hand where the optimum is reached
    cases = [
        graphgen.cliques(2, 4, bridges=[(3, 4)]),
        graphgen.cliques(3, 3, bridges=[(2, 3), (5, 6)]),
        graphgen.cliques(2, 5),
    ]
    for csr in cases:
        g = _og(csr)
        memb, _, _ = oracle.louvain(g, oracle.Params(mode="seq"))
        assert _exact(g, memb) == q_optimum(g.n, entries(g))


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("wl", ["sbm10k", "rmat12-8", "rmat13-16"])
def test_c_loop_matches_step_loop(mode, wl):
    # the C pass loop and the Python pass loop over the C steps agree exactly
    g = _og(graphgen.workload(wl))
    m1, q1, rec = oracle.louvain(g, oracle.Params(mode=mode))
    m2, q2, recs = oracle.louvain_trace(g, oracle.Params(mode=mode))
    assert (m1 == m2).all() and q1 == q2
    assert rec["iterations"] == [r.trace.iterations for r in recs]


@pytest.mark.parametrize("mode", MODES)
def test_dendrogram_lookup_keeps_modularity(mode):
    # after every pass, Q(G, top membership) == Q(G'', singletons)
    g = _og(graphgen.workload("sbm10k"))
    _, _, recs = oracle.louvain_trace(g, oracle.Params(mode=mode))
    seen = 0
    for r in recs:
        if r.next_level is not None:
            assert oracle.modularity_exact(g, oracle.renumber(r.top)[0]) == \
                oracle.modularity_exact(r.next_level, np.arange(r.next_level.n, dtype=np.int32))
            seen += 1
    assert seen >= 2


def test_edge_cases():
    # empty graph, isolated vertices, a lone self-loop
    for csr in [graphgen.from_edges(0, []), graphgen.from_edges(1, []),
                graphgen.from_edges(5, []), graphgen.from_edges(3, [(1, 1)], [4])]:
        g = _og(csr)
        for mode in MODES:
            memb, q, rec = oracle.louvain(g, oracle.Params(mode=mode))
            assert memb.tolist() == list(range(g.n))
            assert q == 0.0
            assert rec["passes"] == (1 if g.n >= 0 else 0)


def test_max_passes_limits():
    g = _og(graphgen.workload("sbm10k"))
    for mp in [0, 1, 2]:
        memb, q, rec = oracle.louvain(g, oracle.Params(mode="seq", max_passes=mp))
        assert rec["passes"] == mp
        assert 0 <= memb.min() and memb.max() < g.n
        assert q == oracle.modularity(g, memb)


def test_sbm_recovers_planted_quality():
    # a well-separated planted partition: Louvain reaches at least the planted Q minus a
    # small margin in sequential mode
    g = _og(graphgen.workload("sbm10k"))
    planted = oracle.modularity(g, graphgen.sbm_blocks(10000, 100))
    _, q, _ = oracle.louvain(g, oracle.Params(mode="seq"))
    assert q > planted - 0.1


@pytest.mark.parametrize("wl", ["sbm10k", "rmat12-8"])
@pytest.mark.parametrize("mp", [1, 2, 3])
@pytest.mark.parametrize("mode", ["seq", "sync"])
def test_pass_limit_lookup_applies_each_pass_once(wl, mp, mode):
    # Alg. 1 when the pass loop runs out of passes (the final lookup runs only when the
    # loop ends early): the membership is the composition of each pass's renumbered
    # labels, applied once per pass.  The
    # composition is rebuilt here from single steps (one local-moving phase per level,
    # numpy's dense renumbering, the aggregated level) and must equal the C pass loop's
    # result; Q(G, membership) must equal the modularity of the last aggregated level
    # under singletons.
    g = _og(graphgen.workload(wl))
    # R-MAT levels shrink by less than the 0.8 test after two passes; an aggregation
    # tolerance of 1 keeps its loop going so that the pass limit is what ends it
    prm = oracle.Params(mode=mode, max_passes=mp,
                        aggregation_tolerance=1.0 if wl.startswith("rmat") else 0.8)
    memb, q, rec = oracle.louvain(g, prm)
    assert rec["passes"] == mp
    top = np.arange(g.n)
    level, tau = g, prm.tolerance
    for p in range(mp):
        st = oracle.MoveState.fresh(level)
        tr = oracle.move(level, st, mode, tau, prm.max_iterations, prm.prune, prm.seed, p,
                         prm.sample_bits)
        nc = len(np.unique(st.C))
        # the loop runs on: no pass stops by convergence or by too few merges
        assert tr.iterations > 1 and nc / level.n <= prm.aggregation_tolerance, (wl, p)
        dense = np.unique(st.C, return_inverse=True)[1].astype(np.int32)
        top = dense[top]
        level = oracle.aggregate(level, dense, nc)
        tau = tau / prm.tolerance_drop
    assert np.array_equal(memb, top)
    assert q == oracle.modularity(level, np.arange(level.n, dtype=np.int32))
    assert q == oracle.modularity(g, top)
    # the membership pin fails for a double lookup of the last pass's labels (renumbered
    # as the loop's result is); Q alone may not see it, since merging communities of
    # isolated vertices (Sigma 0) leaves Q unchanged
    twice = np.unique(dense[top], return_inverse=True)[1]
    assert not np.array_equal(memb, twice)
