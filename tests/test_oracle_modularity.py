"""Pins for the oracle's modularity (Eq. 1) and gain (Eq. 2) against independent definitions."""
from fractions import Fraction

import networkx as nx
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


@pytest.mark.parametrize("seed", range(12))
def test_modularity_matches_pairwise_definition(seed):
    # Eq. 1: the community-sum form equals the pairwise form exactly, self-loops included
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 14))
    edges, w = random_graph(rng, n, 0.35, wmax=7, self_loops=True)
    g = _og(graphgen.from_edges(n, edges, w))
    A = entries(g)
    for _ in range(6):
        C = rng.integers(0, n, size=n).astype(np.int32)
        assert _exact(g, C) == q_pairwise(n, A, C)


@pytest.mark.parametrize("seed", range(8))
def test_modularity_matches_networkx(seed):
    # library routine on self-loop-free graphs (networkx counts each undirected edge once)
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 40))
    edges, w = random_graph(rng, n, 0.2, wmax=4, self_loops=False)
    if not edges:
        edges, w = [(0, 1)], [1]
    g = _og(graphgen.from_edges(n, edges, w))
    G = nx.Graph()
    G.add_nodes_from(range(n))
    for (u, v), x in zip(edges, w):
        G.add_edge(u, v, weight=x)
    for _ in range(4):
        C = rng.integers(0, max(1, n // 3), size=n).astype(np.int32)
        parts = [set(np.flatnonzero(C == c).tolist()) for c in np.unique(C)]
        ref = nx.community.modularity(G, parts, weight="weight")
        assert abs(oracle.modularity(g, C) - ref) < 1e-12


def test_closed_forms():
    rng = np.random.default_rng(7)
    edges, w = random_graph(rng, 12, 0.4, self_loops=False)
    g = _og(graphgen.from_edges(12, edges, w))
    K, W = oracle.vertex_weights(g)
    # everything in one community: Q = 0
    assert _exact(g, np.zeros(12, np.int32)) == 0
    # singletons without self-loops: Q = -sum (K_i/W)^2
    assert _exact(g, np.arange(12, dtype=np.int32)) == -sum(Fraction(int(k), W) ** 2 for k in K)
    # edgeless graph: Q defined as 0
    e = _og(graphgen.from_edges(5, []))
    assert oracle.modularity(e, np.arange(5, dtype=np.int32)) == 0.0


@pytest.mark.parametrize("k,s", [(2, 3), (3, 4), (5, 5), (7, 2), (10, 6)])
def test_disjoint_cliques_closed_form(k, s):
    # k equal disjoint cliques split along the cliques: Q = 1 - 1/k, in FP64 exactly (k-1)/k
    g = _og(graphgen.cliques(k, s))
    C = (np.arange(k * s) // s).astype(np.int32)
    assert _exact(g, C) == Fraction(k - 1, k)
    assert oracle.modularity(g, C) == (k - 1) / k


def test_modularity_range():
    # Section 3.2: Q lies in [-1/2, 1]
    rng = np.random.default_rng(3)
    for _ in range(30):
        n = int(rng.integers(2, 16))
        edges, w = random_graph(rng, n, 0.3, self_loops=True)
        if not edges:
            continue
        g = _og(graphgen.from_edges(n, edges, w))
        C = rng.integers(0, n, size=n).astype(np.int32)
        q = _exact(g, C)
        assert Fraction(-1, 2) <= q <= 1


@pytest.mark.parametrize("seed", range(10))
def test_gain_equals_modularity_difference(seed):
    # Eq. 2 scaled by W^2/2: for every vertex and every target community (an empty one
    # included) 2N/W^2 equals Q(after) - Q(before) exactly, self-loops included
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(2, 11))
    edges, w = random_graph(rng, n, 0.4, wmax=6, self_loops=True)
    if not edges:
        edges, w = [(0, 1)], [2]
    g = _og(graphgen.from_edges(n, edges, w))
    A = entries(g)
    _, W = oracle.vertex_weights(g)
    C = rng.integers(0, max(1, n // 2), size=n).astype(np.int32)
    before = q_pairwise(n, A, C)
    empty = [c for c in range(n) if c not in set(C.tolist())]
    for i in range(n):
        for c in sorted(set(C.tolist()) | set(empty[:1])):
            N = oracle.move_gain(g, C, i, c)
            C2 = C.copy()
            C2[i] = c
            assert Fraction(2 * N, W * W) == q_pairwise(n, A, C2) - before, (i, c)
