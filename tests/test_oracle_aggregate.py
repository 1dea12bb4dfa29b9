"""Pins for renumbering, the community-vertex CSR and aggregation (Alg. 1 and Alg. 3)."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import graphgen
import oracle
from refs import random_graph


def _og(csr):
    return oracle.as_graph(csr.offsets, csr.targets, csr.weights)


@pytest.mark.parametrize("seed", range(6))
def test_renumber_matches_numpy_unique(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 500))
    C = rng.integers(0, n, size=n).astype(np.int32)
    got, nc = oracle.renumber(C)
    uniq, inv = np.unique(C, return_inverse=True)
    assert nc == len(uniq)
    assert (got == inv).all()


@pytest.mark.parametrize("seed", range(6))
def test_community_vertices_match_stable_argsort(seed):
    rng = np.random.default_rng(10 + seed)
    n = int(rng.integers(1, 400))
    nc = int(rng.integers(1, n + 1))
    C = rng.integers(0, nc, size=n).astype(np.int32)
    coff, members = oracle.community_vertices(C, nc)
    assert (coff == np.concatenate([[0], np.cumsum(np.bincount(C, minlength=nc))])).all()
    assert (members == np.argsort(C, kind="stable")).all()


def _sparse(g):
    return sp.csr_matrix((g.weights.astype(np.int64), g.targets, g.offsets), shape=(g.n, g.n))


@pytest.mark.parametrize("seed", range(8))
def test_aggregate_is_indicator_triple_product(seed):
    # the super-vertex graph is P^T A P with P the n x |Gamma| community indicator
    rng = np.random.default_rng(20 + seed)
    if seed % 2:
        csr = graphgen.rmat(9, 6, seed=seed, wmax=4)
    else:
        n = int(rng.integers(2, 60))
        edges, w = random_graph(rng, n, 0.15, wmax=6, self_loops=True)
        csr = graphgen.from_edges(n, edges, w)
    g = _og(csr)
    C, nc = oracle.renumber(rng.integers(0, max(1, g.n // 4), size=g.n).astype(np.int32))
    h = oracle.aggregate(g, C, nc)
    P = sp.csr_matrix((np.ones(g.n, dtype=np.int64), (np.arange(g.n), C)), shape=(g.n, nc))
    ref = (P.T @ _sparse(g) @ P).tocsr()
    ref.sort_indices()
    ref.eliminate_zeros()
    assert h.n == nc
    assert (h.offsets == ref.indptr).all()
    assert (h.targets == ref.indices).all()
    assert (h.weights == ref.data).all()
    # W is preserved and the result is symmetric
    assert int(h.weights.sum()) == int(g.weights.sum())
    Hm = _sparse(h)
    assert (Hm != Hm.T).nnz == 0


@pytest.mark.parametrize("seed", range(6))
def test_singletons_of_aggregate_keep_modularity(seed):
    # Q(G'', singletons) == Q(G', C') exactly
    g = _og(graphgen.rmat(10, 8, seed=seed, wmax=3))
    rng = np.random.default_rng(seed)
    C, nc = oracle.renumber(rng.integers(0, g.n // 8, size=g.n).astype(np.int32))
    h = oracle.aggregate(g, C, nc)
    assert oracle.modularity_exact(h, np.arange(nc, dtype=np.int32)) == \
        oracle.modularity_exact(g, C)


def test_aggregate_of_cliques():
    # k disjoint K_s collapse to k isolated super-vertices with a self-loop of s(s-1)
    k, s = 4, 5
    g = _og(graphgen.cliques(k, s))
    C = (np.arange(k * s) // s).astype(np.int32)
    h = oracle.aggregate(g, C, k)
    assert h.offsets.tolist() == list(range(k + 1))
    assert h.targets.tolist() == list(range(k))
    assert h.weights.tolist() == [s * (s - 1)] * k
    num, den = oracle.modularity_exact(h, np.arange(k, dtype=np.int32))
    assert Fraction(num, den) == Fraction(k - 1, k)
