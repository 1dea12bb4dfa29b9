"""Checks of the seeded input generators (no community-detection arithmetic involved)."""
import numpy as np
import pytest

import graphgen


def test_splitmix_reference_vector():
    # published SplitMix64 outputs for state 1234567 (Steele, Lea and Flood 2014)
    assert graphgen.splitmix_stream(1234567, 5).tolist() == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]
    # the counter form is the k-th output of the stream started at key
    seq = graphgen.splitmix_stream(42, 4).tolist()
    assert [graphgen.splitmix_draw(42, k) for k in range(4)] == seq


def _check_symmetric(csr, allow_self=False):
    n = csr.n
    off = csr.offsets
    assert off[0] == 0 and (np.diff(off) >= 0).all()
    src = np.repeat(np.arange(n), np.diff(off))
    tgt = csr.targets.astype(np.int64)
    assert ((tgt >= 0) & (tgt < n)).all()
    assert (csr.weights >= 1).all()
    if not allow_self:
        assert (src != tgt).all()
    fwd = sorted(zip(src.tolist(), tgt.tolist(), csr.weights.tolist()))
    rev = sorted(zip(tgt.tolist(), src.tolist(), csr.weights.tolist()))
    assert fwd == rev
    # rows sorted by target, no duplicates
    for i in range(n):
        r = csr.targets[off[i]:off[i + 1]]
        assert (np.diff(r) > 0).all()


@pytest.mark.parametrize("wmax", [1, 8])
def test_rmat_structure(wmax):
    g = graphgen.rmat(10, 8, wmax=wmax, seed=5)
    _check_symmetric(g)
    assert g.n == 1024
    assert 0.6 * 2 * 8 * 1024 < g.nnz <= 2 * 8 * 1024
    assert g.weights.sum() <= 2 * 8 * 1024 * wmax


def test_rmat_deterministic_across_threads():
    a = graphgen.rmat(12, 8, seed=9, threads=1)
    b = graphgen.rmat(12, 8, seed=9, threads=4)
    assert (a.offsets == b.offsets).all() and (a.targets == b.targets).all()
    assert (a.weights == b.weights).all()
    c = graphgen.rmat(12, 8, seed=10)
    assert not (a.nnz == c.nnz and (a.targets == c.targets).all())


def test_rmat_skew():
    # the quadrant probabilities make a heavy-tailed degree distribution
    g = graphgen.rmat(14, 16, seed=2)
    deg = np.diff(g.offsets)
    assert deg.max() > 50 * max(1.0, deg.mean())
    assert (deg == 0).mean() > 0.2


def test_sbm_structure_and_density():
    g = graphgen.workload("sbm10k")
    _check_symmetric(g)
    blocks = graphgen.sbm_blocks(10000, 100)
    src = np.repeat(np.arange(g.n), np.diff(g.offsets))
    inside = blocks[src] == blocks[g.targets]
    n_in = inside.sum() // 2
    n_out = (~inside).sum() // 2
    # expected 100 * C(100,2) * 0.05 = 24750 and (C(10000,2) - 495000) * 0.0005 = 24747.5
    assert abs(n_in - 24750) < 5 * np.sqrt(24750)
    assert abs(n_out - 24747.5) < 5 * np.sqrt(24747.5)
    h = graphgen.sbm(10000, 100, 0.05, 0.0005, seed=1, threads=3)
    assert (h.targets == g.targets).all()


def test_sbm_extremes():
    full = graphgen.sbm(20, 4, 1.0, 0.0, seed=3)
    assert full.nnz == 4 * 5 * 4
    empty = graphgen.sbm(20, 4, 0.0, 0.0, seed=3)
    assert empty.nnz == 0
    _check_symmetric(full)


def test_from_edges_merges_and_keeps_self_loops_once():
    g = graphgen.from_edges(3, [(0, 1), (1, 0), (2, 2)], [2, 3, 4])
    assert g.offsets.tolist() == [0, 1, 2, 3]
    assert g.targets.tolist() == [1, 0, 2]
    assert g.weights.tolist() == [5, 5, 4]
