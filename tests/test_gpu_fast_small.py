"""Fast mode on small levels: a level (in a batch, a graph's part of it) of at most 1024
vertices is moved in vertex order by one wavefront, which is the oracle's sequential
sweep (Alg. 2 as one thread runs it; isolated vertices are not visited).  On graphs of at most 1024 vertices every pass is
such a level, so fast mode must equal the oracle's sequential mode bit for bit: per
pass the iterations, exact gain sums, moves, visits, raw labels and the aggregated
level, then the membership and Q; alone, warm-started and inside a batch of graphs.
"""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import canonical, same_graph, to_device
from refs import random_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2312_04876_amd as P
    P.load_library()


def _og(csr):
    return oracle.as_graph(csr.offsets, csr.targets, csr.weights)


def small_graphs():
    yield graphgen.from_edges(4, [(0, 1), (1, 2), (2, 3)], name="path4")
    yield graphgen.cliques(6, 5, name="cliques6x5")
    yield graphgen.cliques(3, 4, bridges=[(3, 4), (7, 8)], name="bridged")
    rng = np.random.default_rng(15)
    for n in (12, 90, 400, 1024):
        e, w = random_graph(rng, n, min(0.3, 12.0 / n), wmax=7, self_loops=True)
        yield graphgen.from_edges(n, e, w, name="rand%d" % n)
    yield graphgen.sbm(1000, 10, 0.05, 0.001, seed=3, name="sbm1000")
    yield graphgen.rmat(10, 8, wmax=4, seed=5, name="rmat10w")


SMALL = list(small_graphs())


def seq_parity(csr, initial=None, prune=True, **knobs):
    import paper_2312_04876_amd as P
    print("fast small-level parity:", csr.name, csr.n, csr.nnz, flush=True)
    g = _og(csr)
    prm = oracle.Params(mode="seq", prune=prune)
    memb_o, q_o, recs = oracle.louvain_trace(g, prm, initial=initial)
    ctx = P.Louvain(*to_device(csr), mode="fast", prune=prune, **knobs)
    if initial is not None:
        import torch
        lab = torch.from_numpy(np.ascontiguousarray(initial, dtype=np.int32)).cuda()
        ctx.set_membership(lab)
    try:
        for k, rec in enumerate(recs):
            it, _ = ctx.move()
            assert it == rec.trace.iterations, ("iterations", k)
            tr = ctx.move_trace()
            assert tr["sumN"] == rec.trace.sumN, ("gain sums", k)
            assert tr["moves"] == rec.trace.moves, ("moves", k)
            # isolated vertices are never visited on the GPU; the oracle visits them in the
            # first iteration (with pruning) or in every iteration (without)
            iso = int((np.diff(rec.level.offsets) == 0).sum())
            assert tr["processed"] == [p - (iso if (j == 0 or not prune) else 0)
                                       for j, p in enumerate(rec.trace.processed)], ("visits", k)
            assert np.array_equal(ctx.level_labels().cpu().numpy(), rec.raw_labels), ("labels", k)
            nc, stop = ctx.aggregate()
            assert nc == rec.communities, ("communities", k)
            if rec.next_level is None:
                assert stop
                break
            assert same_graph(canonical(*ctx.level_graph()), rec.next_level), ("level graph", k)
        memb, q, st = ctx.run()
        assert np.array_equal(memb.cpu().numpy(), memb_o)
        assert q == q_o
        assert st["iterations"] == [r.trace.iterations for r in recs]
    finally:
        ctx.close()


@pytest.mark.parametrize("idx", range(len(SMALL)))
def test_fast_small_graph_is_the_sequential_oracle(idx):
    seq_parity(SMALL[idx])


def test_fast_small_without_pruning_and_warm_started():
    csr = SMALL[-2]  # sbm1000
    seq_parity(csr, prune=False)
    seq_parity(csr, initial=graphgen.sbm_blocks(1000, 10))
    rng = np.random.default_rng(3)
    seq_parity(csr, initial=rng.integers(0, 1000, size=1000).astype(np.int32))


def test_fast_small_heavy_weights():
    # total weight past 2^31: 64-bit totals and 128-bit scores, with rows past 2^31 (64-bit
    # LDS sums) and with every row below it (32-bit LDS sums)
    from gpu_util import heavy
    for seed, wmax, wide_rows in ((41, 1 << 27, True), (42, 1 << 20, False)):
        csr = heavy(graphgen.rmat(10, 8, seed=seed), seed, wmax=wmax)
        src = np.repeat(np.arange(csr.n), np.diff(csr.offsets))
        kmax = np.bincount(src, weights=csr.weights.astype(np.float64), minlength=csr.n).max()
        assert (kmax >= 2.0 ** 31) == wide_rows
        seq_parity(csr)


def test_fast_batch_of_small_graphs_is_the_sequential_oracle():
    import torch
    import paper_2312_04876_amd as P
    graphs = SMALL + [graphgen.from_edges(1, [], name="single"),
                      graphgen.from_edges(5, [], name="edgeless")]
    offs, tgts, ws, go = [], [], [], [0]
    vb = eb = 0
    for c in graphs:
        offs.append(c.offsets[:-1] + eb)
        tgts.append(c.targets + vb)
        ws.append(c.weights)
        vb += c.n
        eb += c.nnz
        go.append(vb)
    off = np.concatenate(offs + [np.array([eb], dtype=np.int64)])
    u = graphgen.CSR(vb, off, np.concatenate(tgts).astype(np.int32),
                     np.concatenate(ws).astype(np.int32), "union")
    for rep in range(2):
        ctx = P.Louvain(*to_device(u), graph_offsets=np.array(go, dtype=np.int32), mode="fast")
        memb, _, _ = ctx.run()
        qs, _ = ctx.batch_results()
        parts = ctx.split_membership(memb)
        ctx.close()
        for g, c in enumerate(graphs):
            m_o, q_o, _ = oracle.louvain(_og(c), oracle.Params(mode="seq"))
            assert np.array_equal(parts[g], m_o), (rep, c.name)
            assert qs[g] == q_o, (rep, c.name)


def test_fast_small_level_knob():
    # small_level = -1 sends every level to the concurrent rounds (a valid partition with
    # the oracle's Q of it); 256 moves the 1000-vertex SBM's first level in rounds and
    # its coarse levels in vertex order
    import paper_2312_04876_amd as P
    csr = SMALL[-2]
    g = _og(csr)
    for knob in (-1, 256):
        memb, q, _ = P.louvain(*to_device(csr), mode="fast", small_level=knob)
        memb = memb.cpu().numpy()
        assert q == oracle.modularity(g, memb)
        _, q_seq, _ = oracle.louvain(g, oracle.Params(mode="seq"))
        assert q >= q_seq - 0.01
