"""GPU parity: the HIP path through its C ABI against the oracle.

Deterministic mode: bit-exact against the oracle's synchronous mode after every
pass (iterations, exact per-iteration gain sums, moves, raw labels, community
counts, canonical super-vertex graph), then the final membership and Q.
Fast mode: a valid partition whose reported Q equals the oracle's Q of the
same membership bit for bit, within 0.01 of the oracle's sequential Q, and an
aggregation that is bit-exact for its own membership.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import canonical, heavy, is_valid_partition, same_graph, seq_floor, to_device
from refs import random_graph

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "reference.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2312_04876_amd as P
    P.load_library()


def _og(csr):
    return oracle.as_graph(csr.offsets, csr.targets, csr.weights)


def _isolated(g):
    return int((np.diff(g.offsets) == 0).sum())


def det_parity(csr, round_bits=1, seed=0, max_passes=10, max_iterations=20, prune=True,
               tolerance=0.01, initial=None, coloured=False, **knobs):
    """Step the GPU deterministic mode pass by pass against the oracle's sync mode
    (warm-started from the labels `initial` when given); with `coloured`, the
    colour-ordered mode against the oracle's colour mode."""
    import paper_2312_04876_amd as P
    print("det parity:", csr.name or "graph", csr.n, csr.nnz, "round_bits", round_bits,
          "seed", seed, "coloured" if coloured else "hashed rounds", flush=True)
    g = _og(csr)
    prm = oracle.Params(mode="colour" if coloured else "sync", seed=seed, sample_bits=round_bits,
                        max_passes=max_passes, max_iterations=max_iterations, prune=prune,
                        tolerance=tolerance)
    memb_o, q_o, recs = oracle.louvain_trace(g, prm, initial=initial)
    off, tgt, w = to_device(csr)
    ctx = P.Louvain(off, tgt, w, mode="coloured" if coloured else "deterministic", seed=seed,
                    round_bits=round_bits,
                    max_passes=max_passes, max_iterations=max_iterations, prune=prune,
                    tolerance=tolerance, **knobs)
    labels0 = None
    if initial is not None:
        import torch
        labels0 = torch.from_numpy(np.ascontiguousarray(initial, dtype=np.int32)).cuda()
        ctx.set_membership(labels0)
    try:
        for k, rec in enumerate(recs):
            it, _dq = ctx.move()
            assert it == rec.trace.iterations, ("iterations", k)
            tr = ctx.move_trace()
            assert tr["sumN"] == rec.trace.sumN, ("gain sums", k)
            assert tr["moves"] == rec.trace.moves, ("moves", k)
            iso = _isolated(rec.level)
            # isolated vertices are never queued on the GPU; the oracle visits them in the
            # first iteration (with pruning) or in every iteration (without)
            exp_proc = [p - (iso if (k2 == 0 or not prune) else 0)
                        for k2, p in enumerate(rec.trace.processed)]
            assert tr["processed"] == exp_proc, ("processed", k)
            labels = ctx.level_labels().cpu().numpy()
            assert np.array_equal(labels, rec.raw_labels), ("labels", k)
            nc, stop = ctx.aggregate()
            assert nc == rec.communities, ("communities", k)
            if rec.next_level is None:
                assert stop
                break
            assert same_graph(canonical(*ctx.level_graph()), rec.next_level), ("level graph", k)
            assert stop == (k + 1 == max_passes)
        memb, q, st = ctx.run()
        memb = memb.cpu().numpy()
        assert np.array_equal(memb, memb_o)
        assert q == q_o
        assert st["iterations"] == [r.trace.iterations for r in recs]
        if coloured:
            want = [oracle.colour(r.level, seed, k)[1] if r.level.nnz else 0
                    for k, r in enumerate(recs)]
            assert st["colours"] == want, ("colours", st["colours"], want)
    finally:
        ctx.close()


# ----------------------------------------------------------------- deterministic mode

def small_graphs():
    yield graphgen.from_edges(4, [(0, 1), (1, 2), (2, 3)], name="path4")
    yield graphgen.cliques(6, 5, name="cliques6x5")
    yield graphgen.cliques(3, 4, bridges=[(3, 4), (7, 8)], name="bridged")
    rng = np.random.default_rng(5)
    for n in (12, 40, 90):
        e, w = random_graph(rng, n, 0.2, wmax=7, self_loops=True)
        yield graphgen.from_edges(n, e, w, name="rand%d" % n)


@pytest.mark.parametrize("small_level", [1024, 0])
@pytest.mark.parametrize("idx", range(6))
def test_det_small(idx, small_level):
    # small_level 1024: these levels are moved by one wavefront each (k_sync_level);
    # 0 (the deterministic default): by the degree bins' rounds
    det_parity(list(small_graphs())[idx], small_level=small_level)


@pytest.mark.parametrize("wl", ["sbm10k", "rmat12-8", "rmat14-16", "rmat16-16"])
def test_det_workloads(wl):
    det_parity(graphgen.workload(wl))


@pytest.mark.parametrize("round_bits,seed", [(0, 0), (2, 7), (3, 11)])
def test_det_round_settings(round_bits, seed):
    det_parity(graphgen.workload("rmat13-8"), round_bits=round_bits, seed=seed)


def test_det_weighted_and_no_prune():
    det_parity(graphgen.rmat(13, 12, wmax=8, seed=9, name="rmat13w"), prune=False)
    det_parity(graphgen.workload("sbm10k"), max_passes=2, max_iterations=5, tolerance=0.0)


def hub_graph():
    """An R-MAT background plus a star whose centre has 10,000 neighbours (hub bin)
    and a dense block, so every degree bin is exercised in moving and aggregation."""
    base = graphgen.rmat(14, 8, seed=21)
    src = np.repeat(np.arange(base.n), np.diff(base.offsets))
    edges = [(int(a), int(b)) for a, b in zip(src, base.targets) if a < b]
    n = base.n
    edges += [(0, v) for v in range(1, 10001)]
    edges += [(i, j) for i in range(10100, 10220) for j in range(i + 1, 10220)]
    return graphgen.from_edges(n, edges, name="hub")


def test_det_wide_totals():
    det_parity(heavy(graphgen.rmat(12, 8, seed=41), 1))
    det_parity(heavy(hub_graph(), 2), round_bits=2, seed=3)
    det_parity(heavy(graphgen.sbm(3000, 30, 0.03, 0.001, seed=42), 3), prune=False)


def test_wide_totals_with_weights_below_2_19():
    # W past 2^31 while every weight is below 2^19: the first aggregation folds the hub
    # communities' windows of 4096 entries with 32-bit sums, which cannot overflow
    det_parity(heavy(hub_graph(), 6, wmax=(1 << 19) - 1))


def test_wide_totals_with_rows_below_2_31():
    # W past 2^31 while every row sum K' stays below 2^31: local moving on the input level
    # keeps 32-bit LDS tables (every bin, hubs included)
    import paper_2312_04876_amd as P
    csr = heavy(hub_graph(), 7, wmax=1 << 16)
    src = np.repeat(np.arange(csr.n), np.diff(csr.offsets))
    assert np.bincount(src, weights=csr.weights.astype(np.float64)).max() < 2.0 ** 31
    det_parity(csr)
    det_parity(csr, coloured=True, seed=2)
    g = _og(csr)
    memb, q, _ = P.louvain(*to_device(csr), mode="fast")
    memb = memb.cpu().numpy()
    assert is_valid_partition(memb)
    assert q == oracle.modularity(g, memb)
    _, q_seq, _ = oracle.louvain(g, oracle.Params(mode="seq"))
    assert abs(q - q_seq) <= 0.01


def test_coloured_wide_totals():
    det_parity(heavy(hub_graph(), 4), coloured=True, seed=1)


def _row_sum_max(csr):
    src = np.repeat(np.arange(csr.n), np.diff(csr.offsets))
    return np.bincount(src, weights=csr.weights.astype(np.float64), minlength=csr.n).max()


# heavy-weight graphs (W past 2^31): random weights make every vertex's heaviest edge a
# strong pull, the case where a label seen before its community total is updated
# drags neighbours after movers
FAST_HEAVY = {
    "rmat13-8": lambda: heavy(graphgen.rmat(13, 8, seed=43), 5),
    "rmat12-16": lambda: heavy(graphgen.rmat(12, 16, seed=7), 11),
    "rmat14-8": lambda: heavy(graphgen.rmat(14, 8, seed=44), 6),
    "sbm10k-w16": lambda: heavy(graphgen.workload("sbm10k"), 8, wmax=1 << 16),
}


@pytest.mark.parametrize("name", sorted(FAST_HEAVY))
def test_fast_wide_totals(name):
    import paper_2312_04876_amd as P
    csr = FAST_HEAVY[name]()
    # rows past 2^31 take the 64-bit LDS tables; the SBM keeps every row below it (32-bit)
    assert (_row_sum_max(csr) >= 2.0 ** 31) == name.startswith("rmat"), name
    g = _og(csr)
    off, tgt, w = to_device(csr)
    _, q_seq, _ = oracle.louvain(g, oracle.Params(mode="seq"))
    for rep in range(3):
        memb, q, _ = P.louvain(off, tgt, w, mode="fast")
        memb = memb.cpu().numpy()
        print("fast", name, "run", rep, "Q %.5f sequential oracle %.5f" % (q, q_seq), flush=True)
        assert is_valid_partition(memb)
        assert q == oracle.modularity(g, memb)
        assert abs(q - q_seq) <= 0.01, (name, rep, q, q_seq)


def test_det_hub_bins():
    det_parity(hub_graph())


@pytest.mark.parametrize("seed", range(6))
def test_det_and_coloured_random_graphs(seed):
    # ragged random graphs (sizes that leave partial tiles in every bin, self-loops,
    # weights up to 9, isolated vertices) in both deterministic modes and round settings,
    # and in fast mode
    rng = np.random.default_rng(4200 + seed)
    n = int(rng.integers(150, 1500))
    e, w = random_graph(rng, n, float(rng.uniform(2.0, 30.0)) / n, wmax=9, self_loops=True)
    e += [(0, v) for v in range(1, min(n, 40 + 120 * seed))]  # one long row
    w += [int(x) for x in rng.integers(1, 10, size=min(n, 40 + 120 * seed) - 1)]
    csr = graphgen.from_edges(n, e, w, name="rand%d" % seed)
    det_parity(csr, round_bits=seed % 3, seed=seed)
    det_parity(csr, round_bits=seed % 3, seed=seed, small_level=1024)
    det_parity(csr, coloured=True, seed=seed)
    # fast mode: a valid partition whose reported Q is the oracle's Q of it, bit for bit,
    # no more than 0.01 below the sequential oracle over its own vertex order and eight
    # relabellings (small random graphs spread more than 0.01 over visiting orders)
    import paper_2312_04876_amd as P
    memb, q, _ = P.louvain(*to_device(csr), mode="fast")
    memb = memb.cpu().numpy()
    assert is_valid_partition(memb)
    assert q == oracle.modularity(_og(csr), memb)
    assert q >= seq_floor(_og(csr)) - 0.01


# ----------------------------------------------------------------- colour-ordered mode

@pytest.mark.parametrize("idx", range(6))
def test_coloured_small(idx):
    det_parity(list(small_graphs())[idx], coloured=True)


@pytest.mark.parametrize("wl,seed", [("sbm10k", 0), ("rmat13-8", 3), ("rmat16-16", 1)])
def test_coloured_workloads(wl, seed):
    det_parity(graphgen.workload(wl), seed=seed, coloured=True)


def test_coloured_more_than_1024_colours():
    # a clique of 1100 vertices needs 1100 colours: rows above 512 entries are coloured
    # in chunks whose bitmaps cover 1024 colours, so the last 76 need the rescan
    det_parity(graphgen.cliques(1, 1100, bridges=[(0, 0)]), seed=2, max_passes=2, coloured=True)


def multi_hub_graph():
    """An R-MAT background with six adjacent centres of 9,000 random neighbours each:
    several hub rows, all of different colours."""
    base = graphgen.rmat(14, 8, seed=23)
    src = np.repeat(np.arange(base.n), np.diff(base.offsets))
    edges = {(int(a), int(b)) for a, b in zip(src, base.targets) if a < b}
    rng = np.random.default_rng(24)
    centres = [11, 222, 3333, 4444, 5555, 16000]
    for c in centres:
        for v in rng.choice(base.n, size=9000, replace=False):
            if int(v) != c:
                edges.add((min(c, int(v)), max(c, int(v))))
    for i, c in enumerate(centres):
        for d in centres[i + 1:]:
            edges.add((min(c, d), max(c, d)))
    return graphgen.from_edges(base.n, sorted(edges), name="multihub")


def test_coloured_hubs_weights_and_no_prune():
    det_parity(hub_graph(), coloured=True)
    det_parity(multi_hub_graph(), seed=5, coloured=True)
    det_parity(graphgen.rmat(13, 12, wmax=8, seed=9, name="rmat13w"), prune=False, seed=4,
               coloured=True)


def big_star(leaves):
    """A centre joined to `leaves` leaves that are also joined in pairs (2k+1, 2k+2).
    Its row of 4M distinct communities overfills the LDS table of every hub partition
    in the first iteration, so the range-splitting passes run."""
    assert leaves % 2 == 0
    n = leaves + 1
    deg = np.full(n, 2, dtype=np.int64)
    deg[0] = leaves
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(deg)
    tgt = np.empty(off[-1], dtype=np.int32)
    tgt[:leaves] = np.arange(1, n, dtype=np.int32)
    leaf = np.arange(1, n, dtype=np.int64)
    partner = np.where(leaf % 2 == 1, leaf + 1, leaf - 1)
    rows = tgt[leaves:].reshape(leaves, 2)
    rows[:, 0] = 0
    rows[:, 1] = partner
    return graphgen.CSR(n=n, offsets=off, targets=tgt, weights=np.ones(off[-1], dtype=np.int32),
                        name="star%d" % leaves)


def test_det_hub_partition_overflow():
    det_parity(big_star(4_000_000), max_passes=2)


def test_det_warm_start():
    # the first pass starts from a given partition (the dynamic re-run): blocks of a
    # coarse SBM labelling, a random labelling, and a cold run's own membership on a
    # perturbed graph
    rng = np.random.default_rng(17)
    sbm = graphgen.workload("sbm10k")
    det_parity(sbm, initial=(np.arange(sbm.n) // 250).astype(np.int32))
    rm = graphgen.workload("rmat14-16")
    det_parity(rm, initial=rng.integers(0, rm.n, size=rm.n).astype(np.int32))
    memb, _, _ = oracle.louvain(_og(rm), oracle.Params(mode="sync"))
    rm2 = graphgen.rmat(14, 16, seed=3, name="rmat14-16-other")
    det_parity(rm2, initial=memb.astype(np.int32), round_bits=2, seed=5)


def test_coloured_warm_start():
    sbm = graphgen.workload("sbm10k")
    det_parity(sbm, initial=(np.arange(sbm.n) // 250).astype(np.int32), coloured=True, seed=2)
    rm = graphgen.workload("rmat14-16")
    memb, _, _ = oracle.louvain(_og(rm), oracle.Params(mode="colour", seed=2))
    det_parity(graphgen.rmat(14, 16, seed=3, name="rmat14-16-other"), initial=memb.astype(np.int32),
               coloured=True, seed=2)


def test_fast_warm_start_from_the_planted_partition():
    # fast mode from SBM-10k's planted partition: hardly any vertex moves in the first
    # iteration (the sequential oracle moves 3.4% in its first sweep) and the first
    # pass ends at least as good as the planted partition
    import paper_2312_04876_amd as P
    import torch
    csr = graphgen.workload("sbm10k")
    g = _og(csr)
    off, tgt, w = to_device(csr)
    planted = graphgen.sbm_blocks(csr.n, 100).astype(np.int32)
    q0 = oracle.modularity(g, planted)
    ctx = P.Louvain(off, tgt, w, mode="fast", max_passes=1)
    try:
        ctx.set_membership(torch.from_numpy(planted).cuda())
        ctx.move()
        tr = ctx.move_trace()
        labels = ctx.level_labels().cpu().numpy()
        q1 = oracle.modularity(g, labels)
        print("from the planted partition: moves", tr["moves"], "Q", q0, "->", q1, flush=True)
        assert tr["moves"][0] < 0.08 * csr.n
        assert q1 >= q0 - 0.002
    finally:
        ctx.close()


def test_warm_start_rejects_bad_labels_and_late_calls():
    import torch
    import paper_2312_04876_amd as P
    csr = graphgen.workload("rmat12-8")
    ctx = P.Louvain(*to_device(csr), mode="deterministic")
    bad = torch.full((csr.n,), csr.n, dtype=torch.int32, device="cuda")
    with pytest.raises(P.LouvainError):
        ctx.set_membership(bad)
    ctx.move()
    ok = torch.zeros(csr.n, dtype=torch.int32, device="cuda")
    with pytest.raises(P.LouvainError):
        ctx.set_membership(ok)
    ctx.close()


def test_run_checks_the_membership_buffer():
    import torch
    import paper_2312_04876_amd as P
    csr = graphgen.workload("rmat12-8")
    ctx = P.Louvain(*to_device(csr), mode="deterministic")
    for bad in [torch.empty(csr.n - 1, dtype=torch.int32, device="cuda"),
                torch.empty(csr.n, dtype=torch.int64, device="cuda"),
                torch.empty(csr.n, dtype=torch.int32)]:
        with pytest.raises(ValueError):
            ctx.run(bad)
    m1, q1, _ = ctx.run()
    m1 = m1.cpu().numpy().copy()
    ctx.reset()
    big = torch.full((csr.n + 5,), -7, dtype=torch.int32, device="cuda")
    m2, q2, _ = ctx.run(big)
    assert np.array_equal(m1, m2.cpu().numpy()) and q1 == q2
    assert (big[csr.n:].cpu().numpy() == -7).all()
    ctx.close()


def test_det_edge_cases():
    for csr in [graphgen.from_edges(0, [], name="empty"), graphgen.from_edges(1, [], name="one"),
                graphgen.from_edges(7, [], name="isolated"),
                graphgen.from_edges(3, [(1, 1)], [5], name="selfloop"),
                graphgen.from_edges(2, [(0, 1)], [3], name="edge")]:
        det_parity(csr)
    det_parity(graphgen.workload("sbm10k"), max_passes=0)
    det_parity(graphgen.workload("sbm10k"), max_passes=1)


def test_det_repeatable_and_reset():
    import paper_2312_04876_amd as P
    csr = graphgen.workload("rmat14-16")
    off, tgt, w = to_device(csr)
    ctx = P.Louvain(off, tgt, w, mode="deterministic")
    m1, q1, _ = ctx.run()
    m1 = m1.cpu().numpy().copy()
    ctx.reset()
    m2, q2, _ = ctx.run()
    assert np.array_equal(m1, m2.cpu().numpy()) and q1 == q2
    ctx.close()


# ----------------------------------------------------------------- fast mode

def _golden():
    return json.load(open(GOLDEN))


def _fast_q(wl):
    import paper_2312_04876_amd as P
    csr = graphgen.workload(wl)
    g = _og(csr)
    off, tgt, w = to_device(csr)
    memb, q, st = P.louvain(off, tgt, w, mode="fast")
    memb = memb.cpu().numpy()
    print(wl, "fast Q", q, "oracle seq Q", _golden()[wl]["seq"]["Q"], st, flush=True)
    assert is_valid_partition(memb)
    assert q == oracle.modularity(g, memb)
    return q


@pytest.mark.parametrize("wl", ["rmat16-16", "rmat18-16"])
def test_fast_quality(wl):
    # the R-MAT workloads run in fast mode: |Q - Q_oracle_seq| <= 0.01
    assert abs(_fast_q(wl) - _golden()[wl]["seq"]["Q"]) <= 0.01


def test_fast_quality_sbm():
    # SBM-10k is a deterministic-mode workload; in fast mode it must not fall more than
    # 0.01 below the sequential oracle (over 100 runs it lands 0.004-0.008 below it, inside
    # the about 0.012 that the oracle's own Q varies over vertex orders on this graph, see
    # the golden relabelling runs)
    assert _fast_q("sbm10k") >= _golden()["sbm10k"]["seq"]["Q"] - 0.01


def test_fast_sbm1m_second_level_does_not_collapse():
    # sbm1m's second level (thousands of super-vertices of a few hundred entries, hundreds of
    # them deciding at once per round) is where concurrent fast-mode joins once piled into a
    # few communities (Q 0.71-0.73 in about one run of ten); every run must stay within 0.01
    # of the sequential oracle
    import paper_2312_04876_amd as P
    csr = graphgen.workload("sbm1m")
    off, tgt, w = to_device(csr)
    ref = _golden()["sbm1m"]["seq"]["Q"]
    for rep in range(6):
        memb, q, st = P.louvain(off, tgt, w, mode="fast")
        n = st["passes"]
        print("sbm1m fast run", rep, q, st["iterations"][:n], st["communities"][:n], flush=True)
        assert abs(q - ref) <= 0.01, (rep, q, ref)
    memb = memb.cpu().numpy()
    assert is_valid_partition(memb)
    assert q == oracle.modularity(_og(csr), memb)


@pytest.mark.parametrize("wl", ["rmat14-16", "sbm10k"])
def test_fast_aggregation_exact_for_own_membership(wl):
    import paper_2312_04876_amd as P
    csr = graphgen.workload(wl)
    g = _og(csr)
    off, tgt, w = to_device(csr)
    ctx = P.Louvain(off, tgt, w, mode="fast")
    level = g
    for _ in range(4):
        ctx.move()
        labels = ctx.level_labels().cpu().numpy()
        nc, stop = ctx.aggregate()
        dense, nco = oracle.renumber(labels)
        assert nc == nco
        if stop:
            break
        nxt = oracle.aggregate(level, dense, nc)
        assert same_graph(canonical(*ctx.level_graph()), nxt)
        # the singletons of the new level keep the modularity of the membership
        assert oracle.modularity_exact(nxt, np.arange(nc, dtype=np.int32)) == \
            oracle.modularity_exact(level, dense)
        level = nxt
    ctx.close()


def test_fast_hub_graph():
    import paper_2312_04876_amd as P
    csr = hub_graph()
    g = _og(csr)
    off, tgt, w = to_device(csr)
    memb, q, _ = P.louvain(off, tgt, w, mode="fast")
    memb = memb.cpu().numpy()
    assert is_valid_partition(memb)
    assert q == oracle.modularity(g, memb)
    _, q_seq, _ = oracle.louvain(g, oracle.Params(mode="seq"))
    assert abs(q - q_seq) <= 0.01


# ----------------------------------------------------------------- full size (R-MAT scale 22)

@pytest.fixture(scope="module")
def rmat22():
    return graphgen.workload("rmat22")


def test_rmat22_fast_full_size(rmat22):
    import paper_2312_04876_amd as P
    print("rmat22 fast mode", rmat22.n, rmat22.nnz, flush=True)
    g = _og(rmat22)
    off, tgt, w = to_device(rmat22)
    memb, q, st = P.louvain(off, tgt, w, mode="fast")
    memb = memb.cpu().numpy()
    print("rmat22 fast Q", q, st, flush=True)
    assert is_valid_partition(memb)
    assert q == oracle.modularity(g, memb)
    assert abs(q - _golden()["rmat22"]["seq"]["Q"]) <= 0.01


def test_rmat22_det_full_size(rmat22):
    import paper_2312_04876_amd as P
    print("rmat22 deterministic mode", flush=True)
    off, tgt, w = to_device(rmat22)
    memb, q, st = P.louvain(off, tgt, w, mode="deterministic", seed=0, round_bits=1)
    memb = memb.cpu().numpy()
    ref = _golden()["rmat22"]["sync"]
    assert st["iterations"] == ref["iterations"]
    assert st["communities"] == ref["communities"]
    assert hashlib.sha256(memb.astype(np.int32).tobytes()).hexdigest() == ref["digest"]
    assert q == ref["Q"]


@pytest.mark.parametrize("wl", ["rmat22", "sbm1m", "rmat18-16", "sbm10k"])
def test_coloured_full_size_matches_the_stored_oracle_run(wl, rmat22):
    # the colour-ordered run at the benchmark's size against the oracle's colour
    # mode on the same input (membership digest, Q, iterations, communities)
    import paper_2312_04876_amd as P
    csr = rmat22 if wl == "rmat22" else graphgen.workload(wl)
    print(wl, "colour-ordered mode", csr.n, csr.nnz, flush=True)
    off, tgt, w = to_device(csr)
    memb, q, st = P.louvain(off, tgt, w, mode="coloured", seed=0)
    memb = memb.cpu().numpy()
    ref = _golden()[wl]["colour"]
    assert st["iterations"] == ref["iterations"]
    assert st["communities"] == ref["communities"]
    assert hashlib.sha256(memb.astype(np.int32).tobytes()).hexdigest() == ref["digest"]
    assert q == ref["Q"]


# ----------------------------------------------------------------- scheduling knobs

@pytest.mark.parametrize("knobs", [{"hub_rows": 2048, "hub_part_pairs": 1024},
                                   {"hub_rows": 4096, "hub_part_pairs": 2048}])
def test_det_parity_under_other_hub_thresholds(knobs):
    # the knobs move rows between the workgroup and hub paths; results stay the oracle's
    det_parity(hub_graph(), **knobs)
    det_parity(graphgen.workload("rmat16-16"), **knobs)
    det_parity(multi_hub_graph(), seed=5, coloured=True, **knobs)


def test_rmat22_det_full_size_with_every_row_above_2048_on_the_hub_path(rmat22):
    import paper_2312_04876_amd as P
    off, tgt, w = to_device(rmat22)
    memb, q, st = P.louvain(off, tgt, w, mode="deterministic", seed=0, round_bits=1,
                            hub_rows=2048, hub_part_pairs=1024)
    ref = _golden()["rmat22"]["sync"]
    assert hashlib.sha256(memb.cpu().numpy().astype(np.int32).tobytes()).hexdigest() == ref["digest"]
    assert q == ref["Q"]


def test_autotune_picks_a_candidate_and_caches_it(tmp_path):
    from paper_2312_04876_amd import autotune
    csr = graphgen.workload("rmat16-16")
    off, tgt, w = to_device(csr)
    cache = str(tmp_path / "tuned.json")
    res = autotune.tune(off, tgt, w, runs=1, warmup=1, cache_path=cache, mode="fast")
    print("autotune", res["hub_rows"], res["hub_part_pairs"], res["table"], flush=True)
    assert (res["hub_rows"], res["hub_part_pairs"]) in autotune.candidates(wide=False)
    # fast mode keeps its small-level kernel (a quality setting there): six candidates
    assert res["small_level"] == 1024
    assert len(res["table"]) == 6 and not res["cached"]
    again = autotune.tune(off, tgt, w, cache_path=cache, mode="fast")
    assert again["cached"] and again["hub_rows"] == res["hub_rows"]
    # deterministic mode also times the small-level settings (results never change)
    det = autotune.tune(off, tgt, w, runs=1, warmup=1, mode="deterministic")
    assert det["small_level"] in (-1, 256, 1024)
    assert len(det["table"]) == 6 + 2 and not det["cached"]
