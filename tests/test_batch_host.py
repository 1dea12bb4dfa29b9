"""Host-side pieces of batches: the union of CSRs and the batched SBM recipe."""
import numpy as np

import graphgen


def test_union_shifts_ids_and_marks_ranges():
    a = graphgen.from_edges(3, [(0, 1), (1, 2)], name="a")
    b = graphgen.from_edges(0, [], name="empty")
    c = graphgen.from_edges(2, [(0, 1), (1, 1)], [2, 5], name="c")
    u, go = graphgen.union([a, b, c])
    assert go.tolist() == [0, 3, 3, 5]
    assert u.n == 5 and u.nnz == a.nnz + c.nnz
    assert u.offsets.tolist() == a.offsets.tolist() + (c.offsets[1:] + a.nnz).tolist()
    assert u.targets[a.nnz:].tolist() == (c.targets + 3).tolist()
    assert u.weights.tolist() == a.weights.tolist() + c.weights.tolist()
    for g in range(3):
        lo, hi = go[g], go[g + 1]
        t = u.targets[u.offsets[lo]:u.offsets[hi]]
        assert ((t >= lo) & (t < hi)).all()


def test_batch_sbm_specs_follow_the_recipe():
    sp = graphgen.batch_sbm_specs(512, seed=4)
    n = np.array([s["n"] for s in sp])
    assert n.min() >= 200 and n.max() <= 50_000
    # log-uniform: the median is near the geometric mean of the bounds
    assert 2000 < np.median(n) < 5000
    for s in sp:
        assert 4 <= s["k"] <= 200 and 0 < s["p_in"] <= 1.0
        assert abs(s["p_out"] - 0.02 * s["p_in"]) < 1e-15
        sz = s["n"] / s["k"]
        dbar = s["p_in"] * ((sz - 1) + 0.02 * (s["n"] - sz))
        assert 8.0 - 1e-9 <= dbar <= 40.0 + 1e-9
    assert graphgen.batch_sbm_specs(8, seed=4) == sp[:8]


def test_perturb_deletes_and_inserts_a_share_of_edges():
    g = graphgen.rmat(10, 8, seed=3)
    h = graphgen.perturb(g, 0.1, seed=4)
    assert h.n == g.n
    # symmetric, sorted rows, no duplicate pairs, positive weights
    src = np.repeat(np.arange(h.n), np.diff(h.offsets))
    pairs = set(zip(src.tolist(), h.targets.tolist()))
    assert all((b, a) in pairs for a, b in pairs)
    for i in range(h.n):
        row = h.targets[h.offsets[i]:h.offsets[i + 1]]
        assert (np.diff(row) > 0).all()
    assert (h.weights > 0).all()
    src_g = np.repeat(np.arange(g.n), np.diff(g.offsets))
    old = set(zip(src_g.tolist(), g.targets.tolist()))
    m = sum(1 for a, b in old if a < b)
    kept = sum(1 for a, b in old if a < b and (a, b) in pairs)
    assert abs((m - kept) - 0.1 * m) <= 0.02 * m + 2   # about a tenth deleted (re-inserts aside)
    assert graphgen.perturb(g, 0.0).targets.tolist() == g.targets.tolist()
