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
