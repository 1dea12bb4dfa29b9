"""Host-side pieces of batches: the union of CSRs and the batched SBM recipe."""
import os

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


def test_batch_vs_oracle_script(tmp_path):
    # the script behind the batch profile's oracle comparison: on a tiny batch whose "union"
    # modularities are the oracle's own sequential results (and whose "one by one" ones are
    # 0.02 lower for one graph) it counts what it should
    import json
    import subprocess
    import sys

    import oracle
    here = os.path.dirname(os.path.abspath(__file__))
    u, go, _ = graphgen.batch_sbm(6, seed=7, n_max=400)
    qs = []
    for g in range(6):
        a, b = int(go[g]), int(go[g + 1])
        e0, e1 = int(u.offsets[a]), int(u.offsets[b])
        og = oracle.as_graph((u.offsets[a:b + 1] - e0).astype(np.int64),
                             (u.targets[e0:e1] - np.int32(a)).astype(np.int32),
                             u.weights[e0:e1].astype(np.int32))
        qs.append(oracle.louvain(og, oracle.Params(mode="seq"))[1])
    worse = list(qs)
    worse[2] -= 0.02
    path = tmp_path / "q.json"
    path.write_text(json.dumps({"graphs": 6, "seed": 7, "batch_nmax": 400,
                                "q_union": qs, "q_one_by_one": worse}))
    out = subprocess.run([sys.executable, os.path.join(here, "golden", "batch_vs_oracle.py"),
                          str(path), "--workers", "2"], capture_output=True, text=True,
                         timeout=300, check=True).stdout
    lines = [l for l in out.splitlines() if l.startswith("q_")]
    assert "below -0.01: 0," in lines[0] and "equal: 6;" in lines[0]
    assert "below -0.01: 1," in lines[1] and "equal: 5;" in lines[1]
