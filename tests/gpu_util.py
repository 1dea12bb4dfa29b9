"""Helpers of the GPU parity tests: upload CSR graphs, canonical forms of level graphs."""
import numpy as np

import graphgen
import oracle


def to_device(csr):
    import torch
    off = torch.from_numpy(csr.offsets32()).cuda()
    tgt = torch.from_numpy(np.ascontiguousarray(csr.targets, dtype=np.int32)).cuda()
    w = torch.from_numpy(np.ascontiguousarray(csr.weights, dtype=np.int32)).cuda()
    return off, tgt, w


def canonical(offsets, degree, targets, weights):
    """A holey GPU level graph as an oracle Graph: rows sorted by target, gaps removed."""
    off = offsets.cpu().numpy().astype(np.int64)
    n = len(off) - 1
    deg = degree.cpu().numpy().astype(np.int64) if degree is not None else np.diff(off)
    tgt = targets.cpu().numpy()
    w = weights.cpu().numpy().astype(np.int64)
    new_off = np.zeros(n + 1, dtype=np.int64)
    new_off[1:] = np.cumsum(deg)
    out_t = np.empty(int(new_off[n]), dtype=np.int32)
    out_w = np.empty(int(new_off[n]), dtype=np.int64)
    for i in range(n):
        a, d = int(off[i]), int(deg[i])
        r_t = tgt[a:a + d]
        order = np.argsort(r_t, kind="stable")
        out_t[new_off[i]:new_off[i + 1]] = r_t[order]
        out_w[new_off[i]:new_off[i + 1]] = w[a:a + d][order]
    return oracle.Graph(n, new_off, out_t, out_w)


def same_graph(a, b) -> bool:
    return (a.n == b.n and np.array_equal(a.offsets, b.offsets)
            and np.array_equal(a.targets, b.targets) and np.array_equal(a.weights, b.weights))


def is_valid_partition(memb: np.ndarray) -> bool:
    """Dense labels: every label in 0..k-1 is used by some vertex."""
    if memb.size == 0:
        return True
    k = int(memb.max()) + 1
    return memb.min() == 0 and np.unique(memb).size == k


def heavy(csr, seed, wmax=1 << 24, name=""):
    """The same graph with every undirected edge's weight drawn in [1, wmax]: the total
    weight W passes 2^31, so the path keeps 64-bit totals, 128-bit scores and 64-bit
    aggregated weights (and the LDS row limit of 8-byte values)."""
    rng = np.random.default_rng(seed)
    src = np.repeat(np.arange(csr.n), np.diff(csr.offsets))
    keep = src <= csr.targets
    u, v = src[keep], csr.targets[keep]
    w = rng.integers(1, wmax + 1, size=len(u))
    out = graphgen.from_edges(csr.n, list(zip(u.tolist(), v.tolist())), w.tolist(),
                              name=name or (csr.name + "-heavy"))
    assert int(out.weights.sum(dtype=np.int64)) >= 1 << 31
    return out


def relabelled(g, perm):
    """The oracle graph g with vertex v renamed perm[v] (rows keep their entries)."""
    n = g.n
    deg = np.diff(g.offsets)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(deg[inv])
    rows = np.concatenate([np.arange(g.offsets[v], g.offsets[v + 1]) for v in inv]) \
        if g.nnz else np.zeros(0, dtype=np.int64)
    return oracle.Graph(n, off, perm[g.targets[rows]].astype(np.int32), g.weights[rows].copy())


def seq_floor(g, orders=8, seed=0):
    """Lowest modularity the sequential oracle reaches on g over its own vertex order and
    `orders` random relabellings of g (the same graph visited in other orders): the
    spread of the asynchronous method itself, which the 0.01 band of fast mode sits on."""
    q = oracle.louvain(g, oracle.Params(mode="seq"))[1]
    rng = np.random.default_rng(seed)
    for _ in range(orders):
        perm = rng.permutation(g.n).astype(np.int64)
        q = min(q, oracle.louvain(relabelled(g, perm), oracle.Params(mode="seq"))[1])
    return q
