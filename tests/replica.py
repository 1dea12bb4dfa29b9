"""First-iteration decisions at any graph size, from the oracle on local replicas.

In the first synchronous iteration with one round, every vertex decides
against the singleton partition, so its decision depends only on W, its own
row, and the weighted degrees K_j of its neighbours.  A replica graph keeps
exactly those: vertex i, its neighbours (ids in the same relative order, so
ties and the singleton rule resolve alike), each neighbour's missing degree as
a self-loop, and one ballast vertex whose self-loop restores W.  The oracle's
own synchronous iteration on the replica then gives i's decision.
"""
import numpy as np

import oracle


def replica(g, K, W, i):
    """(replica Graph, sorted original ids of its first vertices, i's replica id)."""
    row = g.targets[g.offsets[i]:g.offsets[i + 1]].astype(np.int64)
    wr = g.weights[g.offsets[i]:g.offsets[i + 1]].astype(np.int64)
    own = row == i
    self_w = int(wr[own].sum())
    nb, nw = row[~own], wr[~own]
    ids = np.sort(np.concatenate(([i], nb)))
    m = len(ids)
    ri = int(np.searchsorted(ids, i))
    rj = np.searchsorted(ids, nb).astype(np.int64)
    ballast = int(W - K[i] - K[nb].sum())
    assert ballast >= 0
    rest = K[nb] - nw
    keep = rest > 0
    one_i = np.full(len(rj), ri, dtype=np.int64)
    parts = [(one_i, rj, nw), (rj, one_i, nw), (rj[keep], rj[keep], rest[keep])]  # i-j, j-i, j's loops
    if self_w:
        parts.append((np.array([ri]), np.array([ri]), np.array([self_w])))
    if ballast:
        parts.append((np.array([m]), np.array([m]), np.array([ballast])))
    src = np.concatenate([p[0] for p in parts]).astype(np.int64)
    dst = np.concatenate([p[1] for p in parts]).astype(np.int64)
    ww = np.concatenate([p[2] for p in parts]).astype(np.int64)
    order = np.lexsort((dst, src))
    src, dst, ww = src[order], dst[order], ww[order]
    off = np.zeros(m + 2, dtype=np.int64)
    np.add.at(off, src + 1, 1)
    off = np.cumsum(off)
    return oracle.as_graph(off, dst.astype(np.int32), ww), ids, ri


def first_iteration_decision(g, K, W, i):
    """The community (an original vertex id) vertex i joins in the first synchronous
    iteration with one round, from the singleton partition."""
    if g.offsets[i + 1] == g.offsets[i]:
        return i
    rep, ids, ri = replica(g, K, W, i)
    st = oracle.MoveState.fresh(rep)
    oracle.move(rep, st, mode="sync", tau=0.0, max_iter=1, prune=False, seed=0, pass_index=0,
                sample_bits=0)
    c = int(st.C[ri])
    assert c < len(ids), "joined the ballast"
    return int(ids[c])
