"""Brute-force pin of the oracle's synchronous iterations (the deterministic modes' references).

Each case recomputes whole iterations from definitions that share nothing with the oracle:
modularity from its pairwise form (Section 3.2) as the exact integer W^2 Q, the round of a
vertex from the generator module's SplitMix64, and the decision rule of Alg. 2 restated
(every active vertex of a round compares the modularity after moving it alone into each
neighbouring community, all against the state at the start of the round; it takes the
largest gain, ties to the lowest label, only if the gain is positive, and a singleton does
not join another singleton with a larger label); the round's moves then apply together,
and a mover marks every entry of its row active for the next iteration (pruning, Section
4.1.6).  In the colour-ordered mode the rounds are the colour classes of the greedy colouring
in decreasing hashed priority, in ascending colour, and the singleton rule is off."""
import numpy as np
import pytest

import graphgen
import oracle
from refs import entries, random_graph


def _round(seed, p, l, i, bits):
    ctr = (p << 40) | ((l & 0xFF) << 32) | i
    return graphgen.splitmix_draw(seed, ctr) >> (64 - bits) if bits else 0


def _w2q(n, A, K, W, C):
    # W^2 Q = sum over ordered pairs in one community of (W A_ij - K_i K_j)
    t = 0
    for i in range(n):
        for j in range(n):
            if C[i] == C[j]:
                t += W * A.get((i, j), 0) - K[i] * K[j]
    return t


def _greedy_colours(n, rows, seed, p):
    # visit vertices by decreasing SplitMix64 priority; each takes the smallest colour no
    # earlier neighbour holds
    prio = [graphgen.splitmix_draw(seed, (1 << 63) | (p << 40) | v) for v in range(n)]
    col = [-1] * n
    for v in sorted(range(n), key=lambda x: -prio[x]):
        taken = {col[j] for j in rows[v] if j != v}
        c = 0
        while c in taken:
            c += 1
        col[v] = c
    return col


def brute_iterations(n, A, labels, seed, pass_index, bits, iters, coloured=False):
    K = [0] * n
    for (i, _j), w in A.items():
        K[i] += w
    W = sum(K)
    rows = {i: sorted(j for (a, j) in A if a == i) for i in range(n)}
    C = list(labels)
    active = [True] * n
    moves, gains = [], []
    col = _greedy_colours(n, rows, seed, pass_index) if coloured else None
    nrounds = (max(col) + 1 if n else 0) if coloured else 1 << bits
    for it in range(iters):
        nxt = [False] * n
        mv, gsum = 0, 0
        for r in range(nrounds):
            base = _w2q(n, A, K, W, C)
            size = {}
            for c in C:
                size[c] = size.get(c, 0) + 1
            chosen = []
            for v in range(n):
                rv = col[v] if coloured else _round(seed, pass_index, it, v, bits)
                if not active[v] or rv != r:
                    continue
                d = C[v]
                best, bc = None, None
                for c in sorted({C[j] for j in rows[v] if j != v} - {d}):
                    C2 = list(C)
                    C2[v] = c
                    gain = _w2q(n, A, K, W, C2) - base
                    if best is None or gain > best:
                        best, bc = gain, c
                if best is None or best <= 0:
                    continue
                if not coloured and size[d] == 1 and size[bc] == 1 and bc > d:
                    continue
                chosen.append((v, bc, best))
            for v, c, gain in chosen:
                C[v] = c
                mv += 1
                gsum += gain
                for j in rows[v]:
                    nxt[j] = True
        active = nxt
        moves.append(mv)
        gains.append(gsum // 2)  # the gain N = W^2 dQ / 2
    return C, moves, gains


# weights up to 6, and unit weights where equal gains (the tie rule) are common
CASES = [(n, p, wmax, seed, bits, pidx, warm)
         for n, p in [(8, 0.4), (14, 0.3), (20, 0.2)]
         for wmax in (6, 1)
         for seed, bits, pidx, warm in [(0, 0, 0, False), (3, 1, 0, False), (7, 2, 3, True),
                                        (11, 1, 5, True)]]


@pytest.mark.parametrize("n,p,wmax,seed,bits,pidx,warm", CASES)
def test_sync_iterations_equal_the_brute_force(n, p, wmax, seed, bits, pidx, warm):
    rng = np.random.default_rng(1000 * n + seed)
    e, w = random_graph(rng, n, p, wmax=wmax, self_loops=wmax > 1)
    csr = graphgen.from_edges(n, e, w)
    g = oracle.as_graph(csr.offsets, csr.targets, csr.weights)
    labels = (rng.integers(0, max(2, n // 3), size=n) if warm else np.arange(n)).astype(np.int32)
    want_C, want_moves, want_gains = brute_iterations(n, entries(csr), labels.tolist(), seed,
                                                      pidx, bits, 2)
    st = oracle.MoveState.warm(g, labels)
    tr = oracle.move(g, st, "sync", tau=-1.0, max_iter=2, seed=seed, pass_index=pidx,
                     sample_bits=bits)
    assert st.C.tolist() == want_C
    k = len(tr.moves)
    assert tr.moves == want_moves[:k] and all(m == 0 for m in want_moves[k:])
    assert tr.sumN == want_gains[:k]
    assert want_moves[0] > 0  # the case exercises moves


@pytest.mark.parametrize("n,p,wmax,seed,bits,pidx,warm", CASES)
def test_colour_iterations_equal_the_brute_force(n, p, wmax, seed, bits, pidx, warm):
    rng = np.random.default_rng(3000 * n + seed)
    e, w = random_graph(rng, n, p, wmax=wmax, self_loops=wmax > 1)
    csr = graphgen.from_edges(n, e, w)
    g = oracle.as_graph(csr.offsets, csr.targets, csr.weights)
    labels = (rng.integers(0, max(2, n // 3), size=n) if warm else np.arange(n)).astype(np.int32)
    want_C, want_moves, want_gains = brute_iterations(n, entries(csr), labels.tolist(), seed,
                                                      pidx, 0, 2, coloured=True)
    st = oracle.MoveState.warm(g, labels)
    tr = oracle.move(g, st, "colour", tau=-1.0, max_iter=2, seed=seed, pass_index=pidx)
    assert st.C.tolist() == want_C
    k = len(tr.moves)
    assert tr.moves == want_moves[:k] and all(m == 0 for m in want_moves[k:])
    assert tr.sumN == want_gains[:k]
    assert want_moves[0] > 0
