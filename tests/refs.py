"""Independent reference definitions used to pin the oracle (pure Python, exact Fractions).

Nothing here calls the oracle: each function restates a definition from the
paper or from textbook mathematics in the most direct form.
"""
from fractions import Fraction
from typing import Dict, List, Sequence, Tuple

import numpy as np


def entries(g) -> Dict[Tuple[int, int], int]:
    """A_ij from a CSR (offsets, targets, weights): the stored entry weight (self-loop once)."""
    A: Dict[Tuple[int, int], int] = {}
    for i in range(g.n):
        for e in range(int(g.offsets[i]), int(g.offsets[i + 1])):
            A[(i, int(g.targets[e]))] = A.get((i, int(g.targets[e])), 0) + int(g.weights[e])
    return A


def q_pairwise(n: int, A: Dict[Tuple[int, int], int], C: Sequence[int]) -> Fraction:
    """Modularity from its pairwise definition (Section 3.2): the observed weight minus the
    null-model expectation K_i K_j / W over every ordered vertex pair in the same community,
    divided by W = sum of all entries.  Returns 0 for an edgeless graph."""
    K = [0] * n
    for (i, _j), w in A.items():
        K[i] += w
    W = sum(K)
    if W == 0:
        return Fraction(0)
    total = Fraction(0)
    for i in range(n):
        for j in range(n):
            if C[i] == C[j]:
                total += Fraction(A.get((i, j), 0)) - Fraction(K[i] * K[j], W)
    return total / W


def set_partitions(n: int):
    """All set partitions of range(n) as restricted-growth label lists."""
    labels = [0] * n

    def rec(k: int, m: int):
        if k == n:
            yield list(labels)
            return
        for c in range(m + 1):
            labels[k] = c
            yield from rec(k + 1, max(m, c + 1))

    if n == 0:
        yield []
        return
    yield from rec(1, 1)


def q_optimum(n: int, A: Dict[Tuple[int, int], int]) -> Fraction:
    """Maximum modularity over every partition (exhaustive; n <= 10)."""
    K = [0] * n
    for (i, _j), w in A.items():
        K[i] += w
    W = sum(K)
    if W == 0:
        return Fraction(0)
    items = list(A.items())
    best = None
    # Q*W^2 = W*sigma - sum_c Sigma_c^2 is an integer; maximise it exactly
    for lab in set_partitions(n):
        sigma = 0
        for (i, j), w in items:
            if lab[i] == lab[j]:
                sigma += w
        sig = {}
        for i in range(n):
            sig[lab[i]] = sig.get(lab[i], 0) + K[i]
        val = W * sigma - sum(s * s for s in sig.values())
        if best is None or val > best:
            best = val
    return Fraction(best, W * W)


def random_graph(rng: np.random.Generator, n: int, p: float, wmax: int = 5,
                 self_loops: bool = True):
    """Random undirected weighted edges (u <= v) for tests."""
    edges: List[Tuple[int, int]] = []
    weights: List[int] = []
    for u in range(n):
        for v in range(u if self_loops else u + 1, n):
            if rng.random() < p:
                edges.append((u, v))
                weights.append(int(rng.integers(1, wmax + 1)))
    return edges, weights
