"""Seeded synthetic inputs for the Louvain hot path (both the oracle and the GPU path read them).

This module draws graphs; it holds none of the community-detection arithmetic.
Generators (``graphgen.c``, built with gcc + OpenMP into ``libgraphgen.so``):

* ``rmat``  -- R-MAT with quadrant probabilities a, b, c, d (Chakrabarti et al.
  2004), seeded vertex relabelling, self-loops dropped, both directions stored,
  duplicates merged by summing weights; per-draw weights uniform in 1..wmax.
* ``sbm``   -- planted-partition stochastic block model with equal blocks,
  geometric skipping (Batagelj & Brandes 2005), unit weights.
* ``from_edges`` -- a symmetric CSR from an explicit edge list (tests).

All randomness is counter-based SplitMix64, so a graph is a pure function of
its parameters and seed, independent of the thread count.

Workload presets (``workload(name)``) give the shapes the paper's evaluation
calls for, as seeded synthetic stand-ins (no dataset is read):

* ``sbm10k``  -- 10,000 vertices, 100 equal blocks, p_in 0.05, p_out 0.0005
* ``sbm1m``   -- 1,000,000 vertices, 1,000 equal blocks, p_in 0.015, p_out 0.000005
  (about 15 neighbours inside the block and 5 outside)
* ``rmat22``  -- R-MAT scale 22, 16 draws per vertex, a/b/c/d = .57/.19/.19/.05
* ``rmat24``  -- R-MAT scale 24, 64 draws per vertex, weights 1..8 per draw
* ``rmatS-F`` -- R-MAT of scale S and F draws per vertex, same a/b/c/d (small cases)
"""
from __future__ import annotations

import ctypes
import math
import os
import re
import subprocess
from dataclasses import dataclass
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        vp, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint64, ctypes.c_double)
        lib.gg_rmat.restype = vp
        lib.gg_rmat.argtypes = [i32, i64, dbl, dbl, dbl, i32, u64, i32]
        lib.gg_sbm.restype = vp
        lib.gg_sbm.argtypes = [i64, i64, dbl, dbl, u64, i32]
        lib.gg_status.restype = ctypes.c_int
        lib.gg_status.argtypes = [vp]
        lib.gg_n.restype = i64
        lib.gg_n.argtypes = [vp]
        lib.gg_nnz.restype = i64
        lib.gg_nnz.argtypes = [vp]
        lib.gg_copy.restype = None
        lib.gg_copy.argtypes = [vp, vp, vp, vp]
        lib.gg_free.restype = None
        lib.gg_free.argtypes = [vp]
        lib.gg_splitmix_draw.restype = u64
        lib.gg_splitmix_draw.argtypes = [u64, u64]
        lib.gg_splitmix_next.restype = u64
        lib.gg_splitmix_next.argtypes = [ctypes.POINTER(u64)]
        _lib = lib
    return _lib


@dataclass
class CSR:
    """Symmetric CSR: offsets int64[n+1], targets int32[nnz], weights int32[nnz]."""
    n: int
    offsets: np.ndarray
    targets: np.ndarray
    weights: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.offsets[self.n])

    def offsets32(self) -> np.ndarray:
        if self.nnz > np.iinfo(np.int32).max:
            raise OverflowError("nnz does not fit int32 offsets")
        return self.offsets.astype(np.int32)


_ERR = {-1: "out of memory", -2: "merged weight exceeds int32", -3: "bad generator arguments"}


def _take(h, name: str) -> CSR:
    lib = _load()
    if not h:
        raise MemoryError("generator handle allocation failed")
    try:
        st = lib.gg_status(h)
        if st != 0:
            raise RuntimeError("graph generator failed: %s" % _ERR.get(st, st))
        n, nnz = lib.gg_n(h), lib.gg_nnz(h)
        off = np.empty(n + 1, dtype=np.int64)
        tgt = np.empty(max(nnz, 1), dtype=np.int32)
        w = np.empty(max(nnz, 1), dtype=np.int32)
        lib.gg_copy(h, off.ctypes.data, tgt.ctypes.data, w.ctypes.data)
        return CSR(int(n), off, tgt[:nnz], w[:nnz], name)
    finally:
        lib.gg_free(h)


def rmat(scale: int, edge_factor: int, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         wmax: int = 1, seed: int = 2, threads: int = 0, name: str = "") -> CSR:
    """R-MAT with 2^scale vertices and edge_factor * 2^scale draws."""
    draws = int(edge_factor) << int(scale)
    h = _load().gg_rmat(int(scale), draws, a, b, c, int(wmax), int(seed) & ((1 << 64) - 1),
                        int(threads))
    return _take(h, name or "rmat%d-%d" % (scale, edge_factor))


def sbm(n: int, k: int, p_in: float, p_out: float, seed: int = 1, threads: int = 0,
        name: str = "") -> CSR:
    """Planted-partition SBM: block of v is floor(v*k/n)."""
    h = _load().gg_sbm(int(n), int(k), float(p_in), float(p_out), int(seed) & ((1 << 64) - 1),
                       int(threads))
    return _take(h, name or "sbm%d-%d" % (n, k))


def sbm_blocks(n: int, k: int) -> np.ndarray:
    v = np.arange(n, dtype=np.int64)
    return ((v * k) // n).astype(np.int32)


def from_edges(n: int, edges: Iterable[Tuple[int, int]], weights: Optional[Sequence[int]] = None,
               name: str = "") -> CSR:
    """Symmetric CSR from undirected edges (u, v[, w]); a self-loop is stored once,
    repeated pairs are merged by summing their weights."""
    acc = {}
    edges = list(edges)
    if weights is None:
        weights = [1] * len(edges)
    for (u, v), w in zip(edges, weights):
        if not (0 <= u < n and 0 <= v < n) or w < 1:
            raise ValueError("bad edge %r" % ((u, v, w),))
        acc[(u, v)] = acc.get((u, v), 0) + int(w)
        if u != v:
            acc[(v, u)] = acc.get((v, u), 0) + int(w)
    keys = sorted(acc)
    off = np.zeros(n + 1, dtype=np.int64)
    for (u, _v) in keys:
        off[u + 1] += 1
    off = np.cumsum(off).astype(np.int64)
    tgt = np.array([v for (_u, v) in keys], dtype=np.int32)
    w = np.array([acc[k] for k in keys], dtype=np.int32)
    return CSR(n, off, tgt, w, name)


def cliques(k: int, s: int, bridges: Sequence[Tuple[int, int]] = (), name: str = "") -> CSR:
    """k disjoint complete graphs K_s (clique q on ids q*s .. q*s+s-1), optional extra edges."""
    edges = [(q * s + i, q * s + j) for q in range(k) for i in range(s) for j in range(i + 1, s)]
    edges += list(bridges)
    return from_edges(k * s, edges, name=name or "cliques%dx%d" % (k, s))


def union(graphs: Sequence[CSR], name: str = "") -> Tuple[CSR, np.ndarray]:
    """Disjoint union of CSRs (graph g's vertices shifted by the vertices before
    it) and the graph offsets int32[G+1] that mark each graph's vertex range."""
    sizes = np.array([g.n for g in graphs], dtype=np.int64)
    go = np.zeros(len(graphs) + 1, dtype=np.int64)
    go[1:] = np.cumsum(sizes)
    if go[-1] >= 2 ** 31:
        raise ValueError("union too large for int32 vertex ids")
    nnz = np.array([g.nnz for g in graphs], dtype=np.int64)
    eo = np.zeros(len(graphs) + 1, dtype=np.int64)
    eo[1:] = np.cumsum(nnz)
    off = np.zeros(int(go[-1]) + 1, dtype=np.int64)
    tgt = np.empty(int(eo[-1]), dtype=np.int32)
    w = np.empty(int(eo[-1]), dtype=np.int32)
    for i, g in enumerate(graphs):
        off[go[i]:go[i + 1] + 1] = g.offsets + eo[i]
        tgt[eo[i]:eo[i + 1]] = g.targets[:g.nnz] + np.int32(go[i])
        w[eo[i]:eo[i + 1]] = g.weights[:g.nnz]
    return CSR(int(go[-1]), off, tgt, w, name or "union%d" % len(graphs)), go.astype(np.int32)


def batch_sbm_specs(count: int, seed: int = 4, n_min: int = 200, n_max: int = 50_000,
                    ratio: float = 0.02, k_cap: int = 200):
    """Parameters of `count` planted-partition SBMs of uneven size: n log-uniform
    in [n_min, n_max], mean degree uniform in [8, 40], k uniform in 4..k_max
    (the largest k <= k_cap whose p_in stays <= 1), p_out = ratio * p_in.
    Graph g draws from SplitMix64 under key (seed << 32) | g."""
    specs = []
    for g in range(count):
        key = ((int(seed) << 32) | g) & ((1 << 64) - 1)
        u = [splitmix_draw(key, c) / 2.0 ** 64 for c in range(3)]
        n = int(round(math.exp(math.log(n_min) + u[0] * (math.log(n_max) - math.log(n_min)))))
        dbar = 8.0 + 32.0 * u[1]

        def p_in_of(k):
            s = n / k
            return dbar / ((s - 1.0) + ratio * (n - s))

        k_max = 4
        for k in range(4, k_cap + 1):
            if p_in_of(k) <= 1.0:
                k_max = k
        k = 4 + int(u[2] * (k_max - 3))
        k = min(k, k_max)
        p_in = p_in_of(k)
        specs.append({"n": n, "k": k, "p_in": p_in, "p_out": ratio * p_in,
                      "seed": (key + 1) & ((1 << 64) - 1)})
    return specs


def batch_sbm(count: int, seed: int = 4, threads: int = 0, **kw) -> Tuple[CSR, np.ndarray, list]:
    """The union of `count` SBMs from batch_sbm_specs, its graph offsets and the specs."""
    specs = batch_sbm_specs(count, seed, **kw)
    graphs = [sbm(sp["n"], sp["k"], sp["p_in"], sp["p_out"], seed=sp["seed"], threads=threads)
              for sp in specs]
    u, go = union(graphs, name="batch%d" % count)
    return u, go, specs


def perturb(csr: CSR, frac: float, seed: int = 9, name: str = "") -> CSR:
    """An edge batch applied to `csr`: a `frac` share of its undirected non-loop edges
    deleted and as many new unit-weight edges between random distinct vertices
    inserted (merged into existing pairs by summing), from numpy's seeded generator."""
    n = csr.n
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(csr.offsets))
    tgt = csr.targets[:csr.nnz].astype(np.int64)
    w = csr.weights[:csr.nnz].astype(np.int64)
    up = src < tgt
    loop = src == tgt
    u, v, ww = src[up], tgt[up], w[up]
    rng = np.random.default_rng(seed)
    k = int(frac * len(u))
    keep = np.ones(len(u), dtype=bool)
    if k:
        keep[rng.choice(len(u), size=k, replace=False)] = False
    a = rng.integers(0, n, size=k, dtype=np.int64)
    b = rng.integers(0, n, size=k, dtype=np.int64)
    ok = a != b
    a, b = np.minimum(a[ok], b[ok]), np.maximum(a[ok], b[ok])
    U = np.concatenate([u[keep], a, v[keep], b, src[loop]])
    V = np.concatenate([v[keep], b, u[keep], a, tgt[loop]])
    Wt = np.concatenate([ww[keep], np.ones(len(a), np.int64), ww[keep], np.ones(len(a), np.int64),
                         w[loop]])
    key = U * n + V
    order = np.argsort(key, kind="stable")
    key, Wt = key[order], Wt[order]
    first = np.ones(len(key), dtype=bool)
    first[1:] = key[1:] != key[:-1]
    idx = np.flatnonzero(first)
    wsum = np.add.reduceat(Wt, idx) if len(idx) else Wt[:0]
    if len(wsum) and wsum.max() >= 2 ** 31:
        raise ValueError("merged weight exceeds int32")
    ukey = key[idx]
    rows = ukey // n
    off = np.zeros(n + 1, dtype=np.int64)
    np.add.at(off, rows + 1, 1)
    off = np.cumsum(off)
    return CSR(n, off, (ukey % n).astype(np.int32), wsum.astype(np.int32),
               name or "%s+%g" % (csr.name, frac))


def serving_pool_specs(count: int, seed: int = 5, median: float = 2e5, sigma: float = 1.5,
                       cap: float = 5e7):
    """Parameters of a pool of `count` graphs for a serving workload: entry count
    log-normal (median, sigma) capped at `cap`; half SBMs (mean degree uniform in
    [8, 40], n = entries / degree, 4..200 blocks, p_out = 0.02 p_in), half R-MATs
    (scale ceil(log2(entries / 32)), entries / 2 draws).  Graph g draws from
    SplitMix64 under key (seed << 32) | g."""
    specs = []
    for g in range(count):
        key = ((int(seed) << 32) | g) & ((1 << 64) - 1)
        u = [splitmix_draw(key, c) / 2.0 ** 64 for c in range(5)]
        z = math.sqrt(-2.0 * math.log(max(u[0], 1e-300))) * math.cos(2.0 * math.pi * u[1])
        e = min(math.exp(math.log(median) + sigma * z), cap)
        e = max(e, 64.0)
        if u[2] < 0.5:
            scale = max(1, int(math.ceil(math.log2(e / 32.0))))
            ef = max(1, int(round(e / 2.0 / (1 << scale))))
            specs.append({"kind": "rmat", "scale": scale, "edge_factor": ef,
                          "seed": (key + 1) & ((1 << 64) - 1)})
        else:
            dbar = 8.0 + 32.0 * u[3]
            n = max(16, int(round(e / dbar)))
            k = 4 + int(u[4] * 197)

            def p_in_of(kk):
                sz = n / kk
                return dbar / ((sz - 1.0) + 0.02 * (n - sz))
            while k > 1 and (n / k < 2 or p_in_of(k) > 1.0):
                k -= 1
            k = max(k, 1)
            p_in = min(1.0, p_in_of(k))
            specs.append({"kind": "sbm", "n": n, "k": k, "p_in": p_in, "p_out": 0.02 * p_in,
                          "seed": (key + 1) & ((1 << 64) - 1)})
    return specs


def serving_pool(count: int, seed: int = 5, threads: int = 0, **kw) -> List[CSR]:
    """The graphs of serving_pool_specs."""
    out = []
    for g, sp in enumerate(serving_pool_specs(count, seed, **kw)):
        if sp["kind"] == "rmat":
            out.append(rmat(sp["scale"], sp["edge_factor"], seed=sp["seed"], threads=threads,
                            name="pool%d" % g))
        else:
            out.append(sbm(sp["n"], sp["k"], sp["p_in"], sp["p_out"], seed=sp["seed"],
                           threads=threads, name="pool%d" % g))
    return out


_RMAT = re.compile(r"^rmat(\d+)-(\d+)$")


def workload(name: str, seed: Optional[int] = None, threads: int = 0) -> CSR:
    """Named seeded workloads (see module docstring)."""
    if name == "sbm10k":
        return sbm(10000, 100, 0.05, 0.0005, seed=1 if seed is None else seed, threads=threads,
                   name=name)
    if name == "sbm1m":
        return sbm(1_000_000, 1000, 0.015, 0.000005, seed=1 if seed is None else seed,
                   threads=threads, name=name)
    if name == "rmat22":
        return rmat(22, 16, seed=2 if seed is None else seed, threads=threads, name=name)
    if name == "rmat24":
        return rmat(24, 64, wmax=8, seed=3 if seed is None else seed, threads=threads, name=name)
    m = _RMAT.match(name)
    if m:
        return rmat(int(m.group(1)), int(m.group(2)), seed=2 if seed is None else seed,
                    threads=threads, name=name)
    raise KeyError("unknown workload %r" % name)


def splitmix_stream(state: int, count: int) -> np.ndarray:
    """The first `count` outputs of the sequential SplitMix64 generator from `state`."""
    lib = _load()
    st = ctypes.c_uint64(state & ((1 << 64) - 1))
    return np.array([lib.gg_splitmix_next(ctypes.byref(st)) for _ in range(count)], dtype=np.uint64)


def splitmix_draw(key: int, ctr: int) -> int:
    return int(_load().gg_splitmix_draw(key & ((1 << 64) - 1), ctr & ((1 << 64) - 1)))
