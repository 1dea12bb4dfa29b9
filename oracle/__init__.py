"""Louvain oracle: plain serial CPU reference of GVE-Louvain (arXiv 2312.04876).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; it shares no code with
the GPU path (``paper_2312_04876_amd``) and neither imports the other.

The arithmetic lives in ``louvain_oracle.c`` (built with gcc into
``liblouvain_oracle.so``); this module only marshals numpy arrays.  Every
function cites the passage of the paper it follows:

* ``modularity``        -- Eq. 1 (second form), exact num/den then one FP64 divide
* ``move_gain``         -- Eq. 2, scaled by W^2/2 to an exact integer
* ``move``              -- Alg. 2 (louvainMove + scanCommunities), seq and sync modes
* ``renumber``          -- Alg. 1 (renumber communities), order preserving
* ``community_vertices``-- Alg. 3 (countCommunityVertices, exclusiveScan, fill)
* ``aggregate``         -- Alg. 3 (super-vertex graph), canonical CSR output
* ``louvain``           -- Alg. 1 (the pass loop), all in C
* ``louvain_trace``     -- Alg. 1 driven from Python over the C steps, keeping
                           every level for per-pass comparisons

Parity pins live in ``tests/test_oracle_*.py``.  The synchronous iteration
(``mode="sync"``) is not in the paper; its semantics (hashed rounds, each
deciding against the state at the start of the round, min-label rule for
singleton-to-singleton moves) are pinned by hand-worked cases, invariants and a
brute-force recomputation of whole iterations on small graphs
(``tests/test_oracle_sync_bruteforce.py``).  The colour-ordered iteration
(``mode="colour"``, one synchronous round per colour class of a greedy colouring
in hashed priority order) is pinned by the colouring's defining properties, a
hand-worked case, its reduction to the sequential sweep on a clique and the same
brute force with colour classes as rounds.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "louvain_oracle.c")
_LIB = os.path.join(_HERE, "liblouvain_oracle.so")

SYNC = 0
SEQ = 1
COLOUR = 2
_MODES = {"sync": SYNC, "seq": SEQ, "colour": COLOUR}


_LIB_TIMING = os.path.join(_HERE, "liblouvain_oracle_omp.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction, one thread)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
             "-Wall", "-Wextra", "-Wno-unused-parameter", "-Wno-unknown-pragmas", _SRC,
             "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def build_timing() -> str:
    """Compile the CPU-baseline build of the same source on the machine that will run it:
    -O3 -march=native, OpenMP on (the decisions of a synchronous round run on every
    thread; the results are those of the serial build), still no contraction."""
    tmp = _LIB_TIMING + ".tmp%d" % os.getpid()
    subprocess.check_call(
        ["gcc", "-std=gnu11", "-O3", "-march=native", "-fopenmp", "-ffp-contract=off", "-fPIC",
         "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter", _SRC, "-o", tmp])
    os.replace(tmp, _LIB_TIMING)
    return _LIB_TIMING


_lib = None
_lib_timing = None


def timing_library():
    """The -O3 -march=native OpenMP build (compiled here on first use); pass it as `lib=`
    to move() or louvain()."""
    global _lib_timing
    if _lib_timing is None:
        _lib_timing = _bind(ctypes.CDLL(build_timing()))
    return _lib_timing


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    """Argument and result types of the oracle's C entry points on a loaded build."""
    i32, i64, u64, dbl, vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                              ctypes.c_double, ctypes.c_void_p)
    lib.oracle_vertex_weights.restype = i64
    lib.oracle_vertex_weights.argtypes = [i32, vp, vp, vp]
    lib.oracle_modularity_exact.restype = ctypes.c_int
    lib.oracle_modularity_exact.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.oracle_modularity.restype = dbl
    lib.oracle_modularity.argtypes = [i32, vp, vp, vp, vp]
    lib.oracle_move_gain.restype = ctypes.c_int
    lib.oracle_move_gain.argtypes = [i32, vp, vp, vp, vp, i32, i32, vp, vp]
    lib.oracle_move.restype = i32
    lib.oracle_move.argtypes = [i32, i32, vp, vp, vp, vp, i64, vp, vp, vp, vp,
                                i32, dbl, i32, u64, i32, i32, vp, vp, vp, vp]
    lib.oracle_renumber.restype = i32
    lib.oracle_renumber.argtypes = [i32, vp]
    lib.oracle_community_vertices.restype = None
    lib.oracle_community_vertices.argtypes = [i32, vp, i32, vp, vp]
    lib.oracle_aggregate.restype = i64
    lib.oracle_aggregate.argtypes = [i32, vp, vp, vp, vp, i32, vp, vp, vp, i64]
    lib.oracle_louvain.restype = i32
    lib.oracle_louvain.argtypes = [i32, i32, i32, i32, dbl, dbl, dbl, u64, i32, i32, vp,
                                   vp, vp, vp, vp, vp, vp, vp]
    lib.oracle_colour.restype = i32
    lib.oracle_colour.argtypes = [i32, vp, vp, u64, i32, vp]
    lib.oracle_move_coloured.restype = i32
    lib.oracle_move_coloured.argtypes = [i32, vp, vp, vp, vp, i64, vp, vp, vp, vp, i32, dbl,
                                         i32, vp, i32, vp, vp, vp, vp]
    lib.oracle_louvain_from.restype = i32
    lib.oracle_louvain_from.argtypes = [i32, i32, i32, i32, dbl, dbl, dbl, u64, i32, i32,
                                        vp, vp, vp, vp, vp, vp, vp, vp, vp]
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _join128(hi: int, lo: int) -> int:
    return (int(hi) << 64) | (int(lo) & ((1 << 64) - 1))


@dataclass
class Graph:
    """A CSR graph in the oracle's layout: int64 offsets, int32 targets, int64 weights."""
    n: int
    offsets: np.ndarray
    targets: np.ndarray
    weights: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.offsets[self.n])


def as_graph(offsets, targets, weights) -> Graph:
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    tgt = np.ascontiguousarray(np.asarray(targets, dtype=np.int32))
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.int64))
    n = len(off) - 1
    if n < 0 or off[0] != 0 or len(tgt) != off[n] or len(w) != off[n]:
        raise ValueError("malformed CSR")
    return Graph(n, off, tgt, w)


def vertex_weights(g: Graph):
    """K_i = row sums and W = sum_i K_i (Alg. 1, vertexWeights)."""
    K = np.empty(max(g.n, 1), dtype=np.int64)
    W = _load().oracle_vertex_weights(g.n, _p(g.offsets), _p(g.weights), _p(K))
    return K[:g.n], int(W)


def _labels(g: Graph, C) -> np.ndarray:
    C = np.ascontiguousarray(np.asarray(C, dtype=np.int32))
    if C.shape != (g.n,) or (g.n and (C.min() < 0 or C.max() >= g.n)):
        raise ValueError("labels must be int32[n] in [0, n)")
    return C


def modularity_exact(g: Graph, C):
    """Eq. 1 (second form) as the exact pair (sigma_tot*W - sum Sigma_c^2, W^2)."""
    C = _labels(g, C)
    nh, nl, dh, dl = (ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_int64(), ctypes.c_uint64())
    rc = _load().oracle_modularity_exact(g.n, _p(g.offsets), _p(g.targets), _p(g.weights), _p(C),
                                         ctypes.byref(nh), ctypes.byref(nl),
                                         ctypes.byref(dh), ctypes.byref(dl))
    if rc != 0:
        raise RuntimeError("oracle_modularity_exact failed")
    return _join128(nh.value, nl.value), _join128(dh.value, dl.value)


def modularity(g: Graph, C) -> float:
    """Eq. 1 (second form) in FP64: (double)num / (double)den, 0 for an edgeless graph."""
    C = _labels(g, C)
    return float(_load().oracle_modularity(g.n, _p(g.offsets), _p(g.targets), _p(g.weights), _p(C)))


def move_gain(g: Graph, C, i: int, c: int) -> int:
    """Eq. 2 scaled by W^2/2: the exact integer N with dQ = 2N/W^2."""
    C = _labels(g, C)
    hi, lo = ctypes.c_int64(), ctypes.c_uint64()
    rc = _load().oracle_move_gain(g.n, _p(g.offsets), _p(g.targets), _p(g.weights), _p(C),
                                  int(i), int(c), ctypes.byref(hi), ctypes.byref(lo))
    if rc != 0:
        raise RuntimeError("oracle_move_gain failed")
    return _join128(hi.value, lo.value)


@dataclass
class MoveState:
    """State of one level during local moving (Alg. 1 per-pass reset)."""
    K: np.ndarray
    W: int
    Sigma: np.ndarray
    C: np.ndarray
    size: np.ndarray
    active: np.ndarray

    @staticmethod
    def fresh(g: Graph) -> "MoveState":
        K, W = vertex_weights(g)
        return MoveState(K=K, W=W, Sigma=K.copy(), C=np.arange(g.n, dtype=np.int32),
                         size=np.ones(g.n, dtype=np.int32), active=np.ones(g.n, dtype=np.uint8))

    @staticmethod
    def warm(g: Graph, labels) -> "MoveState":
        """Start from the partition `labels` (each in [0, n)): Sigma_c and |c| of it."""
        K, W = vertex_weights(g)
        C = np.asarray(labels, dtype=np.int32).copy()
        if C.shape != (g.n,) or (g.n and (C.min() < 0 or C.max() >= g.n)):
            raise ValueError("labels must be n values in [0, n)")
        Sigma = np.zeros(g.n, dtype=np.int64)
        size = np.zeros(g.n, dtype=np.int32)
        for i in range(g.n):
            Sigma[C[i]] += int(K[i])
            size[C[i]] += 1
        return MoveState(K=K, W=W, Sigma=Sigma, C=C, size=size,
                         active=np.ones(g.n, dtype=np.uint8))


@dataclass
class MoveTrace:
    iterations: int
    sumN: List[int] = field(default_factory=list)
    moves: List[int] = field(default_factory=list)
    processed: List[int] = field(default_factory=list)


def colour(g: Graph, seed: int = 0, pass_index: int = 0) -> Tuple[np.ndarray, int]:
    """Greedy colouring in decreasing hash priority (Jones-Plassmann's result):
    (colour int32[n], number of colours)."""
    col = np.zeros(max(g.n, 1), dtype=np.int32)
    k = _load().oracle_colour(g.n, _p(g.offsets), _p(g.targets), int(seed) & ((1 << 64) - 1),
                              int(pass_index), _p(col))
    if k < 0:
        raise RuntimeError("oracle_colour failed")
    return col[:g.n].copy(), int(k)


def move(g: Graph, st: MoveState, mode: str = "seq", tau: float = 0.01, max_iter: int = 20,
         prune: bool = True, seed: int = 0, pass_index: int = 0,
         sample_bits: int = 1, lib=None) -> MoveTrace:
    """Alg. 2 (louvainMove) in place on ``st``; returns sweeps run and per-sweep traces.

    ``seed``, ``pass_index`` and ``sample_bits`` split a synchronous iteration into
    2**sample_bits rounds (a hash of the vertex, iteration and pass picks the round).
    Mode "colour" uses one synchronous round per colour class of ``colour``."""
    m = max(int(max_iter), 1)
    hi = np.zeros(m, dtype=np.int64)
    lo = np.zeros(m, dtype=np.uint64)
    mv = np.zeros(m, dtype=np.int32)
    pr = np.zeros(m, dtype=np.int32)
    for a, dt in ((st.K, np.int64), (st.Sigma, np.int64), (st.C, np.int32), (st.size, np.int32),
                  (st.active, np.uint8)):
        assert a.dtype == dt and a.flags.c_contiguous and a.shape == (g.n,)
    lib = lib or _load()
    if mode == "colour":
        col, k = colour(g, seed, pass_index)
        col = np.ascontiguousarray(col if g.n else np.zeros(1, dtype=np.int32))
        l = lib.oracle_move_coloured(g.n, _p(g.offsets), _p(g.targets), _p(g.weights),
                                         _p(st.K), st.W, _p(st.Sigma), _p(st.C), _p(st.size),
                                         _p(st.active), 1 if prune else 0, float(tau),
                                         int(max_iter), _p(col), k, _p(hi), _p(lo), _p(mv), _p(pr))
    else:
        l = lib.oracle_move(_MODES[mode], g.n, _p(g.offsets), _p(g.targets), _p(g.weights),
                                _p(st.K), st.W, _p(st.Sigma), _p(st.C), _p(st.size),
                                _p(st.active), 1 if prune else 0, float(tau), int(max_iter),
                                int(seed) & ((1 << 64) - 1), int(pass_index), int(sample_bits),
                                _p(hi), _p(lo), _p(mv), _p(pr))
    if l < 0:
        raise RuntimeError("oracle_move failed")
    return MoveTrace(iterations=int(l), sumN=[_join128(hi[k], lo[k]) for k in range(l)],
                     moves=[int(x) for x in mv[:l]], processed=[int(x) for x in pr[:l]])


def renumber(C):
    """Alg. 1 renumbering: dense ids in label order. Returns (new labels, count)."""
    C = np.ascontiguousarray(np.array(C, dtype=np.int32))
    nc = _load().oracle_renumber(len(C), _p(C))
    if nc < 0:
        raise ValueError("labels out of range")
    return C, int(nc)


def community_vertices(C, nc: int):
    """Alg. 3 community-vertex CSR: (offsets int64[nc+1], members int32[n])."""
    C = np.ascontiguousarray(np.asarray(C, dtype=np.int32))
    coff = np.zeros(nc + 1, dtype=np.int64)
    members = np.zeros(max(len(C), 1), dtype=np.int32)
    _load().oracle_community_vertices(len(C), _p(C), int(nc), _p(coff), _p(members))
    return coff, members[:len(C)]


def aggregate(g: Graph, C, nc: int) -> Graph:
    """Alg. 3 super-vertex graph of the dense membership C, canonical CSR."""
    C = _labels(g, C) if g.n else np.zeros(0, dtype=np.int32)
    cap = max(g.nnz, 1)
    off = np.zeros(nc + 1, dtype=np.int64)
    tgt = np.zeros(cap, dtype=np.int32)
    w = np.zeros(cap, dtype=np.int64)
    got = _load().oracle_aggregate(g.n, _p(g.offsets), _p(g.targets), _p(g.weights), _p(C),
                                   int(nc), _p(off), _p(tgt), _p(w), cap)
    if got < 0:
        raise RuntimeError("oracle_aggregate failed")
    return Graph(int(nc), off, tgt[:got], w[:got])  # views: no second copy of a large level


@dataclass
class Params:
    """The paper's parameter choices (Section 4.1); max_passes is not given there (10 here)."""
    mode: str = "seq"
    max_passes: int = 10
    max_iterations: int = 20
    prune: bool = True
    tolerance: float = 0.01
    tolerance_drop: float = 10.0
    aggregation_tolerance: float = 0.8
    seed: int = 0          # round hash / colouring priority (not in the paper)
    sample_bits: int = 1   # a synchronous iteration runs in 2**sample_bits rounds


def louvain(g: Graph, params: Optional[Params] = None, initial=None, lib=None):
    """Alg. 1 entirely in C. Returns (membership int32[n], Q, records dict).
    ``initial``: labels of a partition the first pass starts from (a warm start).
    ``lib``: another build of the oracle (timing_library()); the serial build by default."""
    p = params or Params()
    mp = max(p.max_passes, 1)
    memb = np.zeros(max(g.n, 1), dtype=np.int32)
    q = ctypes.c_double(0.0)
    it = np.zeros(mp, dtype=np.int32)
    nv = np.zeros(mp, dtype=np.int32)
    nc = np.zeros(mp, dtype=np.int32)
    init = None
    if initial is not None:
        init = np.ascontiguousarray(initial, dtype=np.int32)
        if init.shape != (g.n,) or (g.n and (init.min() < 0 or init.max() >= g.n)):
            raise ValueError("initial labels must be n values in [0, n)")
    passes = (lib or _load()).oracle_louvain_from(_MODES[p.mode], p.max_passes, p.max_iterations,
                                         1 if p.prune else 0, p.tolerance, p.tolerance_drop,
                                         p.aggregation_tolerance, int(p.seed) & ((1 << 64) - 1),
                                         int(p.sample_bits), g.n, _p(g.offsets), _p(g.targets),
                                         _p(g.weights), _p(init) if init is not None else None,
                                         _p(memb), ctypes.byref(q), _p(it), _p(nv), _p(nc))
    if passes < 0:
        raise RuntimeError("oracle_louvain failed")
    rec = {"passes": int(passes), "iterations": it[:passes].tolist(),
           "vertices": nv[:passes].tolist(), "communities": nc[:passes].tolist()}
    return memb[:g.n].copy(), float(q.value), rec


@dataclass
class PassRecord:
    level: Graph                 # G' at the start of the pass
    trace: MoveTrace             # local-moving sweeps of the pass
    raw_labels: np.ndarray       # C' after local moving (labels are vertex ids of G')
    communities: int             # distinct labels in C'
    stop: str                    # "" | "converged" | "low-shrink"
    next_level: Optional[Graph]  # G'' when the pass aggregated
    top: np.ndarray              # top-level membership C after the pass


def louvain_trace(g: Graph, params: Optional[Params] = None, initial=None):
    """Alg. 1 driven step by step; returns (membership, Q, [PassRecord]).
    ``initial``: labels of a partition the first pass starts from (a warm start)."""
    p = params or Params()
    top = np.arange(g.n, dtype=np.int32)
    level = g
    tau = p.tolerance
    broke = False
    recs: List[PassRecord] = []
    Cp = np.zeros(0, dtype=np.int32)
    for pi in range(p.max_passes):
        st = MoveState.warm(level, initial) if (pi == 0 and initial is not None) \
            else MoveState.fresh(level)
        tr = move(level, st, p.mode, tau, p.max_iterations, p.prune, p.seed, pi, p.sample_bits)
        Cp = st.C.copy()
        ncomm = int(len(np.unique(Cp))) if level.n else 0
        rec = PassRecord(level=level, trace=tr, raw_labels=Cp.copy(), communities=ncomm,
                         stop="", next_level=None, top=top)
        recs.append(rec)
        if tr.iterations <= 1:
            rec.stop, broke = "converged", True
            break
        if float(ncomm) / float(level.n) > p.aggregation_tolerance:
            rec.stop, broke = "low-shrink", True
            break
        Cp, nc = renumber(Cp)
        top = Cp[top]
        nxt = aggregate(level, Cp, nc)
        rec.next_level = nxt
        rec.top = top.copy()
        level = nxt
        tau = tau / p.tolerance_drop
    if broke:
        top = Cp[top]
        recs[-1].top = top.copy()
    memb, _ = renumber(top) if g.n else (top, 0)
    return memb, modularity(g, memb), recs
