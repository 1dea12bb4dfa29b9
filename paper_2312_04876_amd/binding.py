"""ctypes binding of ``liblouvain.so`` (the gfx950 Louvain library, see include/louvain.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides the device memory (input CSR, workspace, output
membership) and the stream; the library allocates no device memory.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblouvain.so")

DETERMINISTIC = 0
FAST = 1
COLOURED = 2
_MODES = {"deterministic": DETERMINISTIC, "det": DETERMINISTIC, "fast": FAST,
          "coloured": COLOURED, "colour": COLOURED}

OK, EINVAL, EOVERFLOW, ENOSPC, EHIP, ESTATE = 0, -1, -2, -3, -4, -5
MAX_PASSES = 64
MAX_ITERATIONS = 255

# Every symbol include/louvain.h declares.
EXPORTS = (
    "louvain_default_params", "louvain_workspace_size", "louvain_init", "louvain_move",
    "louvain_aggregate", "louvain_run", "louvain_membership", "louvain_level_labels",
    "louvain_level_graph", "louvain_move_trace", "louvain_reset", "louvain_total_weight",
    "louvain_get_stats", "louvain_kernel_stats", "louvain_destroy", "louvain_strerror",
    "louvain_batch_workspace_size", "louvain_init_batch", "louvain_batch_results",
    "louvain_set_membership", "louvain_run_noalloc",
)

# Bytes of the library's own device scratch array (louvain_run_noalloc).
NOALLOC_BYTES = 64 << 20


class CParams(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32), ("max_passes", ctypes.c_int32),
        ("max_iterations", ctypes.c_int32), ("prune", ctypes.c_int32),
        ("tolerance", ctypes.c_double), ("tolerance_drop", ctypes.c_double),
        ("aggregation_tolerance", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("round_bits", ctypes.c_int32), ("profile", ctypes.c_int32),
        ("hub_rows", ctypes.c_int32), ("hub_part_pairs", ctypes.c_int32),
        ("small_level", ctypes.c_int32),
    ]


class CStats(ctypes.Structure):
    _fields_ = [
        ("passes", ctypes.c_int32),
        ("iterations", ctypes.c_int32 * MAX_PASSES),
        ("vertices", ctypes.c_int32 * MAX_PASSES),
        ("entries", ctypes.c_int64 * MAX_PASSES),
        ("communities", ctypes.c_int32 * MAX_PASSES),
        ("dq_last", ctypes.c_double * MAX_PASSES),
        ("moves", ctypes.c_int64 * MAX_PASSES),
        ("processed", ctypes.c_int64 * MAX_PASSES),
        ("scanned", ctypes.c_int64 * MAX_PASSES),
        ("colours", ctypes.c_int32 * MAX_PASSES),
        ("ms_move", ctypes.c_double * MAX_PASSES),
        ("ms_aggregate", ctypes.c_double * MAX_PASSES),
        ("ms_other", ctypes.c_double * MAX_PASSES),
    ]

    def as_dict(self) -> Dict[str, list]:
        p = self.passes
        out: Dict[str, list] = {"passes": p}
        for name, _ in self._fields_[1:]:
            out[name] = list(getattr(self, name))[:p]
        return out


class CKernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int64),
                ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class LouvainError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s failed: %s (status %d)" % (where, strerror(code), code))


_lib = None


def load_library():
    """Load liblouvain.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblouvain.so is not built (run paper_2312_04876_amd.build.build())")
    # PyTorch first: its HIP runtime must be the one the library binds to.  Loaded the
    # other way round, the library would pull in a second HIP runtime from the system,
    # whose device enumeration fails beside PyTorch's, and whose streams and events are
    # not PyTorch's.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    lib.louvain_default_params.restype = None
    lib.louvain_default_params.argtypes = [P(CParams)]
    lib.louvain_workspace_size.restype = ctypes.c_int
    lib.louvain_workspace_size.argtypes = [i32, i64, i64, P(CParams), P(ctypes.c_size_t)]
    lib.louvain_init.restype = ctypes.c_int
    lib.louvain_init.argtypes = [P(vp), i32, i64, vp, vp, vp, vp, ctypes.c_size_t, P(CParams), vp]
    lib.louvain_move.restype = ctypes.c_int
    lib.louvain_move.argtypes = [vp, P(i32), P(dbl)]
    lib.louvain_aggregate.restype = ctypes.c_int
    lib.louvain_aggregate.argtypes = [vp, P(i32), P(i32)]
    lib.louvain_run.restype = ctypes.c_int
    lib.louvain_run.argtypes = [vp, vp, P(dbl), P(CStats)]
    lib.louvain_membership.restype = ctypes.c_int
    lib.louvain_membership.argtypes = [vp, vp]
    lib.louvain_level_labels.restype = ctypes.c_int
    lib.louvain_level_labels.argtypes = [vp, vp]
    lib.louvain_level_graph.restype = ctypes.c_int
    lib.louvain_level_graph.argtypes = [vp, P(vp), P(vp), P(vp), P(vp), P(i32), P(i32)]
    lib.louvain_move_trace.restype = ctypes.c_int
    lib.louvain_move_trace.argtypes = [vp, i32, vp, vp, vp, vp, P(i32)]
    lib.louvain_reset.restype = ctypes.c_int
    lib.louvain_reset.argtypes = [vp]
    lib.louvain_total_weight.restype = ctypes.c_int
    lib.louvain_total_weight.argtypes = [vp, P(i64)]
    lib.louvain_get_stats.restype = ctypes.c_int
    lib.louvain_get_stats.argtypes = [vp, P(CStats)]
    lib.louvain_kernel_stats.restype = ctypes.c_int
    lib.louvain_kernel_stats.argtypes = [vp, P(CKernelStat), i32, P(i32)]
    lib.louvain_batch_workspace_size.restype = ctypes.c_int
    lib.louvain_batch_workspace_size.argtypes = [i32, i32, i64, i64, P(CParams), P(ctypes.c_size_t)]
    lib.louvain_init_batch.restype = ctypes.c_int
    lib.louvain_init_batch.argtypes = [P(vp), i32, vp, i32, i64, vp, vp, vp, vp, ctypes.c_size_t,
                                       P(CParams), vp]
    lib.louvain_batch_results.restype = ctypes.c_int
    lib.louvain_batch_results.argtypes = [vp, vp, vp]
    lib.louvain_set_membership.restype = ctypes.c_int
    lib.louvain_set_membership.argtypes = [vp, vp]
    lib.louvain_run_noalloc.restype = ctypes.c_int
    lib.louvain_run_noalloc.argtypes = [i32, i64, vp, vp, vp, P(CParams), vp, P(dbl), P(CStats),
                                        vp]
    lib.louvain_destroy.restype = None
    lib.louvain_destroy.argtypes = [vp]
    lib.louvain_strerror.restype = ctypes.c_char_p
    lib.louvain_strerror.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load_library().louvain_strerror(int(code)).decode()


def _check(code: int, where: str):
    if code != OK:
        raise LouvainError(code, where)


def make_params(mode="deterministic", max_passes=10, max_iterations=20, prune=True,
                tolerance=0.01, tolerance_drop=10.0, aggregation_tolerance=0.8, seed=0,
                round_bits=-1, profile=False, hub_rows=0, hub_part_pairs=0,
                small_level=0) -> CParams:
    p = CParams()
    load_library().louvain_default_params(ctypes.byref(p))
    p.mode = _MODES[mode] if isinstance(mode, str) else int(mode)
    p.max_passes = int(max_passes)
    p.max_iterations = int(max_iterations)
    p.prune = 1 if prune else 0
    p.tolerance = float(tolerance)
    p.tolerance_drop = float(tolerance_drop)
    p.aggregation_tolerance = float(aggregation_tolerance)
    p.seed = int(seed) & ((1 << 64) - 1)
    p.round_bits = int(round_bits)
    p.profile = 1 if profile else 0
    p.hub_rows = int(hub_rows)
    p.hub_part_pairs = int(hub_part_pairs)
    p.small_level = int(small_level)
    return p


def workspace_bytes(n: int, nnz: int, total_weight: int = -1, params: Optional[CParams] = None) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().louvain_workspace_size(int(n), int(nnz), int(total_weight),
                                                 ctypes.byref(params) if params else None,
                                                 ctypes.byref(out)), "louvain_workspace_size")
    return int(out.value)


def batch_workspace_bytes(graphs: int, n: int, nnz: int, total_weight: int = -1,
                          params: Optional[CParams] = None) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().louvain_batch_workspace_size(int(graphs), int(n), int(nnz),
                                                       int(total_weight),
                                                       ctypes.byref(params) if params else None,
                                                       ctypes.byref(out)),
           "louvain_batch_workspace_size")
    return int(out.value)


class Louvain:
    """One graph (or a batch of independent graphs) resident on the GPU and its
    Louvain context.

    offsets, targets, weights: int32 CUDA tensors (CSR of a symmetric graph).
    graph_offsets (optional, int32 of G+1 entries, host or device): the CSR is
    the union of G independent graphs, graph g owning vertices
    [graph_offsets[g], graph_offsets[g+1]); each is run as if alone.
    The workspace is allocated here with torch; kernels run on ``stream`` (a
    torch.cuda.Stream, default: the current stream).
    """

    def __init__(self, offsets, targets, weights, stream=None, graph_offsets=None, **params):
        import torch
        self._torch = torch
        lib = load_library()
        for name, t in (("offsets", offsets), ("targets", targets), ("weights", weights)):
            if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("%s must be a contiguous int32 CUDA tensor" % name)
        self.n = int(offsets.numel()) - 1
        self.nnz = int(targets.numel())
        if self.n < 0 or int(weights.numel()) != self.nnz:
            raise ValueError("malformed CSR sizes")
        self.offsets, self.targets, self.weights = offsets, targets, weights
        self.device = offsets.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params = make_params(**params)
        W = int(weights.sum(dtype=torch.int64).item()) if self.nnz else 0
        self.graphs = None
        if graph_offsets is not None:
            go = torch.as_tensor(graph_offsets, dtype=torch.int32).to(self.device).contiguous()
            self.graphs = int(go.numel()) - 1
            self.graph_offsets = go
            nbytes = batch_workspace_bytes(self.graphs, self.n, self.nnz, W, self.params)
        else:
            nbytes = workspace_bytes(self.n, self.nnz, W, self.params)
        self.workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)
        self._ctx = ctypes.c_void_p(None)
        dummy = self.workspace.data_ptr()
        tp = targets.data_ptr() if self.nnz else dummy
        wp = weights.data_ptr() if self.nnz else dummy
        sp = ctypes.c_void_p(self.stream.cuda_stream)
        if self.graphs is None:
            rc = lib.louvain_init(ctypes.byref(self._ctx), self.n, self.nnz, offsets.data_ptr(), tp,
                                  wp, self.workspace.data_ptr(), nbytes, ctypes.byref(self.params),
                                  sp)
            _check(rc, "louvain_init")
        else:
            rc = lib.louvain_init_batch(ctypes.byref(self._ctx), self.graphs, go.data_ptr(), self.n,
                                        self.nnz, offsets.data_ptr(), tp, wp,
                                        self.workspace.data_ptr(), nbytes,
                                        ctypes.byref(self.params), sp)
            _check(rc, "louvain_init_batch")

    # -- lifecycle
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            load_library().louvain_destroy(self._ctx)
            self._ctx = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        _check(load_library().louvain_reset(self._ctx), "louvain_reset")
        self._warm = None

    def set_membership(self, labels):
        """Warm start: the first pass starts from `labels` (int32 CUDA tensor of n values in
        [0, n)), kept referenced here until the next reset.  None clears it."""
        torch = self._torch
        if labels is not None:
            if labels.dtype != torch.int32 or not labels.is_cuda or not labels.is_contiguous() \
                    or labels.numel() != self.n:
                raise ValueError("labels must be a contiguous int32 CUDA tensor of n values")
        self._warm = labels
        _check(load_library().louvain_set_membership(
            self._ctx, labels.data_ptr() if labels is not None else None),
            "louvain_set_membership")

    # -- the method
    def move(self) -> Tuple[int, float]:
        it, dq = ctypes.c_int32(0), ctypes.c_double(0.0)
        _check(load_library().louvain_move(self._ctx, ctypes.byref(it), ctypes.byref(dq)),
               "louvain_move")
        return int(it.value), float(dq.value)

    def aggregate(self) -> Tuple[int, bool]:
        nc, stop = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(load_library().louvain_aggregate(self._ctx, ctypes.byref(nc), ctypes.byref(stop)),
               "louvain_aggregate")
        return int(nc.value), bool(stop.value)

    def run(self, membership=None):
        """The whole method; returns (membership int32 tensor, Q, per-pass stats dict)."""
        torch = self._torch
        if membership is None:
            membership = torch.empty(max(self.n, 1), dtype=torch.int32, device=self.device)
        elif membership.dtype != torch.int32 or membership.device != self.device \
                or not membership.is_contiguous() or membership.numel() < self.n:
            raise ValueError("membership must be a contiguous int32 tensor of at least n values "
                             "on the graph's device")
        q = ctypes.c_double(0.0)
        st = CStats()
        _check(load_library().louvain_run(self._ctx, membership.data_ptr(), ctypes.byref(q),
                                          ctypes.byref(st)), "louvain_run")
        return membership[:self.n], float(q.value), st.as_dict()

    def batch_results(self):
        """After run() of a batch: (per-graph modularity list, per-graph community counts)."""
        import numpy as np
        q = np.zeros(self.graphs, dtype=np.float64)
        c = np.zeros(self.graphs, dtype=np.int32)
        _check(load_library().louvain_batch_results(self._ctx, q.ctypes.data, c.ctypes.data),
               "louvain_batch_results")
        return q.tolist(), c.tolist()

    def split_membership(self, membership):
        """Per-graph memberships (host numpy arrays, ids from 0) of a batch's union membership."""
        import numpy as np
        m = membership.cpu().numpy() if hasattr(membership, "cpu") else np.asarray(membership)
        go = self.graph_offsets.cpu().numpy()
        out = []
        for g in range(self.graphs):
            part = m[go[g]:go[g + 1]]
            out.append(part - part.min() if part.size else part.copy())
        return out

    def membership(self):
        out = self._torch.empty(max(self.n, 1), dtype=self._torch.int32, device=self.device)
        _check(load_library().louvain_membership(self._ctx, out.data_ptr()), "louvain_membership")
        return out[:self.n]

    def level_labels(self):
        n_level = self.level_size()
        out = self._torch.empty(max(n_level, 1), dtype=self._torch.int32, device=self.device)
        _check(load_library().louvain_level_labels(self._ctx, out.data_ptr()),
               "louvain_level_labels")
        return out[:n_level]

    def level_size(self) -> int:
        n = ctypes.c_int32(0)
        _check(load_library().louvain_level_graph(self._ctx, None, None, None, None,
                                                  ctypes.byref(n), None), "louvain_level_graph")
        return int(n.value)

    def _view(self, ptr: int, count: int, dtype):
        """Tensor view of `count` elements at device address ptr (inside the workspace or
        one of the input tensors)."""
        torch = self._torch
        esz = torch.tensor([], dtype=dtype).element_size()
        for base in (self.workspace, self.offsets, self.targets, self.weights):
            b0 = base.data_ptr()
            nb = base.numel() * base.element_size()
            if b0 <= ptr and ptr + count * esz <= b0 + nb:
                raw = base.view(torch.uint8).reshape(-1) if base.dtype != torch.uint8 else base
                start = ptr - b0
                return raw[start:start + count * esz].view(dtype)
        raise RuntimeError("pointer outside the context's buffers")

    def level_graph(self):
        """Copies of the current level: (offsets, degree or None, targets, weights) on the GPU."""
        torch = self._torch
        off, deg, tgt, w = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        n, wb = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(load_library().louvain_level_graph(self._ctx, ctypes.byref(off), ctypes.byref(deg),
                                                  ctypes.byref(tgt), ctypes.byref(w),
                                                  ctypes.byref(n), ctypes.byref(wb)),
               "louvain_level_graph")
        n = int(n.value)
        offsets = self._view(off.value, n + 1, torch.int32).clone()
        cap = int(offsets[n].item()) if n >= 0 else 0
        degree = self._view(deg.value, n, torch.int32).clone() if deg.value else None
        targets = self._view(tgt.value, cap, torch.int32).clone() if cap else \
            torch.empty(0, dtype=torch.int32, device=self.device)
        wdt = torch.int32 if wb.value == 4 else torch.int64
        weights = self._view(w.value, cap, wdt).clone() if cap else \
            torch.empty(0, dtype=wdt, device=self.device)
        return offsets, degree, targets, weights

    def total_weight(self) -> int:
        W = ctypes.c_int64(0)
        _check(load_library().louvain_total_weight(self._ctx, ctypes.byref(W)),
               "louvain_total_weight")
        return int(W.value)

    def move_trace(self) -> Dict[str, list]:
        import numpy as np
        m = MAX_ITERATIONS + 1
        hi = np.zeros(m, dtype=np.int64)
        lo = np.zeros(m, dtype=np.uint64)
        mv = np.zeros(m, dtype=np.int64)
        pr = np.zeros(m, dtype=np.int64)
        cnt = ctypes.c_int32(0)
        _check(load_library().louvain_move_trace(self._ctx, m, hi.ctypes.data, lo.ctypes.data,
                                                 mv.ctypes.data, pr.ctypes.data,
                                                 ctypes.byref(cnt)), "louvain_move_trace")
        k = int(cnt.value)
        sums = [(int(hi[i]) << 64) | int(lo[i]) for i in range(k)]
        return {"sumN": sums, "moves": mv[:k].tolist(), "processed": pr[:k].tolist()}

    def stats(self) -> Dict[str, list]:
        st = CStats()
        _check(load_library().louvain_get_stats(self._ctx, ctypes.byref(st)), "louvain_get_stats")
        return st.as_dict()

    def kernel_stats(self) -> List[Dict[str, float]]:
        buf = (CKernelStat * 64)()
        cnt = ctypes.c_int32(0)
        _check(load_library().louvain_kernel_stats(self._ctx, buf, 64, ctypes.byref(cnt)),
               "louvain_kernel_stats")
        return [{"name": buf[i].name.decode(), "launches": int(buf[i].launches),
                 "ms": float(buf[i].ms), "bytes": float(buf[i].bytes)}
                for i in range(min(int(cnt.value), 64))]


def louvain(offsets, targets, weights, **params):
    """One-shot Louvain: returns (membership int32 CUDA tensor, modularity, stats)."""
    ctx = Louvain(offsets, targets, weights, **params)
    try:
        return ctx.run()
    finally:
        ctx.close()


def louvain_noalloc(offsets, targets, weights, membership, stream=None, **params):
    """louvain_run_noalloc: the whole method with the library's own device scratch array
    as the workspace (no device memory allocated here or in the library).  membership:
    a caller-allocated contiguous int32 CUDA tensor of at least n values.  Returns
    (Q, per-pass stats dict)."""
    import torch
    lib = load_library()
    for name, t in (("offsets", offsets), ("targets", targets), ("weights", weights),
                    ("membership", membership)):
        if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("%s must be a contiguous int32 CUDA tensor" % name)
    n = int(offsets.numel()) - 1
    nnz = int(targets.numel())
    if n < 0 or int(weights.numel()) != nnz or int(membership.numel()) < n:
        raise ValueError("malformed CSR or membership sizes")
    prm = make_params(**params)
    if stream is None:
        stream = torch.cuda.current_stream(offsets.device)
    q = ctypes.c_double(0.0)
    st = CStats()
    _check(lib.louvain_run_noalloc(n, nnz, offsets.data_ptr(), targets.data_ptr() if nnz else
                                   offsets.data_ptr(), weights.data_ptr() if nnz else
                                   offsets.data_ptr(), ctypes.byref(prm), membership.data_ptr(),
                                   ctypes.byref(q), ctypes.byref(st),
                                   ctypes.c_void_p(stream.cuda_stream)), "louvain_run_noalloc")
    return float(q.value), st.as_dict()
