"""Autotuner for the scheduling knobs of the library.

Three knobs decide how rows are scheduled (deterministic runs are
bit-identical under every setting):

* ``hub_rows``: rows (and, in aggregation, communities) longer than this take
  the hub path, whose rows are counting-sorted into hash partitions, instead of
  one 512-thread workgroup with an LDS table;
* ``hub_part_pairs``: pairs per hash partition of a hub row in local moving;
* ``small_level``: a level (in a batch, a graph's part of it) of at most this
  many vertices is moved by one wavefront in one launch instead of by the
  degree bins' rounds.  In deterministic mode this moves work between kernels
  like the other two knobs; in fast mode it also decides the order of the
  moves (vertex order instead of thousands of concurrent decisions), which is
  what keeps the coarse levels of small graphs from herding, so fast mode keeps
  its built-in value and is tuned over the first two knobs only.

:func:`tune` times every candidate setting on the caller's own graph (or batch
union) with inputs resident on the GPU and returns the fastest, so a workload
picks its own thresholds instead of the built-in ones.  Results can be kept in
a JSON cache keyed by a coarse signature of the graph.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Iterable, List, Optional, Tuple

from .binding import Louvain

HUB_ROWS = (2048, 4096, 8192)
HUB_PART_PAIRS = (1024, 2048)
SMALL_LEVELS = (-1, 256, 1024)
WIDE_LDS_ROWS = 4096  # the hub threshold is clamped to this with 8-byte accumulators


def signature(offsets, weights, graph_offsets=None, **params) -> str:
    """A coarse key for the cache: sizes (rounded to powers of two), the degree
    histogram in octaves, the weight width, the mode and the batch size."""
    import torch
    n = int(offsets.numel()) - 1
    nnz = int(weights.numel())
    deg = (offsets[1:] - offsets[:-1]).to(torch.int64)
    hist = torch.bincount(torch.floor(torch.log2(deg.clamp(min=1).double())).to(torch.int64),
                          minlength=24)[:24]
    share = (hist.double() / max(n, 1) * 100).round().to(torch.int64).tolist()
    wide = int(weights.to(torch.int64).sum().item()) >= (1 << 31)
    g = 0 if graph_offsets is None else len(graph_offsets) - 1
    return "n2^%d-e2^%d-%s-%s-g%d-%s" % (max(n, 1).bit_length(), max(nnz, 1).bit_length(),
                                         "wide" if wide else "narrow", params.get("mode", "det"),
                                         g, ".".join(str(x) for x in share))


def candidates(wide: bool) -> List[Tuple[int, int]]:
    rows = sorted({min(r, WIDE_LDS_ROWS) if wide else r for r in HUB_ROWS})
    return [(r, p) for r in rows for p in HUB_PART_PAIRS]


def tune(offsets, targets, weights, graph_offsets=None, runs: int = 2, warmup: int = 1,
         cache_path: Optional[str] = None, stream=None, **params) -> Dict:
    """Time every candidate (hub_rows, hub_part_pairs) over `runs` whole runs after
    `warmup` untimed ones, then (deterministic mode) every small_level with the best
    of them; returns
    {"hub_rows", "hub_part_pairs", "small_level", "ms", "table", "seconds",
    "signature", "cached"}.  `params` are the run's other parameters."""
    import torch
    key = signature(offsets, weights, graph_offsets, **params)
    cache: Dict = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            hit = dict(cache[key])
            hit["cached"] = True
            return hit
    wide = int(weights.to(torch.int64).sum().item()) >= (1 << 31)
    t_start = time.perf_counter()
    table = []
    n = int(offsets.numel()) - 1
    memb = torch.empty(max(n, 1), dtype=torch.int32, device=offsets.device)

    def timed(rows, pairs, small):
        ctx = Louvain(offsets, targets, weights, stream=stream, graph_offsets=graph_offsets,
                      hub_rows=rows, hub_part_pairs=pairs, small_level=small, **params)
        try:
            for _ in range(warmup):
                ctx.reset()
                ctx.run(memb)
            times = []
            for _ in range(max(runs, 1)):
                ctx.reset()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.run(memb)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
        finally:
            ctx.close()
        table.append({"hub_rows": rows, "hub_part_pairs": pairs, "small_level": small,
                      "ms": min(times) * 1e3})

    for rows, pairs in candidates(wide):
        timed(rows, pairs, 0)
    best = min(table, key=lambda r: r["ms"])
    # the built-in small_level (0) is 1024 in fast mode and none (-1) in deterministic
    # mode; only deterministic mode, where it cannot change a result, is tuned over it
    fast = params.get("mode") == "fast"
    builtin = 1024 if fast else -1
    if not fast:
        for small in SMALL_LEVELS:
            if small != builtin:
                timed(best["hub_rows"], best["hub_part_pairs"], small)
        best = min(table, key=lambda r: r["ms"])
    out = {"hub_rows": best["hub_rows"], "hub_part_pairs": best["hub_part_pairs"],
           "small_level": best["small_level"] or builtin, "ms": best["ms"], "table": table,
           "seconds": time.perf_counter() - t_start, "signature": key, "cached": False}
    if cache_path:
        cache[key] = out
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return out


def tuned_params(result: Dict) -> Dict[str, int]:
    return {"hub_rows": int(result["hub_rows"]), "hub_part_pairs": int(result["hub_part_pairs"]),
            "small_level": int(result.get("small_level", 0))}
