"""Digests that let full-size parity compare large results without storing them.

`labels_digest` hashes a label array as stored.  `graph_digest` summarises a CSR
level graph independently of the order of the entries inside each row and of
any holes between rows (the GPU writes aggregated rows in a free order into a
holey CSR; the oracle writes them sorted and dense): each entry (row, target,
weight) is mixed to 64 bits with the SplitMix64 output function (Steele, Lea
and Flood 2014) and the mixes are summed modulo 2^64, next to the number of
rows, the number of entries, the total weight and a sum of mixed (row, length)
pairs.  No value here comes from the method's arithmetic.
"""
import hashlib

import numpy as np

_M = np.uint64(0xFFFFFFFFFFFFFFFF)


def _mix(z):
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def labels_digest(labels) -> str:
    return hashlib.sha256(np.ascontiguousarray(labels, dtype=np.int32).tobytes()).hexdigest()


def graph_digest(offsets, degree, targets, weights, chunk_rows=1 << 20) -> dict:
    """offsets int[n+1] (or int[n] with degree), degree int[n] or None (dense CSR),
    targets int32, weights int (numpy arrays)."""
    off = np.asarray(offsets, dtype=np.int64)
    if degree is None:
        n = len(off) - 1
        deg = np.diff(off)
    else:
        deg = np.asarray(degree, dtype=np.int64)
        n = len(deg)
    ent = np.uint64(0)
    rows_sum = np.uint64(0)
    total_w = 0
    count = 0
    with np.errstate(over="ignore"):
        for r0 in range(0, n, chunk_rows):
            r1 = min(n, r0 + chunk_rows)
            d = deg[r0:r1]
            rid = np.arange(r0, r1, dtype=np.uint64)
            rows_sum += np.sum(_mix((rid << np.uint64(32)) | d.astype(np.uint64)), dtype=np.uint64)
            tot = int(d.sum())
            if tot == 0:
                continue
            rows = np.repeat(np.arange(r0, r1, dtype=np.int64), d)
            start = np.repeat(off[r0:r1], d)
            first = np.repeat(np.cumsum(d) - d, d)
            pos = start + (np.arange(tot, dtype=np.int64) - first)
            t = np.asarray(targets[pos], dtype=np.uint64)
            w = np.asarray(weights[pos], dtype=np.int64)
            key = _mix((rows.astype(np.uint64) << np.uint64(32)) | t)
            ent += np.sum(_mix(key + w.astype(np.uint64)), dtype=np.uint64)
            total_w += int(w.sum())
            count += tot
    return {"n": int(n), "entries": int(count), "weight": int(total_w),
            "rows": "%016x" % int(rows_sum), "entry_mix": "%016x" % int(ent)}
