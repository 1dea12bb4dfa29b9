"""Write tests/golden/reference.json: oracle results on the seeded workloads.

Calls only the oracle (and the seeded generators for its inputs).  For each
workload it records the sequential-mode modularity (the quality reference of
the GPU fast mode), the synchronous-mode and colour-ordered results
(membership digest, Q, iterations and communities per pass; the bit-exact
references of the GPU deterministic and colour-ordered modes), plus the
spread of sequential-mode Q over random vertex relabellings, which calibrates
the fast-mode tolerance.

Usage: python tests/golden/make_golden.py [--only colour] [workload ...]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "reference.json")
DEFAULT = ["sbm10k", "rmat16-16", "rmat18-16", "rmat22", "sbm1m"]


def digest(memb: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(memb, dtype=np.int32).tobytes()).hexdigest()


def relabel(csr, perm):
    """The same graph with vertex v renamed perm[v] (rows rebuilt, sorted by target)."""
    n = csr.n
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    deg = np.diff(csr.offsets)
    new_deg = deg[inv]
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(new_deg)
    src = np.repeat(np.arange(n), deg)
    ns, nt = perm[src], perm[csr.targets]
    order = np.lexsort((nt, ns))
    return oracle.as_graph(off, nt[order].astype(np.int32), csr.weights[order])


def colour_record(g):
    t = time.time()
    memb, q, r = oracle.louvain(g, oracle.Params(mode="colour", seed=0))
    return {"Q": q, "digest": digest(memb), "passes": r["passes"], "iterations": r["iterations"],
            "communities": r["communities"], "seed": 0, "seconds": round(time.time() - t, 2)}


def run(name: str, spread_orders: int, only=None, old=None):
    csr = graphgen.workload(name)
    g = oracle.as_graph(csr.offsets, csr.targets, csr.weights)
    if only == "colour":
        rec = dict(old or {})
        rec["colour"] = colour_record(g)
        return rec
    rec = {"n": csr.n, "nnz": csr.nnz, "W": int(csr.weights.sum(dtype=np.int64))}
    t = time.time()
    memb, q, r = oracle.louvain(g, oracle.Params(mode="seq"))
    rec["seq"] = {"Q": q, "digest": digest(memb), "passes": r["passes"],
                  "iterations": r["iterations"], "communities": r["communities"],
                  "seconds": round(time.time() - t, 2)}
    t = time.time()
    memb, q, r = oracle.louvain(g, oracle.Params(mode="sync", seed=0, sample_bits=1))
    rec["sync"] = {"Q": q, "digest": digest(memb), "passes": r["passes"],
                   "iterations": r["iterations"], "communities": r["communities"],
                   "seed": 0, "round_bits": 1, "seconds": round(time.time() - t, 2)}
    qs = []
    rng = np.random.default_rng(12345)
    for _ in range(spread_orders):
        perm = rng.permutation(csr.n)
        _, q, _ = oracle.louvain(relabel(csr, perm), oracle.Params(mode="seq"))
        qs.append(q)
    if qs:
        rec["seq_relabel_Q"] = qs
    rec["colour"] = colour_record(g)
    return rec


def main(argv):
    only = None
    if argv[:1] == ["--only"]:
        only, argv = argv[1], argv[2:]
    names = argv or DEFAULT
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        orders = 4 if name not in ("rmat22", "sbm1m") else 0
        print("oracle on", name, flush=True)
        data[name] = run(name, orders, only, data.get(name))
        print(json.dumps(data[name]), flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
