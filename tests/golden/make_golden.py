"""Write tests/golden/reference.json: oracle results on the seeded workloads.

Calls only the oracle (and the seeded generators for its inputs).  For each
workload it records the sequential-mode modularity (the quality reference of
the GPU fast mode), the synchronous-mode and colour-ordered results
(membership digest, Q, iterations and communities per pass; the bit-exact
references of the GPU deterministic and colour-ordered modes), plus the
spread of sequential-mode Q over random vertex relabellings, which calibrates
the fast-mode tolerance.

Usage: python tests/golden/make_golden.py [--only colour] [workload ...]
       python tests/golden/make_golden.py --full rmat24   (pass-by-pass records of a
       workload whose levels are too large for the oracle's own pass loop)
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
sys.path.insert(0, HERE)

import graphgen  # noqa: E402
import oracle  # noqa: E402
from digest import graph_digest, labels_digest  # noqa: E402

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


def lean_louvain(g, prm, lib=None, log=print):
    """Alg. 1 over the oracle's single steps (local moving, renumbering, aggregation)
    without keeping the levels, for graphs whose levels do not fit in memory twice:
    the pass loop of oracle.louvain_trace.  Returns (membership, Q, per-pass records:
    the local-moving trace, a digest of the raw labels, the communities and a digest of
    the aggregated level)."""
    top = np.arange(g.n, dtype=np.int32)
    level, tau, broke, Cp = g, prm.tolerance, False, None
    passes = []
    for p in range(prm.max_passes):
        t = time.time()
        st = oracle.MoveState.fresh(level)
        tr = oracle.move(level, st, prm.mode, tau, prm.max_iterations, prm.prune, prm.seed, p,
                         prm.sample_bits, lib=lib)
        Cp = st.C
        del st
        nc = int(np.unique(Cp).size) if level.n else 0
        rec = {"vertices": level.n, "entries": level.nnz, "iterations": tr.iterations,
               "sumN": [str(x) for x in tr.sumN], "moves": tr.moves, "processed": tr.processed,
               "labels": labels_digest(Cp), "communities": nc}
        passes.append(rec)
        log("  pass %d: %d vertices, %d iterations, %d communities (%.0f s)" %
            (p, level.n, tr.iterations, nc, time.time() - t))
        if tr.iterations <= 1 or float(nc) / float(level.n) > prm.aggregation_tolerance:
            broke = True
            break
        Cp, nc = oracle.renumber(Cp)
        top = Cp[top]
        t = time.time()
        nxt = oracle.aggregate(level, Cp, nc)
        rec["next_level"] = graph_digest(nxt.offsets, None, nxt.targets, nxt.weights)
        log("  aggregated: %d vertices, %d entries (%.0f s)" % (nxt.n, nxt.nnz, time.time() - t))
        level = nxt
        tau = tau / prm.tolerance_drop
    if broke:
        top = Cp[top]
    memb, _ = oracle.renumber(top)
    return memb, oracle.modularity(g, memb), passes


def full_record(name: str):
    """Records of a workload too large for oracle.louvain's level buffers (R-MAT-24): the
    sequential run (quality reference of fast mode) and the synchronous run pass by pass
    (bit-exact reference of deterministic mode), both through lean_louvain; the
    synchronous run uses the OpenMP build, whose results equal the serial build's
    (tests/test_oracle_timing_build.py)."""
    t = time.time()
    csr = graphgen.workload(name, threads=min(16, os.cpu_count() or 1))
    print("generated %s: n=%d nnz=%d (%.0f s)" % (name, csr.n, csr.nnz, time.time() - t),
          flush=True)
    rec = {"n": csr.n, "nnz": csr.nnz, "W": int(csr.weights.sum(dtype=np.int64))}
    g = oracle.as_graph(csr.offsets, csr.targets, csr.weights)
    del csr
    lib = oracle.timing_library()
    for mode, params in (("sync", {"seed": 0, "sample_bits": 1}), ("seq", {})):
        t = time.time()
        print("oracle %s on %s" % (mode, name), flush=True)
        memb, q, passes = lean_louvain(g, oracle.Params(mode=mode, **params), lib=lib,
                                       log=lambda m: print(m, flush=True))
        r = {"Q": q, "digest": digest(memb), "passes": len(passes),
             "iterations": [x["iterations"] for x in passes],
             "communities": [x["communities"] for x in passes],
             "seconds": round(time.time() - t, 1)}
        if mode == "sync":
            r.update({"seed": 0, "round_bits": 1, "per_pass": passes})
        rec[mode] = r
        print(json.dumps({k: v for k, v in r.items() if k != "per_pass"}), flush=True)
    return rec


def main(argv):
    only = None
    if argv[:1] == ["--full"]:
        data = json.load(open(OUT)) if os.path.exists(OUT) else {}
        for name in argv[1:]:
            data[name] = full_record(name)
            with open(OUT, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
        return
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
