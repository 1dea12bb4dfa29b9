"""Benchmark of the Louvain hot path on one MI355X.

A step is one whole Louvain run (every pass of local moving and aggregation,
the final dendrogram lookup and the modularity) over a seeded R-MAT graph
that is already resident in HBM: louvain_reset + louvain_run through the C
ABI.  value = input CSR entries / seconds per step (the paper's processing
rate, |E| over the runtime of the method).

The roofline object covers the dominant kernel family of a second timed
region run with per-kernel HIP events (on the library's stream):
achieved = algorithmic bytes of those launches / their summed duration.
The CPU baseline is the oracle (serial C, one core) timed on a bounded
sample of the same workload.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("edges/s per Louvain pass + HBM roofline %; modularity Δ vs oracle; "
          "p50/p99 job latency")
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "rmat22": "R-MAT scale 22 (4,194,304 vertices), 16 draws per vertex, a/b/c/d = "
              ".57/.19/.19/.05, duplicates merged, unit weights, seed 2",
    "rmat24": "R-MAT scale 24, 64 draws per vertex, weights 1..8 per draw, seed 3",
    "sbm10k": "planted-partition SBM, 10,000 vertices, 100 blocks, p_in .05, p_out .0005",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--mode", default="fast", choices=["fast", "deterministic"])
    ap.add_argument("--round-bits", type=int, default=1)
    ap.add_argument("--cpu-baseline", default="same",
                    help="workload the oracle is timed on: 'same' (the benchmark workload, "
                         "one whole run), a workload name, or 'none'")
    ap.add_argument("--no-profile", action="store_true")
    return ap.parse_args()


def run_steps(ctx, memb, steps):
    import torch
    res = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.reset()
        res = ctx.run(memb)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / max(steps, 1), res


def cpu_baseline(name):
    import numpy as np
    import graphgen
    import oracle
    csr = graphgen.workload(name)
    g = oracle.as_graph(csr.offsets, csr.targets, csr.weights)
    t0 = time.perf_counter()
    _, q, rec = oracle.louvain(g, oracle.Params(mode="seq"))
    dt = time.perf_counter() - t0
    return {"value": csr.nnz / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "one whole sequential-mode oracle Louvain run on %s (%d vertices, %d "
                      "entries), %.2f s, Q=%.5f" % (name, csr.n, csr.nnz, dt, q),
            "seconds": round(dt, 3)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the Louvain path here runs on a single MI355X "
              "(multi-GPU sharding is a design note only); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import graphgen
    import paper_2312_04876_amd as P

    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    csr = graphgen.workload(args.workload, threads=threads)
    gen_s = time.perf_counter() - t0
    print("generated %s: n=%d nnz=%d in %.1fs" % (args.workload, csr.n, csr.nnz, gen_s),
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    off = torch.from_numpy(csr.offsets32()).to(dev)
    tgt = torch.from_numpy(csr.targets).to(dev)
    w = torch.from_numpy(csr.weights).to(dev)
    memb = torch.empty(csr.n, dtype=torch.int32, device=dev)
    opts = dict(mode=args.mode, round_bits=args.round_bits)

    # timed region 1: the plain path
    ctx = P.Louvain(off, tgt, w, **opts)
    run_steps(ctx, memb, args.warmup)
    sec, (m, q, st) = run_steps(ctx, memb, args.steps)
    ctx.close()
    print("plain: %.3f ms/step Q=%.6f passes=%d iterations=%s" %
          (sec * 1e3, q, st["passes"], st["iterations"]), file=sys.stderr, flush=True)

    roofline = None
    kernels = []
    prof_sec = None
    if not args.no_profile:
        # timed region 2: same steps with HIP events around every kernel launch
        ctxp = P.Louvain(off, tgt, w, profile=True, **opts)
        run_steps(ctxp, memb, args.warmup)
        before = {k["name"]: k for k in ctxp.kernel_stats()}
        prof_sec, _ = run_steps(ctxp, memb, args.steps)
        after = ctxp.kernel_stats()
        ctxp.close()
        for k in after:
            b = before.get(k["name"], {"ms": 0.0, "bytes": 0.0, "launches": 0})
            ms = k["ms"] - b["ms"]
            kernels.append({"name": k["name"], "launches": k["launches"] - b["launches"],
                            "ms_per_step": ms / args.steps,
                            "bytes_per_step": (k["bytes"] - b["bytes"]) / args.steps})
        hot = [k for k in kernels if k["name"].startswith(("move_", "agg_"))]
        dom = max(hot, key=lambda k: k["ms_per_step"])
        gbs = dom["bytes_per_step"] / (dom["ms_per_step"] * 1e-3) / 1e9 if dom["ms_per_step"] else 0.0
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom["name"],
                    "launches_per_step": dom["launches"] / args.steps,
                    "ms_per_step": round(dom["ms_per_step"], 4),
                    "algorithmic_bytes_per_step": dom["bytes_per_step"]}
        print("profiled: %.3f ms/step" % (prof_sec * 1e3), file=sys.stderr, flush=True)
        for k in sorted(kernels, key=lambda k: -k["ms_per_step"])[:12]:
            print("  %-20s %8.3f ms/step %9.1f GB/s %6d launches" %
                  (k["name"], k["ms_per_step"],
                   k["bytes_per_step"] / max(k["ms_per_step"], 1e-9) * 1e-6,
                   k["launches"]), file=sys.stderr)

    golden = {}
    gpath = os.path.join(ROOT, "tests", "golden", "reference.json")
    if os.path.exists(gpath):
        golden = json.load(open(gpath)).get(args.workload, {})
    q_ref = golden.get("seq", {}).get("Q")

    cpu = None
    if args.cpu_baseline != "none":
        cpu = cpu_baseline(args.workload if args.cpu_baseline == "same" else args.cpu_baseline)
        print("cpu baseline: %s" % cpu["sample"], file=sys.stderr, flush=True)

    line = {
        "metric": METRIC,
        "value": csr.nnz / sec,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "int32/int64",
        "data": "synthetic: " + WORKLOADS.get(args.workload, args.workload),
        "config": {"workload": args.workload, "n": csr.n, "nnz": csr.nnz, "mode": args.mode,
                   "round_bits": args.round_bits},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "modularity": q,
        "modularity_delta_vs_oracle": (q - q_ref) if q_ref is not None else None,
        "passes": st["passes"],
        "iterations": st["iterations"],
        "communities": st["communities"],
        "per_pass_entries": st["entries"],
        "profiled_ms_per_step": prof_sec * 1e3 if prof_sec else None,
        "kernels": sorted(kernels, key=lambda k: -k["ms_per_step"])[:8],
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
