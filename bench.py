"""Benchmark of the Louvain hot path on one MI355X.

A step is one whole Louvain run (every pass of local moving and aggregation,
the final dendrogram lookup and the modularity) over a seeded R-MAT graph
that is already resident in HBM: louvain_reset + louvain_run through the C
ABI.  value = input CSR entries / seconds per step (the paper's processing
rate, |E| over the runtime of the method).  The default workload is R-MAT
scale 24 (2.0e9 entries) in fast mode; R-MAT scale 22 follows as a secondary
block.

Roofline objects cover the dominant kernel family overall, the dominant
local-moving family and the dominant aggregation family of a second timed
region run with per-kernel HIP events (on the library's stream): achieved =
algorithmic bytes of those launches / their summed duration.  The CPU
baseline is the oracle (its -O3 -march=native OpenMP build, whose results
equal the serial build's) timed on a bounded sample of the same workload.

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
    "sbm1m": "planted-partition SBM, 1,000,000 vertices, 1,000 blocks, p_in .015, p_out .000005",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat24")
    ap.add_argument("--secondary", default="rmat22",
                    help="a second workload timed after the main one (its own block in the line); "
                         "'none' to skip")
    ap.add_argument("--mode", default="fast", choices=["fast", "deterministic", "coloured"])
    ap.add_argument("--autotune", action="store_true",
                    help="pick the hub threshold and hub partition size by timing the candidates "
                         "on this workload first (paper_2312_04876_amd.autotune)")
    ap.add_argument("--round-bits", type=int, default=None,
                    help="2^round_bits rounds per iteration (default: the library's, 3 in fast "
                         "mode on one graph, else 1)")
    ap.add_argument("--q-runs", type=int, default=0, metavar="K",
                    help="after the timed runs, K more whole runs of the main workload whose "
                         "modularities go into the line (fast mode is nondeterministic)")
    ap.add_argument("--small-level", type=int, default=0,
                    help="batches: levels of a graph with at most this many vertices run in the "
                         "small-level kernel (0: the library's default, -1: none)")
    ap.add_argument("--cpu-baseline", default="same",
                    help="workload the oracle is timed on: 'same' (the benchmark workload, "
                         "one whole run), a workload name, or 'none'")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 3 plain device copies of MIB MiB (calibrates the HBM byte "
                         "counters of a profiler against a kernel of known traffic) and exit")
    ap.add_argument("--pmc-summary", nargs="+", metavar="DIR",
                    help="summarise rocprofv3 --pmc output directories into --pmc-out: FETCH_SIZE "
                         "and WRITE_SIZE of one bench step, the same of the copy probe, and "
                         "optionally TCC_ATOMIC_sum + TCC_EA0_ATOMIC_sum of one bench step")
    ap.add_argument("--pmc-out", default=None,
                    help="PMC summary file (default profiles/<workload>_<mode>_pmc.json)")
    ap.add_argument("--batch", type=int, default=0, metavar="G",
                    help="only run the batched workload: G planted-partition SBMs of uneven size "
                         "(n log-uniform 200..50,000, mean degree 8..40, p_out/p_in = 0.02) as one "
                         "union run, against the same graphs run one by one")
    ap.add_argument("--batch-nmax", type=int, default=50_000)
    ap.add_argument("--batch-q-out", default=None, metavar="PATH",
                    help="write each graph's modularity (union run and one by one) to this JSON "
                         "file, for comparison with the oracle offline")
    ap.add_argument("--serve", type=float, nargs="*", metavar="RATE",
                    help="only run the serving workload: Poisson arrivals at each RATE jobs/s "
                         "drawn from a pool of SBM and R-MAT graphs")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--serve-pool", type=int, default=1024)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-budget-gib", type=float, default=160.0)
    ap.add_argument("--dynamic", type=float, nargs="*", metavar="FRAC",
                    help="only run the dynamic workload: after an edge batch that deletes and "
                         "inserts FRAC of the edges, a cold run against a run warm-started from "
                         "the membership before the batch")
    return ap.parse_args()


# Kernel family (as named by louvain_kernel_stats) -> the device kernels of one launch.
FAMILY_KERNELS = {
    "move_bin0_1lane": [r"k_move_wave<[^>]*>, 1, 8, 4,"],
    "move_bin1_4lanes": [r"k_move_wave<[^>]*>, 4, 8, 6,"],
    "move_bin2_16lanes": [r"k_move_wave<[^>]*>, 16, 8, 8,"],
    "move_bin3_wave": [r"k_move_wave<[^>]*>, 64, 8, 10,"],
    "move_bin4_block": [r"k_move_block<[^>]*>, 256,"],
    "move_bin5_bigblock": [r"k_move_block<[^>]*>, 512,"],
    "move_bin6_hub": [r"k_move_hub<", r"k_hub_count<", r"k_hub_fill<", r"k_hub_part<",
                      r"k_hub_mark<"],
    "move_seq": [r"k_seq_level<"],
    "agg_bin0_4lanes": [r"k_agg_wave<[^>]*>, 4, 4>"],
    "agg_bin1_4lanes": [r"k_agg_wave<[^>]*>, 4, 6>"],
    "agg_bin2_8lanes": [r"k_agg_wave<[^>]*>, (8|16), 8>"],  # 16 lanes with 8-byte sums
    "agg_bin3_wave": [r"k_agg_wave<[^>]*>, 64, 10>"],
    "agg_bin6_hub": [r"k_agg_hub_part<", r"k_agg_hub_count<", r"k_agg_hub_fill<"],
}


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2312_04876_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(f.encode())
        h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "louvain.h"), "rb").read())
    return h.hexdigest()


def _pmc_rows(d):
    import csv
    import glob
    rows = []
    for p in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        rows += list(csv.DictReader(open(p)))
    return rows


def pmc_summary(dirs, out, workload=None):
    """Per-kernel HBM traffic per dispatch from FETCH_SIZE / WRITE_SIZE runs, scaled by what the
    same counters read for the copy probe (bytes actually moved / counter bytes)."""
    import re
    fetch, write, cfetch, cwrite = (_pmc_rows(d) for d in dirs[:4])
    atom = _pmc_rows(dirs[4]) if len(dirs) > 4 else []

    def per_kernel(rows, counter):
        acc = {}
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            k = acc.setdefault(r["Kernel_Name"], [0, 0.0])
            k[0] += 1
            k[1] += float(r["Counter_Value"]) * 1024.0  # KiB per dispatch
        return acc

    def copy_factor(rows, counter):
        got = sum(v[1] for k, v in per_kernel(rows, counter).items() if "copyBuffer" in k)
        return (3 * 1024 * (1 << 20)) / got  # the probe copies 1 GiB three times

    ff, wf = copy_factor(cfetch, "FETCH_SIZE"), copy_factor(cwrite, "WRITE_SIZE")
    f, w = per_kernel(fetch, "FETCH_SIZE"), per_kernel(write, "WRITE_SIZE")
    # L2 atomic requests and those forwarded to the memory side (counts, not KiB)
    a_l2 = {k: v[1] / 1024.0 for k, v in per_kernel(atom, "TCC_ATOMIC_sum").items()}
    a_ea = {k: v[1] / 1024.0 for k, v in per_kernel(atom, "TCC_EA0_ATOMIC_sum").items()}
    kernels = {}
    for name in f:
        kernels[name] = {"dispatches": f[name][0], "fetch_bytes": f[name][1] * ff,
                         "write_bytes": w.get(name, [0, 0.0])[1] * wf}
        if atom:
            kernels[name]["atomics"] = a_l2.get(name, 0.0)
            kernels[name]["atomics_memory_side"] = a_ea.get(name, 0.0)
    fam = {}
    for family, pats in FAMILY_KERNELS.items():
        ks = [k for k in kernels if any(re.search(p, k) for p in pats)]
        if not ks:
            continue
        main = [k for k in ks if re.search(pats[0], k)]
        launches = sum(kernels[k]["dispatches"] for k in main)
        total = sum(kernels[k]["fetch_bytes"] + kernels[k]["write_bytes"] for k in ks)
        fam[family] = {"launches": launches, "bytes_per_launch": total / max(launches, 1)}
        if atom:
            fam[family]["atomics_per_launch"] = sum(kernels[k].get("atomics", 0.0)
                                                    for k in ks) / max(launches, 1)
            fam[family]["memory_side_atomics_per_launch"] = sum(
                kernels[k].get("atomics_memory_side", 0.0) for k in ks) / max(launches, 1)
    data = {"sources_sha256": sources_digest(), "workload": workload, "fetch_factor": ff,
            "write_factor": wf, "families": fam, "kernels": kernels}
    with open(out, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(json.dumps({"fetch_factor": ff, "write_factor": wf, "families": fam}, indent=1))


def measured_traffic(family, path, key="bytes_per_launch", workload=None):
    """HBM bytes (or, with key, another per-launch figure) of `family` from the PMC summary,
    if it was taken on these sources (and on this workload)."""
    if not os.path.exists(path):
        return None
    data = json.load(open(path))
    if data.get("sources_sha256") != sources_digest():
        return None
    if workload is not None and data.get("workload") not in (None, workload):
        return None
    f = data.get("families", {}).get(family)
    return f.get(key) if f else None


def copy_probe(mib):
    """Three device-to-device copies of a known size: reads and writes mib MiB each."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                      "copies": 3}))


def run_steps(ctx, memb, steps, per_step=None):
    """Mean seconds per whole run over `steps` runs (one synchronisation on each side of
    the timed region); each run's own time is appended to `per_step` if given (a run
    ends with a host read-back, so timing it alone adds no synchronisation)."""
    import torch
    res = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = t0
    for _ in range(steps):
        ctx.reset()
        res = ctx.run(memb)
        if per_step is not None:
            now = time.perf_counter()
            per_step.append(now - last)
            last = now
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / max(steps, 1), res


def host_info():
    """CPU model, logical CPUs, CPUs this process may use, and RAM of the machine."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram = 0
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = int(line.split()[1]) * 1024
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "cpus_available": len(os.sched_getaffinity(0)), "ram_gib": round(ram / 2 ** 30, 1)}


def cpu_baseline(name):
    """The oracle's whole sequential run on a small workload (one core, serial build)."""
    import graphgen
    import oracle
    csr = graphgen.workload(name)
    g = oracle.as_graph(csr.offsets, csr.targets, csr.weights)
    t0 = time.perf_counter()
    _, q, rec = oracle.louvain(g, oracle.Params(mode="seq"))
    dt = time.perf_counter() - t0
    out = {"value": csr.nnz / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
           "sample": "one whole sequential-mode oracle Louvain run on %s (%d vertices, %d "
                     "entries), %.2f s, Q=%.5f" % (name, csr.n, csr.nnz, dt, q),
           "seconds": round(dt, 3)}
    out.update(host_info())
    return out


def _fresh(g, K, W):
    import numpy as np
    import oracle
    return oracle.MoveState(K=K, W=W, Sigma=K.copy(), C=np.arange(g.n, dtype=np.int32),
                            size=np.ones(g.n, dtype=np.int32), active=np.ones(g.n, dtype=np.uint8))


def _first_sweep(g, K, W, lib, v_end):
    """Seconds of the oracle's first synchronous local-moving iteration (pass 1, two
    rounds) over the rows of vertices [0, v_end) of g, and the entries those rows hold.
    The decisions of a synchronous round are independent of one another, so a prefix of
    the (randomly relabelled) vertices is a sample of the whole iteration."""
    import oracle
    st = _fresh(g, K, W)
    st.active[v_end:] = 0
    t0 = time.perf_counter()
    oracle.move(g, st, "sync", 0.0, 1, True, 0, 0, 1, lib=lib)
    return time.perf_counter() - t0, int(g.offsets[v_end])


def cpu_baseline_sampled(csr, target_s=12.0):
    """Oracle (-O3 -march=native OpenMP build) on a bounded sample of the workload: the
    first synchronous local-moving iteration over a prefix of the vertices sized for about
    target_s seconds, on every available thread and on one thread; entries scanned per
    second.  The GPU's figure for the same unit is reported beside it."""
    import ctypes

    import oracle
    g = oracle.as_graph(csr.offsets, csr.targets, csr.weights)
    K, W = oracle.vertex_weights(g)
    lib = oracle.timing_library()
    gomp = ctypes.CDLL("libgomp.so.1")
    threads = len(os.sched_getaffinity(0))
    out = {}
    for label, nt in (("multicore", threads), ("single_core", 1)):
        gomp.omp_set_num_threads(nt)
        # grow the prefix until the sweep takes about target_s (each call also pays the
        # oracle's per-call set-up: its level-sized snapshots and scan tables)
        v_end = max(1, g.n // 64)
        for _ in range(4):
            dt, ent = _first_sweep(g, K, W, lib, v_end)
            if v_end >= g.n or dt >= 0.5 * target_s:
                break
            v_end = int(min(g.n, max(2 * v_end, v_end * target_s / max(dt, 1e-3))))
        out[label] = {"value": ent / dt, "threads": nt, "vertices": v_end, "entries": ent,
                      "seconds": round(dt, 3)}
    gomp.omp_set_num_threads(threads)
    mc, sc = out["multicore"], out["single_core"]
    res = {"value": mc["value"], "unit": "edges/s", "cores": mc["threads"], "kind": "oracle",
           "sample": "first synchronous local-moving iteration (pass 1, two rounds) of the "
                     "oracle's -O3 -march=native OpenMP build over the rows of the first %d of "
                     "%d vertices of %s (%d of %d entries, %.1f s on %d threads): entries "
                     "scanned per second" % (mc["vertices"], g.n, csr.name, mc["entries"],
                                             g.nnz, mc["seconds"], mc["threads"]),
           "seconds": mc["seconds"], "single_core": sc}
    res.update(host_info())
    return res


def batch_main(args):
    """Batched workload: one union run of G graphs vs G per-graph runs (inputs resident)."""
    import numpy as np
    import torch

    import graphgen
    import paper_2312_04876_amd as P

    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    u, go, specs = graphgen.batch_sbm(args.batch, seed=4, threads=threads, n_max=args.batch_nmax)
    print("generated %d graphs: n=%d nnz=%d in %.1fs" % (args.batch, u.n, u.nnz,
                                                         time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    opts = dict(mode=args.mode, round_bits=args.round_bits)
    sopts = dict(opts, small_level=args.small_level)  # the autotuner picks small_level itself
    off = torch.from_numpy(u.offsets32()).to(dev)
    tgt = torch.from_numpy(u.targets).to(dev)
    w = torch.from_numpy(u.weights).to(dev)
    memb = torch.empty(max(u.n, 1), dtype=torch.int32, device=dev)
    uopts = dict(sopts)
    tuned = None
    if args.autotune:
        from paper_2312_04876_amd import autotune
        tuned = autotune.tune(off, tgt, w, graph_offsets=go, runs=2, warmup=1, **opts)
        uopts.update(autotune.tuned_params(tuned))
        print("autotune (union): hub_rows %d, hub_part_pairs %d, small_level %d (%.1f s; %s)" %
              (tuned["hub_rows"], tuned["hub_part_pairs"], tuned["small_level"], tuned["seconds"],
               ", ".join("%d/%d/%d %.1f ms" % (r["hub_rows"], r["hub_part_pairs"],
                                               r["small_level"], r["ms"]) for r in tuned["table"])),
              file=sys.stderr, flush=True)
    ctx = P.Louvain(off, tgt, w, graph_offsets=go, **uopts)
    run_steps(ctx, memb, args.warmup)
    sec_b, (m, _q, st) = run_steps(ctx, memb, args.steps)
    q_b, comm_b = ctx.batch_results()
    ctx.close()
    print("batched: %.1f ms per batch, %.3g edges/s, passes %d" %
          (sec_b * 1e3, u.nnz / sec_b, st["passes"]), file=sys.stderr, flush=True)
    # the same graphs one by one (each resident with its own context)
    ctxs = []
    for g in range(args.batch):
        a, b = int(go[g]), int(go[g + 1])
        e0, e1 = int(u.offsets[a]), int(u.offsets[b])
        o = torch.from_numpy((u.offsets[a:b + 1] - e0).astype(np.int32)).to(dev)
        t = torch.from_numpy(u.targets[e0:e1] - np.int32(a)).to(dev)
        ww = torch.from_numpy(u.weights[e0:e1]).to(dev)
        ctxs.append((P.Louvain(o, t, ww, **sopts), torch.empty(max(b - a, 1), dtype=torch.int32,
                                                               device=dev)))
    q_s = [0.0] * args.batch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, (c, mm) in enumerate(ctxs):
        c.reset()
        _, q_s[g], _ = c.run(mm)
    torch.cuda.synchronize()
    sec_s = time.perf_counter() - t0
    for c, _ in ctxs:
        c.close()
    print("one by one: %.1f ms, %.3g edges/s" % (sec_s * 1e3, u.nnz / sec_s), file=sys.stderr,
          flush=True)
    dq = [abs(a - b) for a, b in zip(q_b, q_s)]
    if args.batch_q_out:
        with open(args.batch_q_out, "w") as fh:
            json.dump({"graphs": args.batch, "batch_nmax": args.batch_nmax, "seed": 4,
                       "mode": args.mode, "round_bits": args.round_bits, "options": uopts,
                       "q_union": list(map(float, q_b)), "q_one_by_one": list(map(float, q_s))},
                      fh)
    line = {
        "metric": "edges/s of a batch of graphs (one union run) vs the same graphs run one by one",
        "value": u.nnz / sec_b, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec_b * 1e3, "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": "int32/int64",
        "data": "synthetic: %d planted-partition SBMs, n log-uniform 200..%d, mean degree 8..40, "
                "4..200 blocks, p_out/p_in 0.02, unit weights, seed 4" % (args.batch,
                                                                            args.batch_nmax),
        "config": {"workload": "batch%d" % args.batch, "graphs": args.batch, "n": u.n,
                   "nnz": u.nnz, "mode": args.mode, "round_bits": args.round_bits,
                   "small_level": args.small_level},
        "one_by_one": {"value": u.nnz / sec_s, "ms": sec_s * 1e3},
        "autotune": tuned,
        "speedup": sec_s / sec_b,
        "max_abs_q_difference": max(dq) if dq else 0.0,
        "identical_q": sum(1 for d in dq if d == 0.0),
        "mean_q": float(np.mean(q_b)) if q_b else 0.0,
        "passes": st["passes"],
    }
    print(json.dumps(line))


def serve_main(args):
    """Serving workload: Poisson arrivals from a resident pool; p50/p99 latency and edges/s."""
    import random
    import threading

    import numpy as np
    import torch

    import graphgen
    from paper_2312_04876_amd.serve import GpuExecutor, Job, Server, latency_stats

    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    pool = {k: g for k, g in enumerate(graphgen.serving_pool(args.serve_pool, seed=5,
                                                             threads=threads))}
    nnz = np.array([g.nnz for g in pool.values()])
    print("pool of %d graphs: median %d entries, mean %d, max %d, generated in %.1fs" %
          (len(pool), int(np.median(nnz)), int(nnz.mean()), int(nnz.max()),
           time.perf_counter() - t0), file=sys.stderr, flush=True)
    ex = GpuExecutor(pool, slots=args.serve_slots, mode=args.mode, round_bits=args.round_bits)
    # warm-up: one small batch on every slot
    warm = Server(ex, memory_budget=int(args.serve_budget_gib * (1 << 30)), slots=args.serve_slots)
    for k in range(2 * args.serve_slots):
        warm.submit(Job(key=k, nnz=pool[k].nnz, n=pool[k].n))
    warm.close()
    results = []
    for rate in args.serve:
        rng = random.Random(5)
        srv = Server(ex, memory_budget=int(args.serve_budget_gib * (1 << 30)),
                     slots=args.serve_slots)
        jobs = []
        start = time.perf_counter()

        def feed():
            t = start
            while True:
                t += rng.expovariate(rate)
                if t - start > args.serve_seconds:
                    return
                d = t - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                k = rng.randrange(len(pool))
                jobs.append(srv.submit(Job(key=k, nnz=pool[k].nnz, n=pool[k].n)))

        th = threading.Thread(target=feed)
        th.start()
        th.join()
        srv.drain()
        end = time.perf_counter()
        srv.close()
        done = [j for j in jobs if j.error is None]
        st = latency_stats(jobs)
        ent = sum(j.nnz for j in done)
        res = {"rate_jobs_per_s": rate, "jobs": len(jobs), "completed": len(done),
               "failed": len(jobs) - len(done), "batches": srv.batches,
               "p50_ms": st.get("p50_ms"), "p99_ms": st.get("p99_ms"), "max_ms": st.get("max_ms"),
               "edges_per_s": ent / (end - start), "offered_edges_per_s":
                   sum(j.nnz for j in jobs) / args.serve_seconds,
               "wall_s": end - start, "peak_memory_gib": srv.peak_memory / (1 << 30)}
        results.append(res)
        print("rate %.0f/s: %d jobs, %d batches, p50 %.1f ms p99 %.1f ms, %.3g edges/s" %
              (rate, len(jobs), srv.batches, res["p50_ms"] or 0, res["p99_ms"] or 0,
               res["edges_per_s"]), file=sys.stderr, flush=True)
    best = results[-1] if results else {}
    line = {"metric": "p50/p99 job latency and edges/s of the continuous-batching server",
            "value": best.get("edges_per_s"), "unit": "edges/s", "n_gpus": 1,
            "steps": len(results), "warmup": 1, "ms_per_step": None, "higher_is_better": True,
            "scaling": "strong", "vs_baseline": None, "dtype": "int32/int64",
            "data": "synthetic: pool of %d graphs, half SBM half R-MAT, entries log-normal "
                    "(median 2e5, sigma 1.5, cap 5e7), Poisson arrivals, seed 5" % len(pool),
            "config": {"workload": "serve", "mode": args.mode, "slots": args.serve_slots,
                       "seconds": args.serve_seconds,
                       "memory_budget_gib": args.serve_budget_gib},
            "rates": results}
    print(json.dumps(line))


def dynamic_main(args):
    """Dynamic workload: cold vs warm-started runs after edge batches of each size."""
    import numpy as np
    import torch

    import graphgen
    import paper_2312_04876_amd as P

    threads = min(16, os.cpu_count() or 1)
    csr = graphgen.workload(args.workload, threads=threads)
    dev = torch.device("cuda:0")

    def upload(c):
        return (torch.from_numpy(c.offsets32()).to(dev), torch.from_numpy(c.targets).to(dev),
                torch.from_numpy(c.weights).to(dev))
    opts = dict(mode=args.mode, round_bits=args.round_bits)
    base = P.Louvain(*upload(csr), **opts)
    m0, q0, _ = base.run()
    m0 = m0.clone()
    base.close()
    rows = []
    for frac in args.dynamic:
        t0 = time.perf_counter()
        g2 = graphgen.perturb(csr, frac, seed=9)
        print("edge batch %.4g: %d -> %d entries in %.1fs" % (frac, csr.nnz, g2.nnz,
                                                              time.perf_counter() - t0),
              file=sys.stderr, flush=True)
        ctx = P.Louvain(*upload(g2), **opts)
        memb = torch.empty(g2.n, dtype=torch.int32, device=dev)

        def timed(warm):
            res = None
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                ctx.reset()
                if warm:
                    ctx.set_membership(m0)
                res = ctx.run(memb)
            torch.cuda.synchronize()
            return (time.perf_counter() - t) / args.steps, res
        for _ in range(args.warmup):
            timed(False)
            timed(True)
        cold_s, (_, cold_q, cold_st) = timed(False)
        warm_s, (_, warm_q, warm_st) = timed(True)
        ctx.close()
        row = {"fraction": frac, "entries": g2.nnz, "cold_ms": cold_s * 1e3, "cold_q": cold_q,
               "cold_iterations": cold_st["iterations"], "warm_ms": warm_s * 1e3,
               "warm_q": warm_q, "warm_iterations": warm_st["iterations"],
               "speedup": cold_s / warm_s}
        rows.append(row)
        print("  cold %.2f ms Q=%.5f its %s | warm %.2f ms Q=%.5f its %s" %
              (cold_s * 1e3, cold_q, cold_st["iterations"], warm_s * 1e3, warm_q,
               warm_st["iterations"]), file=sys.stderr, flush=True)
    line = {"metric": "edges/s of a warm-started re-run after an edge batch (vs a cold run)",
            "value": rows[-1]["entries"] / (rows[-1]["warm_ms"] * 1e-3) if rows else None,
            "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": rows[-1]["warm_ms"] if rows else None, "higher_is_better": True,
            "scaling": "strong", "vs_baseline": None, "dtype": "int32/int64",
            "data": "synthetic: %s, then edge batches deleting and inserting a share of its "
                    "edges (seed 9)" % WORKLOADS.get(args.workload, args.workload),
            "config": {"workload": args.workload + "-dynamic", "mode": args.mode,
                       "base_q": q0}, "batches": rows}
    print(json.dumps(line))


def main():
    args = parse()
    if args.round_bits is None:
        # the library's default: 8 rounds for one graph in fast mode, else 2 (batches and
        # serving run batches)
        single = not args.batch and args.serve is None
        args.round_bits = 3 if args.mode == "fast" and single else 1
    if args.dynamic:
        if args.gpus != 1:
            print("bench.py measures one GPU; use --gpus 1", file=sys.stderr)
            sys.exit(2)
        dynamic_main(args)
        return
    if args.serve:
        if args.gpus != 1:
            print("bench.py measures one GPU; use --gpus 1", file=sys.stderr)
            sys.exit(2)
        serve_main(args)
        return
    if args.batch:
        if args.gpus != 1:
            print("bench.py measures one GPU; use --gpus 1", file=sys.stderr)
            sys.exit(2)
        batch_main(args)
        return
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.pmc_summary:
        if len(args.pmc_summary) not in (4, 5):
            print("--pmc-summary takes 4 or 5 directories", file=sys.stderr)
            sys.exit(2)
        pmc_summary(args.pmc_summary, workload=args.workload, out=args.pmc_out or os.path.join(
            ROOT, "profiles", "%s_%s_pmc.json" % (args.workload, args.mode)))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the Louvain path here runs on a single MI355X "
              "(multi-GPU sharding is a design note only); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import graphgen

    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    csr = graphgen.workload(args.workload, threads=threads)
    print("generated %s: n=%d nnz=%d in %.1fs" % (args.workload, csr.n, csr.nnz,
                                                  time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    main_block = measure(args, csr, args.workload, args.steps, args.warmup)

    secondary = None
    if args.secondary and args.secondary != "none" and args.secondary != args.workload:
        csr2 = graphgen.workload(args.secondary, threads=threads)
        print("generated %s: n=%d nnz=%d" % (args.secondary, csr2.n, csr2.nnz), file=sys.stderr,
              flush=True)
        secondary = measure(args, csr2, args.secondary, min(args.steps, 10), min(args.warmup, 2))
        del csr2

    cpu = None
    if args.cpu_baseline != "none":
        if args.cpu_baseline == "same" and csr.nnz > 200_000_000:
            cpu = cpu_baseline_sampled(csr)
            cpu["gpu_same_unit"] = main_block.pop("first_iteration")
        else:
            cpu = cpu_baseline(args.workload if args.cpu_baseline == "same" else args.cpu_baseline)
        print("cpu baseline: %s" % cpu["sample"], file=sys.stderr, flush=True)
    main_block.pop("first_iteration", None)
    if secondary:
        secondary.pop("first_iteration", None)

    line = {
        "metric": METRIC,
        "value": main_block["value"],
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_block["ms_per_step"],
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "int32/int64",
        "data": "synthetic: " + WORKLOADS.get(args.workload, args.workload),
        "config": main_block["config"],
        "roofline": main_block["roofline"],
        "cpu_baseline": cpu,
    }
    for k, v in main_block.items():
        if k not in line and k not in ("value", "ms_per_step"):
            line[k] = v
    line["secondary"] = secondary
    print(json.dumps(line))


def measure(args, csr, name, steps, warmup):
    """Timed whole runs of one workload, pass-by-pass timing, and a profiled region with
    per-kernel HIP events; returns the workload's block of the bench line."""
    import numpy as np
    import torch

    import paper_2312_04876_amd as P
    dev = torch.device("cuda:0")
    off = torch.from_numpy(csr.offsets32()).to(dev)
    tgt = torch.from_numpy(csr.targets).to(dev)
    w = torch.from_numpy(csr.weights).to(dev)
    memb = torch.empty(csr.n, dtype=torch.int32, device=dev)
    opts = dict(mode=args.mode, round_bits=args.round_bits)
    tuned = None
    if args.autotune:
        from paper_2312_04876_amd import autotune
        tuned = autotune.tune(off, tgt, w, runs=2, warmup=1, **opts)
        opts.update(autotune.tuned_params(tuned))
        print("autotune: hub_rows %d, hub_part_pairs %d, small_level %d (%.1f s; %s)" %
              (tuned["hub_rows"], tuned["hub_part_pairs"], tuned["small_level"], tuned["seconds"],
               ", ".join("%d/%d/%d %.2f ms" % (r["hub_rows"], r["hub_part_pairs"],
                                               r["small_level"], r["ms"])
                         for r in tuned["table"])), file=sys.stderr, flush=True)

    # timed region 1: the plain path
    ctx = P.Louvain(off, tgt, w, **opts)
    run_steps(ctx, memb, warmup)
    runs = []
    sec, (m, q, st) = run_steps(ctx, memb, steps, runs)
    # untimed: more whole runs for the spread of a nondeterministic mode's modularity
    q_more = []
    for _ in range(args.q_runs if name == args.workload else 0):
        ctx.reset()
        q_more.append(ctx.run(memb)[1])
    # per pass (moving + renumbering + aggregation, Alg. 1), stepped through the C ABI
    # pass by pass with the host waiting after each: median over the timed runs
    per_pass = []
    for _ in range(max(1, min(steps, 5))):
        ctx.reset()
        times = []
        while True:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.move()
            _nc, stop = ctx.aggregate()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            if stop:
                break
        per_pass.append(times)
    pst = ctx.stats()
    ctx.close()
    del ctx  # its workspace (tens of GB at R-MAT-24) goes back before the next context
    npass = min(len(t) for t in per_pass)
    pass_ms = [float(np.median([t[p] for t in per_pass])) * 1e3 for p in range(npass)]
    pass_rate = [pst["entries"][p] / (pass_ms[p] * 1e-3) for p in range(min(npass, pst["passes"]))]
    print("%s: %.3f ms/step Q=%.6f passes=%d iterations=%s" %
          (name, sec * 1e3, q, st["passes"], st["iterations"]), file=sys.stderr, flush=True)
    print("per pass: %s ms, %s edges/s" % (["%.2f" % x for x in pass_ms],
                                          ["%.3g" % x for x in pass_rate]),
          file=sys.stderr, flush=True)

    # the first local-moving iteration alone (the unit of the sampled CPU baseline)
    one = P.Louvain(off, tgt, w, max_iterations=1, max_passes=1, **opts)
    first = []
    for _ in range(3):
        one.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one.move()
        torch.cuda.synchronize()
        first.append(time.perf_counter() - t0)
    one.close()
    del one
    first_s = float(np.median(first))

    roofline = roof_move = roof_agg = None
    kernels = []
    prof_sec = None
    phases = None
    scan_rate = None
    pmc_path = os.path.join(ROOT, "profiles", "%s_%s_pmc.json" % (name, args.mode))
    if args.pmc_out and name == args.workload:
        pmc_path = args.pmc_out
    if not args.no_profile:
        # timed region 2: same steps with HIP events around every kernel launch
        ctxp = P.Louvain(off, tgt, w, profile=True, **opts)
        run_steps(ctxp, memb, warmup)
        before = {k["name"]: k for k in ctxp.kernel_stats()}
        prof_sec, (_m, _q, pst2) = run_steps(ctxp, memb, steps)
        after = ctxp.kernel_stats()
        ctxp.close()
        del ctxp
        for k in after:
            b = before.get(k["name"], {"ms": 0.0, "bytes": 0.0, "launches": 0})
            kernels.append({"name": k["name"], "launches": k["launches"] - b["launches"],
                            "ms_per_step": (k["ms"] - b["ms"]) / steps,
                            "bytes_per_step": (k["bytes"] - b["bytes"]) / steps})

        def roof(fams):
            if not fams:
                return None
            dom = max(fams, key=lambda k: k["ms_per_step"])
            gbs = dom["bytes_per_step"] / (dom["ms_per_step"] * 1e-3) / 1e9 \
                if dom["ms_per_step"] else 0.0
            per_launch_s = dom["ms_per_step"] * 1e-3 * steps / max(dom["launches"], 1)
            traffic = measured_traffic(dom["name"], pmc_path, workload=name)
            atomics = measured_traffic(dom["name"], pmc_path, "atomics_per_launch", workload=name)
            return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": dom["name"],
                    "algorithmic_bytes_per_launch": dom["bytes_per_step"] * steps /
                    max(dom["launches"], 1),
                    "launches_per_step": dom["launches"] / steps,
                    "ms_per_step": round(dom["ms_per_step"], 4),
                    "ms_per_launch": round(per_launch_s * 1e3, 4),
                    "algorithmic_bytes_per_step": dom["bytes_per_step"],
                    "atomics_per_launch": atomics,
                    "atomics_per_s": atomics / per_launch_s if atomics else None}
        moves = [k for k in kernels if k["name"].startswith("move_")]
        aggs = [k for k in kernels if k["name"].startswith("agg_")]
        roofline = roof(moves + aggs)
        roof_move = roof(moves)
        roof_agg = roof(aggs)
        move_ms = sum(k["ms_per_step"] for k in moves)
        scan_rate = sum(pst2["scanned"]) / (move_ms * 1e-3) if move_ms else None
        # the per-pass split of the run by phase (local moving, aggregation, other)
        phases = {"ms_move": [round(x / 1.0, 3) for x in pst2["ms_move"]],
                  "ms_aggregate": [round(x, 3) for x in pst2["ms_aggregate"]],
                  "ms_other": [round(x, 3) for x in pst2["ms_other"]],
                  "note": "last profiled run, per pass; HIP-event time of each phase's kernels"}
        print("profiled: %.3f ms/step; scan rate %.3g entries/s" % (prof_sec * 1e3, scan_rate or 0),
              file=sys.stderr, flush=True)
        for k in sorted(kernels, key=lambda k: -k["ms_per_step"])[:12]:
            print("  %-20s %8.3f ms/step %9.1f GB/s %6d launches" %
                  (k["name"], k["ms_per_step"],
                   k["bytes_per_step"] / max(k["ms_per_step"], 1e-9) * 1e-6,
                   k["launches"]), file=sys.stderr)

    golden = {}
    gpath = os.path.join(ROOT, "tests", "golden", "reference.json")
    if os.path.exists(gpath):
        golden = json.load(open(gpath)).get(name, {})
    q_ref = golden.get("seq", {}).get("Q")
    del off, tgt, w, memb
    torch.cuda.empty_cache()
    return {
        "value": csr.nnz / sec,
        "ms_per_step": sec * 1e3,
        "config": {"workload": name, "n": csr.n, "nnz": csr.nnz, "mode": args.mode,
                   "round_bits": args.round_bits},
        "roofline": roofline,
        "roofline_move": roof_move,
        "roofline_aggregate": roof_agg,
        "scan_rate": scan_rate,
        "phases": phases,
        "modularity": q,
        "modularity_oracle_seq": q_ref,
        "modularity_delta_vs_oracle": (q - q_ref) if q_ref is not None else None,
        "q_runs": ({"runs": len(q_more), "min": min(q_more), "median": float(np.median(q_more)),
                    "max": max(q_more),
                    "more_than_0.01_below_oracle_seq": (sum(1 for x in q_more if x < q_ref - 0.01)
                                                        if q_ref is not None else None)}
                   if q_more else None),
        "passes": st["passes"],
        "iterations": st["iterations"],
        "communities": st["communities"],
        "per_pass_entries": st["entries"],
        "per_pass_ms": pass_ms,
        "per_pass_edges_per_s": pass_rate,
        "autotune": tuned,
        "colours": st["colours"] if args.mode == "coloured" else None,
        "step_ms": {"median": float(np.median(runs)) * 1e3, "min": min(runs) * 1e3,
                    "max": max(runs) * 1e3},
        "profiled_ms_per_step": prof_sec * 1e3 if prof_sec else None,
        "kernels": sorted(kernels, key=lambda k: -k["ms_per_step"])[:8],
        "first_iteration": {"value": csr.nnz / first_s, "unit": "edges/s",
                            "seconds": round(first_s, 4),
                            "what": "the GPU's first local-moving iteration of pass 1 (%s mode, "
                                    "level setup included), median of 3" % args.mode},
    }


if __name__ == "__main__":
    main()
