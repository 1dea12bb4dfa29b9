"""Each graph of a fast-mode batch run against the oracle's sequential run of that graph.

Reads the per-graph modularities that `bench.py --batch G --batch-q-out PATH` writes
(`q_union`: the union run, `q_one_by_one`: every graph alone), regenerates the same seeded
SBM batch on the CPU, runs the oracle's sequential mode on every graph, and prints, per run:
the mean and spread of Q - Q_seq, how many graphs end more than 0.01 / 0.02 below or 0.01
above, and how many equal Q_seq exactly.  For the graphs more than 0.01 below, it also
computes the lowest Q the sequential oracle reaches over the graph's own order and 8 random
relabellings (`seq_floor`, the order spread of the method itself) and counts those within
0.01 of it.  Calls only the oracle and the input generators.

    python3 tests/golden/batch_vs_oracle.py gpurun_out/batch_fast_q.json [--workers 8]
"""
import argparse
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import graphgen  # noqa: E402
import oracle  # noqa: E402
from gpu_util import seq_floor  # noqa: E402

_U = _GO = None


def _load(graphs, seed, n_max):
    global _U, _GO
    _U, _GO, _ = graphgen.batch_sbm(graphs, seed=seed, n_max=n_max)


def _graph(g):
    a, b = int(_GO[g]), int(_GO[g + 1])
    e0, e1 = int(_U.offsets[a]), int(_U.offsets[b])
    return oracle.as_graph((_U.offsets[a:b + 1] - e0).astype(np.int64),
                           (_U.targets[e0:e1] - np.int32(a)).astype(np.int32),
                           _U.weights[e0:e1].astype(np.int32))


def _seq_q(g):
    return oracle.louvain(_graph(g), oracle.Params(mode="seq"))[1]


def _floor(g):
    return seq_floor(_graph(g))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("q_json")
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    qf = json.load(open(args.q_json))
    # the workers are forked after the batch is generated and share it
    _load(qf["graphs"], qf["seed"], qf["batch_nmax"])
    with Pool(args.workers) as pool:
        q_seq = np.array(pool.map(_seq_q, range(qf["graphs"]), chunksize=8))
        for key in ("q_union", "q_one_by_one"):
            q = np.array(qf[key])
            d = q - q_seq
            bad = np.where(d < -0.01)[0]
            floors = np.array(pool.map(_floor, bad.tolist(), chunksize=1)) if bad.size else np.array([])
            within = int((q[bad] >= floors - 0.01).sum()) if bad.size else 0
            print("%s: mean %+.4f, 1st percentile %+.4f, worst %+.4f; below -0.01: %d, below -0.02: %d, "
                  "above +0.01: %d, equal: %d; of those below -0.01, within 0.01 of the order floor: %d"
                  % (key, d.mean(), np.percentile(d, 1), d.min(), bad.size, int((d < -0.02).sum()),
                     int((d > 0.01).sum()), int((d == 0).sum()), within))
            if bad.size:
                print("  worst against the floor: %+.4f" % float((q[bad] - floors).min()))


if __name__ == "__main__":
    main()
