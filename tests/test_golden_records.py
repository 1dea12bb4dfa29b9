"""The stored oracle records (tests/golden/reference.json) are what the oracle
computes now, for the workloads small enough to rerun in the CPU suite."""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "reference.json")


def _digest(memb):
    return hashlib.sha256(np.ascontiguousarray(memb, dtype=np.int32).tobytes()).hexdigest()


@pytest.mark.parametrize("wl", ["sbm10k", "rmat16-16"])
@pytest.mark.parametrize("mode,params", [("seq", {}), ("sync", {"seed": 0, "sample_bits": 1}),
                                         ("colour", {"seed": 0})])
def test_stored_record_is_the_oracle_run(wl, mode, params):
    ref = json.load(open(GOLDEN))[wl][mode]
    csr = graphgen.workload(wl)
    g = oracle.as_graph(csr.offsets, csr.targets, csr.weights)
    memb, q, r = oracle.louvain(g, oracle.Params(mode=mode, **params))
    assert _digest(memb) == ref["digest"] and q == ref["Q"]
    assert r["iterations"] == ref["iterations"] and r["communities"] == ref["communities"]
