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


@pytest.mark.parametrize("wl", ["sbm10k", "rmat14-16"])
@pytest.mark.parametrize("mode,params", [("seq", {}), ("sync", {"seed": 0, "sample_bits": 1})])
def test_lean_pass_loop_is_the_oracle_run(wl, mode, params):
    # the pass loop that writes the full-size records (levels not kept, OpenMP build)
    # gives the oracle's own pass loop's results, pass by pass
    import sys
    sys.path.insert(0, os.path.dirname(GOLDEN))
    from digest import graph_digest, labels_digest
    from make_golden import lean_louvain
    csr = graphgen.workload(wl)
    g = oracle.as_graph(csr.offsets, csr.targets, csr.weights)
    prm = oracle.Params(mode=mode, **params)
    memb, q, passes = lean_louvain(g, prm, lib=oracle.timing_library(), log=lambda m: None)
    memb_o, q_o, recs = oracle.louvain_trace(g, prm)
    assert np.array_equal(memb, memb_o) and q == q_o
    assert len(passes) == len(recs)
    for p, r in zip(passes, recs):
        assert p["iterations"] == r.trace.iterations and p["moves"] == r.trace.moves
        assert p["sumN"] == [str(x) for x in r.trace.sumN]
        assert p["labels"] == labels_digest(r.raw_labels) and p["communities"] == r.communities
        if r.next_level is not None:
            nl = r.next_level
            assert p["next_level"] == graph_digest(nl.offsets, None, nl.targets, nl.weights)
