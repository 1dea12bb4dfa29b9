"""louvain_run_noalloc (the library's own device scratch array as the workspace)
against louvain_init + louvain_run on the same graphs: bit for bit in deterministic
mode, two calls in a row with the second on a smaller graph (the array keeps the
first call's contents), then fast mode to its tolerance."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import is_valid_partition, to_device

pytestmark = pytest.mark.gpu


def _noalloc(csr, **params):
    import torch
    import paper_2312_04876_amd as P
    off, tgt, w = to_device(csr)
    memb = torch.full((max(csr.n, 1),), -1, dtype=torch.int32, device="cuda")
    q, st = P.louvain_noalloc(off, tgt, w, memb, **params)
    torch.cuda.synchronize()
    return memb[:csr.n].cpu().numpy(), q, st


def test_noalloc_equals_the_workspace_entry_point_on_two_calls():
    import paper_2312_04876_amd as P
    for wl in ("rmat14-16", "sbm10k"):  # the second graph is smaller
        csr = graphgen.workload(wl)
        need = P.workspace_bytes(csr.n, csr.nnz, -1, P.make_params())
        assert need <= P.NOALLOC_BYTES
        print("noalloc deterministic:", wl, csr.n, csr.nnz, "workspace", need, flush=True)
        m1, q1, st1 = _noalloc(csr, mode="deterministic")
        m0, q0, st0 = P.louvain(*to_device(csr), mode="deterministic")
        assert np.array_equal(m1, m0.cpu().numpy()), wl
        assert q1 == q0 and st1 == st0, wl


def test_noalloc_fast_mode_within_tolerance():
    csr = graphgen.workload("rmat14-16")
    print("noalloc fast: rmat14-16", flush=True)
    m, q, _ = _noalloc(csr, mode="fast")
    g = oracle.as_graph(csr.offsets, csr.targets, csr.weights)
    assert is_valid_partition(m)
    assert q == oracle.modularity(g, m)
    _, q_seq, _ = oracle.louvain(g, oracle.Params(mode="seq"))
    assert abs(q - q_seq) <= 0.01


def test_noalloc_rejects_a_graph_beyond_the_array():
    import paper_2312_04876_amd as P
    csr = graphgen.workload("rmat16-16")
    assert P.workspace_bytes(csr.n, csr.nnz, -1, P.make_params()) > P.NOALLOC_BYTES
    print("noalloc: rmat16-16 must be rejected", flush=True)
    with pytest.raises(P.LouvainError) as e:
        _noalloc(csr)
    assert e.value.code == P.binding.ENOSPC
