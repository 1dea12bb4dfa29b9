"""Host-side parts of the scheduling autotuner (candidate sets and the cache key)."""
import numpy as np
import torch

import graphgen
from paper_2312_04876_amd import autotune


def test_candidates_cover_both_knobs_and_respect_the_wide_lds_limit():
    narrow = autotune.candidates(wide=False)
    assert narrow == [(r, p) for r in (2048, 4096, 8192) for p in (1024, 2048)]
    wide = autotune.candidates(wide=True)
    assert wide == [(r, p) for r in (2048, 4096) for p in (1024, 2048)]


def test_signature_tells_graphs_apart_and_is_stable():
    a = graphgen.rmat(12, 8, seed=1)
    b = graphgen.sbm(4096, 16, 0.02, 0.001, seed=1)
    def sig(c, **kw):
        return autotune.signature(torch.from_numpy(c.offsets32()), torch.from_numpy(c.weights), **kw)
    assert sig(a, mode="fast") == sig(a, mode="fast")
    assert sig(a, mode="fast") != sig(b, mode="fast")
    assert sig(a, mode="fast") != sig(a, mode="deterministic")
    heavy = torch.from_numpy(np.full(a.nnz, 1 << 20, dtype=np.int32))
    assert autotune.signature(torch.from_numpy(a.offsets32()), heavy, mode="fast").split("-")[2] == "wide"
