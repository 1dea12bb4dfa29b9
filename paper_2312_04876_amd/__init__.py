"""MI355X-native Louvain hot path (GVE-Louvain, arXiv 2312.04876).

The local-moving and aggregation phases run in hand-written HIP kernels for
gfx950 behind the C ABI of ``include/louvain.h`` (``liblouvain.so``, built
in-tree by ``paper_2312_04876_amd.build``); this package is its Python
binding.  There is no CPU fallback: without the built library every entry
point raises.
"""
from .binding import (DETERMINISTIC, FAST, EXPORTS, NOALLOC_BYTES, Louvain, LouvainError,
                      batch_workspace_bytes, load_library, louvain, louvain_noalloc, make_params,
                      strerror, workspace_bytes)

__all__ = ["DETERMINISTIC", "FAST", "EXPORTS", "NOALLOC_BYTES", "Louvain", "LouvainError",
           "batch_workspace_bytes", "load_library", "louvain", "louvain_noalloc", "make_params",
           "strerror", "workspace_bytes"]
