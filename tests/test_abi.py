"""The C-ABI library loads, exports every declared symbol and rejects bad arguments
before touching a GPU (host-only calls; no kernels run here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "louvain.h")


@pytest.fixture(scope="module")
def lib():
    import paper_2312_04876_amd as P
    if not os.path.exists(P.binding.LIB_PATH):
        from paper_2312_04876_amd import build
        build.build()
    return P.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(louvain_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    import paper_2312_04876_amd as P
    assert declared_functions() == sorted(P.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_default_params_are_the_papers(lib):
    import paper_2312_04876_amd as P
    p = P.binding.CParams()
    lib.louvain_default_params(ctypes.byref(p))
    assert (p.max_iterations, p.prune, p.tolerance, p.tolerance_drop,
            p.aggregation_tolerance) == (20, 1, 0.01, 10.0, 0.8)
    # round_bits -1: the mode's own round count (8 rounds for one graph in fast mode, else 2)
    assert p.mode == P.DETERMINISTIC and p.max_passes == 10 and p.round_bits == -1


def test_workspace_size_checks(lib):
    import paper_2312_04876_amd as P
    out = ctypes.c_size_t()
    assert lib.louvain_workspace_size(-1, 0, 0, None, ctypes.byref(out)) == P.binding.EINVAL
    assert lib.louvain_workspace_size(10, 2**31, 0, None, ctypes.byref(out)) == \
        P.binding.EOVERFLOW
    assert lib.louvain_workspace_size(10, 20, 20, None, ctypes.byref(out)) == P.binding.OK
    narrow = out.value
    assert lib.louvain_workspace_size(10, 20, -1, None, ctypes.byref(out)) == P.binding.OK
    assert out.value >= narrow
    bad = P.make_params(max_iterations=0)
    assert lib.louvain_workspace_size(10, 20, 20, ctypes.byref(bad), ctypes.byref(out)) == \
        P.binding.EINVAL
    # scheduling knobs: 0 (built-in) or inside the documented ranges
    for kw, ok in (({"hub_rows": 2048}, True), ({"hub_rows": 8192}, True), ({"hub_rows": 2047}, False),
                   ({"hub_rows": 8193}, False), ({"hub_part_pairs": 1024}, True),
                   ({"hub_part_pairs": 2048}, True), ({"hub_part_pairs": 512}, False),
                   ({"hub_part_pairs": 4096}, False)):
        prm = P.make_params(**kw)
        code = lib.louvain_workspace_size(10, 20, 20, ctypes.byref(prm), ctypes.byref(out))
        assert code == (P.binding.OK if ok else P.binding.EINVAL), kw


def test_init_rejects_bad_arguments_without_a_gpu(lib):
    import paper_2312_04876_amd as P
    ctx = ctypes.c_void_p()
    assert lib.louvain_init(None, 1, 0, None, None, None, None, 0, None, None) == P.binding.EINVAL
    assert lib.louvain_init(ctypes.byref(ctx), -1, 0, None, None, None, None, 0, None, None) == \
        P.binding.EINVAL
    fake = ctypes.c_void_p(4096)
    assert lib.louvain_init(ctypes.byref(ctx), 4, 2**31, fake, fake, fake, fake, 1 << 40, None,
                            None) == P.binding.EOVERFLOW
    assert lib.louvain_init(ctypes.byref(ctx), 4, 8, fake, fake, fake, fake, 16, None, None) == \
        P.binding.ENOSPC
    out = ctypes.c_size_t()
    for rb in (9, -2):
        bad = P.make_params(round_bits=rb)
        assert lib.louvain_init(ctypes.byref(ctx), 4, 8, fake, fake, fake, fake, 1 << 40,
                                ctypes.byref(bad), None) == P.binding.EINVAL
        assert lib.louvain_workspace_size(4, 8, 8, ctypes.byref(bad), ctypes.byref(out)) == \
            P.binding.EINVAL
    for rb in (-1, 0, 4):
        assert lib.louvain_workspace_size(4, 8, 8, ctypes.byref(P.make_params(round_bits=rb)),
                                          ctypes.byref(out)) == P.binding.OK
    assert ctx.value is None


def test_calls_on_null_context(lib):
    import paper_2312_04876_amd as P
    i = ctypes.c_int32()
    d = ctypes.c_double()
    assert lib.louvain_move(None, ctypes.byref(i), ctypes.byref(d)) == P.binding.EINVAL
    assert lib.louvain_aggregate(None, None, None) == P.binding.EINVAL
    assert lib.louvain_run(None, None, None, None) == P.binding.EINVAL
    assert lib.louvain_reset(None) == P.binding.EINVAL
    lib.louvain_destroy(None)
    for code in (0, -1, -2, -3, -5, -99):
        assert isinstance(lib.louvain_strerror(code), bytes)


def test_product_path_does_not_import_the_oracle():
    # the GPU package must not reach the CPU oracle or any fallback
    pkg = os.path.join(ROOT, "paper_2312_04876_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "louvain_oracle" not in text, f


def test_batch_workspace_size_checks(lib):
    import paper_2312_04876_amd as P
    out = ctypes.c_size_t()
    assert lib.louvain_batch_workspace_size(0, 10, 20, 20, None, ctypes.byref(out)) == \
        P.binding.EINVAL
    assert lib.louvain_batch_workspace_size(3, 10, 20, 20, None, ctypes.byref(out)) == P.binding.OK
    batch = out.value
    assert lib.louvain_workspace_size(10, 20, 20, None, ctypes.byref(out)) == P.binding.OK
    assert batch > out.value


def test_batch_init_rejects_bad_arguments_before_any_kernel(lib):
    import paper_2312_04876_amd as P
    ctx = ctypes.c_void_p()
    assert lib.louvain_init_batch(ctypes.byref(ctx), 0, None, 0, 0, None, None, None, None, 0,
                                  None, None) == P.binding.EINVAL
    assert lib.louvain_batch_results(None, None, None) == P.binding.EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # without the built library the package raises; it never falls back to CPU code
    from paper_2312_04876_amd import binding
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "liblouvain.so"))
    with pytest.raises(RuntimeError, match="not built"):
        binding.load_library()


def test_noalloc_rejects_sizes_beyond_its_array_before_any_gpu_call(lib):
    # the size checks come before the device lookup: no pointer is touched
    import paper_2312_04876_amd as P
    text = open(HEADER).read()
    m = re.search(r"#define LOUVAIN_NOALLOC_BYTES \((\d+)ull << (\d+)\)", text)
    assert m and (int(m.group(1)) << int(m.group(2))) == P.NOALLOC_BYTES
    q = ctypes.c_double()
    # a graph whose workspace exceeds the array
    assert lib.louvain_run_noalloc(1 << 20, 1 << 25, None, None, None, None, None,
                                   ctypes.byref(q), None, None) == P.binding.ENOSPC
    # just below and above the limit, by the documented size rule
    out = ctypes.c_size_t()
    n = 20000
    lo, hi = 1, 1 << 24
    while lo < hi:  # largest nnz that fits
        mid = (lo + hi + 1) // 2
        lib.louvain_workspace_size(n, mid, -1, None, ctypes.byref(out))
        if out.value <= P.NOALLOC_BYTES:
            lo = mid
        else:
            hi = mid - 1
    assert lib.louvain_run_noalloc(n, lo + 1, None, None, None, None, None, ctypes.byref(q),
                                   None, None) == P.binding.ENOSPC
    prof = P.make_params(profile=True)
    assert lib.louvain_run_noalloc(10, 20, None, None, None, ctypes.byref(prof), None,
                                   ctypes.byref(q), None, None) == P.binding.EINVAL
    assert lib.louvain_run_noalloc(-1, 0, None, None, None, None, None, ctypes.byref(q), None,
                                   None) == P.binding.EINVAL
