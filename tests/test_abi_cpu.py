"""C-ABI checks that need no GPU: the built library loads, exports every
function include/mm.h declares, rejects invalid arguments synchronously, and
round-trips its autotune cache."""
import ctypes
import json
import os
import re

import pytest

from paper_2408_15384_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mm.h")


def declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return api.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(n for n, _, _ in api.EXPORTS) == names   # binding declares exactly the header


def test_peak_library_exports_its_header():
    # the MFMA-only measurement aid is a library of its own beside libmm
    import torch  # noqa: F401  -- same HIP runtime binding order as libmm
    from paper_2408_15384_amd import build as B
    peak = ctypes.CDLL(B.PEAK_LIB)
    names = declared_functions(os.path.join(ROOT, "include", "mm_peak.h"))
    assert names == ["mm_peak_mfma", "mm_peak_overlap"]
    assert all(hasattr(peak, n) for n in names)
    fn = peak.mm_peak_mfma
    fn.restype = ctypes.c_int32
    fn.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    assert fn(3, 8, 1, 1, 1024, None) == -1      # bad dtype: rejected before any launch
    assert fn(0, 12, 1, 1, 1024, None) == -1     # unsupported chain count
    assert fn(0, 8, 0, 1, 1024, None) == -1      # no blocks
    assert fn(0, 8, 1, 1, None, None) == -1      # no output
    ov = peak.mm_peak_overlap
    ov.restype = ctypes.c_int32
    ov.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    assert ov(3, 1, 1, 1024, None) == -1         # bad role
    assert ov(0, 0, 1, 1024, None) == -1         # no blocks
    assert ov(0, 1, 0, 1024, None) == -1         # no iterations
    assert ov(0, 1, 1, None, None) == -1         # no output


def test_status_strings(lib):
    assert lib.mm_status_string(api.MM_E_INVAL) == b"invalid argument"
    assert lib.mm_version().startswith(b"libmm")


def test_invalid_arguments_without_gpu(lib):
    p = 1 << 20
    assert lib.mm_gemm_f64(-1, 4, 4, p, 4, p, 4, p * 4, 4, None) == api.MM_E_INVAL
    assert lib.mm_gemm_f64(4, 4, 5, p, 4, p, 4, p * 4, 4, None) == api.MM_E_INVAL      # lda < K
    assert lib.mm_gemm_f32(4, 4, 4, p, 4, p, 3, p * 4, 4, None) == api.MM_E_INVAL      # ldb < N
    assert lib.mm_gemm_f64(4, 4, 4, p, 4, p + 4096, 4, p + 8, 4, None) == api.MM_E_INVAL  # C overlaps A
    assert b"overlap" in lib.mm_last_error()
    assert lib.mm_gemm_f64(0, 4, 4, None, 4, None, 4, None, 4, None) == api.MM_OK      # empty: no-op
    assert lib.mm_gemm_split_bf16(4, 4, 4, p, 4, p, 4, p * 4, 4, 0, 4, None, 0, None) == api.MM_E_INVAL
    assert lib.mm_split_bf16(4, 4, p, 4, 4, 0, p * 4, 16, None) == api.MM_E_INVAL      # nplanes
    assert lib.mm_split_workspace_bytes(8, 8, 8, 6) > 0
    assert lib.mm_split_workspace_bytes(8, 8, 8, 5) == 0
    probs = (api.Problem * 1)(api.Problem(4, 4, 4, p, 2, p, 4, p * 4, 4))
    assert lib.mm_gemm_grouped(probs, 1, api.MM_F64, None, None) == api.MM_E_INVAL
    assert b"problem 0" in lib.mm_last_error()
    assert lib.mm_gemm_grouped(probs, 0, api.MM_F64, None, None) == api.MM_OK
    assert lib.mm_gemm_grouped_config(probs, 0, api.MM_F64, 0, 4, None, None) == api.MM_E_INVAL   # schedule 0..3
    assert b"schedule" in lib.mm_last_error()
    assert lib.mm_gemm_grouped_config(probs, 0, api.MM_F64, 0, 3, None, None) == api.MM_OK


def test_extent_overflow_rejected_by_every_product_entry_point(lib):
    # a leading dimension that makes (rows-1)*ld + cols exceed 2^62 elements
    # is refused before any device work, transposed layouts and the residual
    # probe included (the addresses are never dereferenced)
    a, b, c, x = 1 << 40, 1 << 41, 1 << 42, 1 << 43
    huge = 1 << 61
    E = api.MM_E_INVAL
    assert lib.mm_gemm_f64(8, 2, 2, a, huge, b, 2, c, 2, None) == E
    assert b"overflow" in lib.mm_last_error()
    for m in (api.MM_F64, api.MM_F32, api.MM_SPLIT_BF16_6):
        # A stored transposed: K x M rows of length M, ld huge
        assert lib.mm_gemm_ex(m, 1, 0, 2, 2, 8, a, huge, b, 2, c, 2, None, 0, None) == E
        assert b"overflow" in lib.mm_last_error()
        # B stored transposed: N x K
        assert lib.mm_gemm_ex(m, 0, 1, 2, 8, 2, a, 2, b, huge, c, 8, None, 0, None) == E
    assert lib.mm_gemm_ex(api.MM_F64, 0, 0, 2, 2, (1 << 40) + 1, a, (1 << 40) + 1, b, 2, c, 2, None, 0, None) == E
    out = ctypes.c_double()
    assert lib.mm_residual_f64(8, 2, 2, a, 2, b, 2, c, huge, 0, 0, x, ctypes.byref(out), None, 0, None) == E
    assert b"overflow" in lib.mm_last_error()
    assert lib.mm_split_bf16(8, 2, a, huge, 2, 0, b, 16, None) == E
    assert lib.mm_split_bf16(1 << 31, 1 << 31, a, 1 << 31, 2, 0, b, 1 << 62, None) == E


def test_split_k_limit_without_gpu(lib):
    # the split tiles address 16 plane rows with 32-bit byte offsets: K above
    # 2^26 - 32 is refused by every entry point that takes a split method,
    # before any device work (the addresses below are never dereferenced)
    kmax = (1 << 26) - 32
    K = kmax + 1
    a, b, c = 1 << 40, 1 << 41, 1 << 42
    E = api.MM_E_UNSUPPORTED
    assert lib.mm_gemm_split_bf16(2, 2, K, a, K, b, 2, c, 2, 0, 6, None, 0, None) == E
    assert b"2^26" in lib.mm_last_error()
    for m in (api.MM_SPLIT_BF16_3, api.MM_SPLIT_BF16_6):
        assert lib.mm_gemm_ex(m, 0, 0, 2, 2, K, a, K, b, 2, c, 2, None, 0, None) == E
        assert lib.mm_gemm_variant(m, 0, 2, 2, K, a, K, b, 2, c, 2, None, 0, None) == E
        probs = (api.Problem * 1)(api.Problem(2, 2, K, a, K, b, 2, c, 2))
        assert lib.mm_gemm_grouped(probs, 1, m, None, None) == E
        assert b"problem 0" in lib.mm_last_error()


def test_variant_tables(lib):
    for m in ("f64", "f32", "split3", "split6"):
        n = api.variant_count(m)
        assert n >= 3
        for v in range(n):
            bm, bn, bk = api.variant_info(m, v)
            assert bm % 16 == 0 and bn % 16 == 0 and bk % 4 == 0
        with pytest.raises(api.MMError):
            api.variant_info(m, n)
    # selection is a pure function of the shape: large products take a
    # large tile (binary64 128x128 with 16 waves, FP32 256x256, the split
    # methods 256x128), small ones a tile of at most 64x64
    assert api.select_variant("f64", 8192, 8192, 8192) == api.select_variant("f64", 8192, 8192, 8192)
    for m in ("f64", "f32", "split3", "split6"):
        big = {"f64": (128, 128), "f32": (256, 256)}.get(m, (256, 128))
        assert api.variant_info(m, api.select_variant(m, 8192, 8192, 8192))[:2] == big
        bm, bn, _ = api.variant_info(m, api.select_variant(m, 256, 256, 256))
        assert bm <= 64 and bn <= 64


def test_grouped_pairs(lib):
    # size-class pairs: two variants of one workgroup size per pair, ids from
    # MM_PAIR_BASE (the value the binding mirrors), accepted by the grouped
    # entry points' argument checks and rejected past the table
    hdr = open(HEADER).read()
    assert re.search(r"#define MM_PAIR_BASE (\d+)", hdr).group(1) == str(api.PAIR_BASE)
    for m in ("f64", "f32", "split3", "split6"):
        n = api.grouped_pair_count(m)
        assert n >= 2
        for p in range(n):
            small, large, pct = api.grouped_pair_info(m, p)
            bs, bl = api.variant_info(m, small), api.variant_info(m, large)
            assert bs[0] * bs[1] < bl[0] * bl[1] and bs[2] == bl[2]   # smaller tile, same K step
            assert 0 < pct <= 100
            if m.startswith("split"):
                assert small >= 15 and large >= 15                   # ring-fused members
        with pytest.raises(api.MMError):
            api.grouped_pair_info(m, n)
        with pytest.raises(api.MMError):
            api.grouped_pair_info(m, -1)
    p = 1 << 20
    probs = (api.Problem * 1)(api.Problem(4, 4, 4, p, 4, p, 4, p * 4, 4))
    n = api.grouped_pair_count("f64")
    assert lib.mm_gemm_grouped_config(probs, 0, api.MM_F64, api.PAIR_BASE + n - 1, 3, None, None) == api.MM_OK
    assert lib.mm_gemm_grouped_config(probs, 0, api.MM_F64, api.PAIR_BASE + n, 3, None, None) == api.MM_E_INVAL
    assert b"pair" in lib.mm_last_error()
    assert lib.mm_gemm_grouped_config(probs, 0, api.MM_F64, api.variant_count("f64"), 3, None, None) == api.MM_E_INVAL


def test_autotune_cache_roundtrip(lib, tmp_path):
    path = str(tmp_path / "cache.json")
    api.autotune_clear()
    api.autotune_save(path)
    doc = json.load(open(path))
    assert doc["arch"] == "gfx950" and doc["entries"] == []
    # an entry selecting a non-default variant changes selection after load
    default = api.select_variant("f64", 1000, 1000, 1000)
    default_4000 = api.select_variant("f64", 4000, 1000, 1000)
    other = (default + 1) % api.variant_count("f64")
    doc["entries"] = [[api.MM_F64, 10, 10, 10, other, 1.5, 0]]
    json.dump(doc, open(path, "w"))
    api.autotune_load(path)
    assert api.select_variant("f64", 1000, 1000, 1000) == other
    assert api.select_variant("f64", 4000, 1000, 1000) == default_4000  # other bucket untouched
    api.autotune_save(path)
    assert json.load(open(path))["entries"][0][4] == other
    # wrong architecture or bad variant: rejected, cache unchanged
    bad = dict(doc, arch="gfx942")
    json.dump(bad, open(path, "w"))
    with pytest.raises(api.MMError):
        api.autotune_load(path)
    doc["entries"] = [[api.MM_F64, 10, 10, 10, 99, 1.5, 0]]
    json.dump(doc, open(path, "w"))
    with pytest.raises(api.MMError):
        api.autotune_load(path)
    # a size-class pair is a grouped variant only
    doc["entries"] = [[api.MM_F64, 10, 10, 10, api.PAIR_BASE, 1.5, 0]]
    json.dump(doc, open(path, "w"))
    with pytest.raises(api.MMError):
        api.autotune_load(path)
    doc["entries"] = [[100 + api.MM_F64, 9, 18, 9, api.PAIR_BASE, 1.5, 3],
                      [100 + api.MM_F64, 9, 18, 10, api.PAIR_BASE + api.grouped_pair_count("f64"), 1.5, 3]]
    json.dump(doc, open(path, "w"))
    with pytest.raises(api.MMError):
        api.autotune_load(path)
    assert api.select_variant("f64", 1000, 1000, 1000) == other
    api.autotune_clear()
    assert api.select_variant("f64", 1000, 1000, 1000) == default
    doc["entries"] = [[100 + api.MM_F64, 9, 18, 9, api.PAIR_BASE + 1, 1.5, 3]]
    json.dump(doc, open(path, "w"))
    api.autotune_load(path)
    api.autotune_save(path)
    assert json.load(open(path))["entries"] == [[100 + api.MM_F64, 9, 18, 9, api.PAIR_BASE + 1, 1.5, 3]]
    api.autotune_clear()


def test_binding_rejects_views_that_are_not_row_major_matrices():
    """Expanded or broadcast views have overlapping rows (row stride below the
    row length); the binding must refuse them rather than hand the kernels a
    leading dimension that walks past the tensor's storage."""
    torch = pytest.importorskip("torch")
    base = torch.zeros(6, 8, dtype=torch.float64)
    assert api.row_major_ld(base) == 8
    assert api.row_major_ld(base[:, :5]) == 8          # column slice: padded rows
    assert api.row_major_ld(base[2:3, 1:4]) == 3       # one row: its length
    assert api.row_major_ld(base[:0]) == 8             # empty
    with pytest.raises(ValueError, match="not a row-major matrix"):
        api.row_major_ld(torch.zeros(1, 8).expand(6, 8))          # stride(0) == 0
    with pytest.raises(ValueError, match="not a row-major matrix"):
        api.row_major_ld(torch.zeros(40).as_strided((6, 8), (4, 1)))   # overlapping rows
    with pytest.raises(ValueError, match="row-major"):
        api.row_major_ld(base.t())                      # column-major view
    with pytest.raises(ValueError, match="GPU tensor"):
        api._ld(base, "A")
