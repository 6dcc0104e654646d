"""The C-ABI library loads, exports every symbol include/*.h declares, and
rejects bad arguments on the host before any launch (CPU only: no call here
reaches a kernel or the HIP runtime)."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lc[a-z]*_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_1804_09996_amd as lc
    return lc.lib()


def test_headers_declare_the_three_calls():
    names = _declared(os.path.join(ROOT, "include", "lc.h"))
    for n in ("lc_build_lut", "lc_search", "lc_refine", "lc_index_bind", "lc_search_workspace_bytes"):
        assert n in names


@pytest.mark.parametrize("header", sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))))
def test_every_declared_symbol_is_exported(header):
    import paper_1804_09996_amd as lc
    libs = {"lc.h": os.path.join(ROOT, "paper_1804_09996_amd", "liblc.so"),
            "lc_build.h": os.path.join(ROOT, "paper_1804_09996_amd", "liblc_build.so")}
    path = libs[os.path.basename(header)]
    so = C.CDLL(path)
    for name in _declared(header):
        assert hasattr(so, name), f"{name} declared in {os.path.basename(header)} but not exported by {path}"
    if os.path.basename(header) == "lc.h":
        assert sorted(lc.exported_symbols()) == _declared(header)


def test_strerror(L):
    assert L.lc_strerror(0) == b"ok"
    assert L.lc_strerror(2) == b"workspace too small"
    assert L.lc_strerror(99) == b"unknown error"


def test_bind_rejects_bad_views(L):
    import paper_1804_09996_amd as lc
    h = C.c_void_p(1)
    assert L.lc_index_bind(None, C.byref(h)) == lc.LC_EINVAL and h.value is None
    v = lc.IndexView()
    assert L.lc_index_bind(C.byref(v), C.byref(h)) == lc.LC_EINVAL  # n = 0

    def good():
        g = lc.IndexView()
        g.n, g.d, g.d_pad, g.m, g.ksub, g.code_stride = 100, 96, 96, 16, 256, 16
        g.deg0, g.deg_up, g.k_reg, g.n_beta, g.entry, g.max_level, g.n_up_rows = 32, 32, 16, 256, 0, 0, 0
        g.m_beta = 1
        for name in ("centroids", "codes", "adj0", "up_base", "beta", "beta_idx"):
            setattr(g, name, 0x1000)
        return g

    cases = {
        "ksub": ("ksub", 16, lc.LC_EINVAL), "stride": ("code_stride", 8, lc.LC_EINVAL),
        "stride_big": ("code_stride", 64, lc.LC_EINVAL), "kreg": ("k_reg", 33, lc.LC_EINVAL),
        "nbeta": ("n_beta", 257, lc.LC_EINVAL), "entry": ("entry", 100, lc.LC_EINVAL),
        "dpad": ("d_pad", 100, lc.LC_EINVAL), "codes": ("codes", None, lc.LC_EINVAL),
        "deg0": ("deg0", 48, lc.LC_ENOTSUP), "level_rows": ("max_level", 2, lc.LC_EINVAL),
        "mbeta0": ("m_beta", 0, lc.LC_EINVAL), "mbeta3": ("m_beta", 3, lc.LC_EINVAL),  # blocks must divide m
    }
    for key, (field, value, want) in cases.items():
        g = good()
        setattr(g, field, value)
        if key == "deg0":
            g.k_reg = 16
        assert L.lc_index_bind(C.byref(g), C.byref(h)) == want, key
    g = good()
    g.m, g.code_stride = 12, 16  # m must be a multiple of 8
    assert L.lc_index_bind(C.byref(g), C.byref(h)) == lc.LC_ENOTSUP
    g = good()
    g.d_pad, g.proj = 112, None  # a projection is required when d_pad != d
    assert L.lc_index_bind(C.byref(g), C.byref(h)) == lc.LC_EINVAL


def test_calls_reject_bad_arguments_before_launch(L):
    import paper_1804_09996_amd as lc
    p = C.c_void_p(0x1000)
    assert L.lc_build_lut(None, p, 1, 0, p, None, None) == lc.LC_EINVAL
    assert L.lc_search(None, p, 0, None, 1, None, 8, 8, p, p, p, None, p, 1, None) == lc.LC_EINVAL
    assert L.lc_refine(None, p, 1, p, p, 8, 8, 0, p, p, None) == lc.LC_EINVAL
    assert L.lc_search_workspace_bytes(None, 1, 8, 8) == 0
    assert L.lc_search_budget(None, p, 0, None, 1, None, 8, 8, 10, None, p, p, p, None, p, 1, None, None) == \
        lc.LC_EINVAL
    assert L.lc_assign_beta(None, p, 0, 1, p, None) == lc.LC_EINVAL
    assert L.lc_project_queries(None, p, 1, p, None) == lc.LC_EINVAL
    assert L.lc_build_lut_projected(None, p, 1, 0, p, None, None) == lc.LC_EINVAL
    assert L.lc_refine_projected(None, p, 1, p, p, 8, 8, 0, p, p, None) == lc.LC_EINVAL


def test_library_is_built_from_these_sources(L):
    # a library built from other sources (another lc_index_view layout, an
    # older kernel) must never be loaded
    from paper_1804_09996_amd import build_ext
    assert L.lc_build_id().decode() == build_ext.source_id()


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    # no CPU fallback: without liblc.so every entry point raises instead of computing elsewhere
    import paper_1804_09996_amd as lc
    monkeypatch.setattr(lc, "LIB_PATH", str(tmp_path / "absent" / "liblc.so"))
    monkeypatch.setattr(lc, "_lib", None)
    with pytest.raises(ImportError, match="no CPU fallback"):
        lc.lib()
    with pytest.raises(ImportError):
        lc.Index({"codes": np.zeros((4, 8), np.uint8)}, {"d": 8, "d_pad": 8, "m": 8, "deg0": 32, "deg_up": 32,
                                                         "k_reg": 1, "entry": 0, "max_level": 0}, device="cpu")


def test_bind_rejects_bad_two_level_views(L):
    # 2-level codec fields: coarse_k in [0, 65536], an even d_pad, all three arrays, 4-byte aligned codes
    import paper_1804_09996_amd as lc
    h = C.c_void_p()

    def coarse():
        g = lc.IndexView()
        g.n, g.d, g.d_pad, g.m, g.ksub, g.code_stride = 100, 96, 96, 16, 256, 16
        g.deg0, g.deg_up, g.k_reg, g.n_beta, g.entry, g.max_level, g.n_up_rows = 32, 32, 16, 256, 0, 0, 0
        g.m_beta = 1
        for name in ("centroids", "codes", "adj0", "up_base", "beta", "beta_idx", "coarse_cent", "coarse_codes",
                     "coarse_norm"):
            setattr(g, name, 0x1000)
        g.coarse_k = 64
        return g

    for field, value in (("coarse_k", -1), ("coarse_k", 65537), ("coarse_cent", None), ("coarse_codes", None),
                         ("coarse_norm", None), ("coarse_codes", 0x1002)):
        g = coarse()
        setattr(g, field, value)
        assert L.lc_index_bind(C.byref(g), C.byref(h)) == lc.LC_EINVAL, (field, value)
    g = coarse()
    g.d, g.d_pad, g.m, g.code_stride, g.proj = 8, 9, 1, 1, 0x1000  # odd d_pad: the first level halves the vector
    assert L.lc_index_bind(C.byref(g), C.byref(h)) == lc.LC_EINVAL
    assert L.lc_lut_stride(None, 0) == 0
