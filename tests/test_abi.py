"""The C-ABI library loads and exports every symbol include/lbm.h declares
(no device calls: runs without a GPU)."""
import ctypes
import os

import pytest

from paper_1303_0107_amd import lbm

EXPECTED = {
    "lbm_create_geometry", "lbm_run_to_steady", "lbm_outlet_stats", "lbm_shape_update",
    "lbm_last_exchange", "lbm_get_mask", "lbm_get_macro", "lbm_get_state", "lbm_set_state",
    "lbm_footprint_bytes", "lbm_device_bytes", "lbm_destroy", "lbm_last_error", "lbm_bench_sweep",
    "lbm_profile_sweeps", "lbm_tb_variant_count", "lbm_tb_variant_info", "lbm_tb_variant_kind",
    "lbm_set_tb_variant", "lbm_autotune", "lbm_batch_create", "lbm_batch_run",
    "lbm_batch_configure", "lbm_batch_tune", "lbm_batch_info", "lbm_batch_destroy",
    "lbm_batch_set_graphs", "lbm_state_digest", "lbm_server_create", "lbm_server_submit",
    "lbm_server_poll", "lbm_server_drain", "lbm_server_stats_get", "lbm_server_destroy",
    "lbm_precision_info", "lbm_outlet_stats_noalloc", "lbm_get_tb_variant",
    "lbm_shape_update_many",
}


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1303_0107_amd import _build
        _build.build()
    return lbm.load()


def test_header_declares_the_boundary():
    assert set(lbm.declared_functions()) == EXPECTED


def test_library_exports_every_declared_symbol(lib):
    for name in lbm.declared_functions():
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    # sizes implied by the header's field lists (natural alignment, x86-64)
    assert ctypes.sizeof(lbm.lbm_geometry_desc) == 4 * 12 + 3 * 8 + 8
    assert ctypes.sizeof(lbm.lbm_stats) == 8 + 16 + 7 * 8 + 8 + 8
    assert ctypes.sizeof(lbm.lbm_shape_params) == 8 + 8 + 16
    assert ctypes.sizeof(lbm.lbm_server_config) == 8 + 16
    assert ctypes.sizeof(lbm.lbm_request) == ctypes.sizeof(lbm.lbm_geometry_desc) + 8 + 16 + 32
    assert ctypes.sizeof(lbm.lbm_result) == 8 + 8 + 8 + 8 + 8 + 24 + ctypes.sizeof(lbm.lbm_stats)
    assert ctypes.sizeof(lbm.lbm_server_stats) == 8 * 8 + 4 * 8 + 8 + 3 * 8
    assert ctypes.sizeof(lbm.lbm_shape_result) == 8 + 32 + 16


def test_footprint_and_validation_need_no_device(lib):
    d = lbm.make_desc(1024, 512, 0.6, 0.04, precision=lbm.LBM_F32)
    fp = lbm.lbm_footprint_bytes(d)
    # two buffers of nine float planes dominate
    assert fp >= 2 * 9 * 1024 * 512 * 4
    bad = lbm.make_desc(1024, 512, 0.5, 0.04)
    assert lbm.lbm_footprint_bytes(bad) == 0
    bad = lbm.make_desc(2, 512, 0.6, 0.04)
    assert lbm.lbm_footprint_bytes(bad) == 0
    # work lists pack tile columns and rows into 16 and 15 bits: sides <= 65536
    assert lbm.lbm_footprint_bytes(lbm.make_desc(65536, 16, 0.6, 0.04)) > 0
    assert lbm.lbm_footprint_bytes(lbm.make_desc(65537, 16, 0.6, 0.04)) == 0
    assert lbm.lbm_footprint_bytes(lbm.make_desc(16, 65537, 0.6, 0.04)) == 0


def test_invalid_descriptor_is_rejected_before_any_device_call(lib):
    d = lbm.make_desc(64, 32, 0.4, 0.04)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create_geometry(d, None, None)
    assert e.value.code == lbm.LBM_EINVAL
    assert "tau" in lbm.lbm_last_error()


def test_region_shapes_fit_the_chip(lib):
    """Host-only queries: every compiled shape leaves an interior tile, its
    region copies (two, or one updated in place) and cell list fit 160 KB,
    and rows split evenly over 16 waves."""
    sizes = {lbm.LBM_F64: 8, lbm.LBM_F32: 4, lbm.LBM_F32_S_F16: 2, lbm.LBM_F32_S_BF16: 2}
    for prec, es in sizes.items():
        n = lbm.lbm_tb_variant_count(prec)
        assert n >= 2
        for v in range(n):
            rows, halo, tw, th = lbm.lbm_tb_variant_info(prec, v)
            assert tw == 64 - 2 * halo and th == rows - 2 * halo and th > 0
            kind, lds = lbm.lbm_tb_variant_kind(prec, v)
            copies = 1 if kind == lbm.LBM_TB_INPLACE else 2
            listed = 64 * rows * 4 if kind == lbm.LBM_TB_COMPACT else 0
            assert kind in (lbm.LBM_TB_DENSE, lbm.LBM_TB_COMPACT, lbm.LBM_TB_INPLACE)
            assert lds == copies * 9 * 64 * rows * es + listed <= 160 * 1024
            assert rows % 16 == 0
        with pytest.raises(lbm.LbmError):
            lbm.lbm_tb_variant_info(prec, n)
    assert lbm.lbm_tb_variant_count(99) == 0


def test_precision_comments_match_the_build(lib):
    """Each precision form's comment in the header names its storage and its
    arithmetic ("stored in X, relaxed in Y"); the library reports the sizes
    of the types it was built with."""
    import re
    txt = open(lbm.HEADER_PATH).read()
    block = txt[txt.index("---- precision forms"):txt.index("#define LBM_F64")]
    block = " ".join(line.strip().lstrip("*").strip() for line in block.splitlines())
    sizes = {"double": 8, "float": 4, "half": 2, "bfloat16": 2}
    found = re.findall(r"(LBM_F\w+):.*?stored in (\w+).*?relaxed in (\w+)", block)
    assert [f[0] for f in found] == ["LBM_F64", "LBM_F32", "LBM_F32_S_F16", "LBM_F32_S_BF16"]
    for name, stored, relaxed in found:
        sb, ab = lbm.lbm_precision_info(getattr(lbm, name))
        assert (sb, ab) == (sizes[stored], sizes[relaxed]), name
    with pytest.raises(lbm.LbmError):
        lbm.lbm_precision_info(7)
