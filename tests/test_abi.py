"""The C-ABI library loads and exports every symbol include/fastatlas.h
declares; host-side argument checks (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastatlas.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|void|const char\*)\s+(fa_\w+)\s*\(", txt,
                                 re.M)))


def test_library_exports_every_declared_symbol():
    import paper_2502_17712_amd as fa
    lib = ctypes.CDLL(fa.LIB_PATH)
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(fa.EXPORTS) == names


def test_struct_layouts():
    import paper_2502_17712_amd as fa
    assert ctypes.sizeof(fa.fa_config) == 64
    assert ctypes.sizeof(fa.fa_mesh) == 40
    assert ctypes.sizeof(fa.fa_camera) == 72
    assert ctypes.sizeof(fa.fa_atlas_out) == 56
    assert fa.CHART_DTYPE.itemsize == 64 and fa.META_DTYPE.itemsize == 64


def test_create_rejects_bad_config_on_host():
    import paper_2502_17712_amd as fa
    h = ctypes.c_void_p()
    assert fa.fa_create(None, ctypes.byref(h)) == fa.FA_ERR_INVALID_ARG
    fp = fa.FA_FLAG_FOOTPRINT_PUSH
    for bad in (dict(num_scales=65), dict(max_atlas=1000), dict(max_charts=-1),
                dict(max_atlas=16384), dict(gutter=-1), dict(flags=fp, gutter=0),
                dict(flags=fp, max_profile_columns=(1 << 28) + 1),
                dict(flags=fp, max_profile_columns=-5), dict(hbm_budget_bytes=-1)):
        kw = dict(device=0, num_scales=64, max_triangles=10, max_vertices=10, max_charts=16,
                  max_atlas=1024, gutter=1, min_box=2, flags=0, max_views=1)
        kw.update(bad)
        cfg = fa.fa_config(**kw)
        assert fa.fa_create(ctypes.byref(cfg), ctypes.byref(h)) == fa.FA_ERR_INVALID_ARG, bad
        assert not h.value
    assert fa.fa_status_string(fa.FA_ERR_NOFIT) == b"no candidate scale fits the atlas"


def test_tuning_table_rejects_null_arguments():
    import paper_2502_17712_amd as fa
    assert fa.fa_load_tuning_table(None, b"") == fa.FA_ERR_INVALID_ARG

