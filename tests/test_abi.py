"""The C-ABI library loads and exports every entry point the header
declares; argument checks that happen before any device work (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "peanut.h")


@pytest.fixture(scope="module")
def pn():
    from paper_1403_1706_amd import peanut
    return peanut


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pn_[a-z_]+)\s*\(", text)))


def test_header_declares_the_path():
    names = declared_functions()
    for must in ("pn_index_build", "pn_index_build_dev", "pn_map", "pn_map_dev", "pn_ref_load",
                 "pn_filter", "pn_validate"):
        assert must in names


def test_library_exports_every_declared_symbol(pn):
    lib = ctypes.CDLL(pn.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(pn.EXPORTED) == declared_functions()


def test_strerror_covers_codes(pn):
    for code in range(0, -8, -1):
        assert pn.pn_strerror(code) and pn.pn_strerror(code) != "unknown status"
    assert pn.pn_strerror(-99) == "unknown status"


def test_null_and_range_arguments_rejected(pn):
    lib = pn._lib
    out = ctypes.c_void_p()
    assert lib.pn_index_build(None, b"ACGT", None, 1, 4, 64, ctypes.byref(out)) == pn.PN_EINVAL
    assert lib.pn_map(None, None, None, 5, None, 0, None, None) == pn.PN_EINVAL
    assert lib.pn_ref_load(None, b"ACGT", 4, ctypes.byref(out)) == pn.PN_EINVAL
    assert lib.pn_ctx_create(0, None) == pn.PN_EINVAL
    assert lib.pn_ctx_set_timing(None, 1) == pn.PN_EINVAL
    # freeing NULL handles is a no-op
    lib.pn_ref_free(None)
    lib.pn_index_free(None)
    lib.pn_hits_free(None)
    lib.pn_ctx_destroy(None)


def test_no_device_gives_device_error(pn):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible")
    with pytest.raises(pn.PnError) as e:
        pn.pn_ctx_create(0)
    assert e.value.status == pn.PN_EDEVICE


def test_struct_layouts(pn):
    assert pn.HIT_DTYPE.itemsize == 12
    assert pn.CAND_DTYPE.itemsize == 16
    assert ctypes.sizeof(pn._IndexInfo) == 64


def test_new_entry_points_check_arguments(pn):
    lib = pn._lib
    hp, n = ctypes.c_void_p(), ctypes.c_uint64()
    assert lib.pn_map_batched(None, None, None, None, 0, None, 0, None, ctypes.byref(hp),
                              ctypes.byref(n)) == pn.PN_EINVAL
    assert lib.pn_poll(None, 1, ctypes.byref(hp), ctypes.byref(n), None) == pn.PN_EINVAL
    out = ctypes.c_void_p()
    assert lib.pn_server_create(None, None, None, ctypes.byref(out)) == pn.PN_EINVAL
    assert pn.PN_PENDING == 1
    assert lib.pn_ref_mask(None, 12, 5) == pn.PN_EINVAL
    assert lib.pn_index_sample_s(None) == pn.PN_EINVAL
    assert lib.pn_align(None, None, None, None, 0, None, None, None, 0, None) == pn.PN_EINVAL
