"""CPU checks of the C ABI: the library loads and exports every function
declared in include/mnfpty.h, and the Python binding declares the same set."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mnfpty.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2608_01746_amd import lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2608_01746_amd import build
        build.build()
    return L


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ["mnf_create", "mnf_destroy", "mnf_last_error", "fuse_exposures", "ptycho_forward",
              "ptycho_iterate", "ptycho_grad"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    L = lib.load()
    for n in _declared():
        assert hasattr(L, n), n


def test_binding_signatures_cover_the_header(lib):
    assert sorted(lib.SIGNATURES) == _declared()


def test_struct_layouts_match_header(lib):
    import ctypes
    assert ctypes.sizeof(lib.FuseParamsC) == 4 * 5 + 4 * 16 + 4
    assert ctypes.sizeof(lib.PtychoParamsC) == 7 * 4


def test_supported_sizes_without_gpu(lib):
    import ctypes
    buf = (ctypes.c_int32 * 16)()
    n = lib.load().mnf_supported_sizes(buf, 16)
    assert list(buf)[:n] == [16, 32, 64, 128, 192, 256, 384, 512]


def test_create_without_device_fails_cleanly(lib):
    import ctypes
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    c = ctypes.c_void_p()
    assert lib.load().mnf_create(ctypes.byref(c), 0) == lib.MNF_EINVAL
    assert not c.value
