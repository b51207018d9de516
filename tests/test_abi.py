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
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:\w+\s+)*\w+\**\s+\**(\w+)\s*\(", text, flags=re.M)))


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


def test_struct_layouts_match_header(lib, tmp_path):
    # compile the header with the host C compiler and compare every field offset
    import ctypes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"mnf_fuse_params": lib.FuseParamsC, "ptycho_params": lib.PtychoParamsC,
               "ptycho_scan": lib.PtychoScanC}
    src = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        src.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            src.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    src += ["return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run([cc, str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


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


def test_error_codes_match_header(lib):
    text = open(HEADER).read()
    codes = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(MNF_\w+)\s+(-?\d+)", text)}
    for name in ["MNF_OK", "MNF_EINVAL", "MNF_EUNSUPPORTED", "MNF_EHIP", "MNF_ENOMEM", "MNF_ENONFINITE",
                 "MNF_EDIVERGED"]:
        assert getattr(lib, name) == codes[name], name
    assert set(lib.ERROR_NAMES.values()) == {n for n in codes if n != "MNF_OK"}


def test_host_paths_reject_a_null_context(lib):
    # argument checks run before any device call
    L = lib.load()
    assert L.mnf_status(None, None) == lib.MNF_EINVAL
    assert L.ptycho_grad(None, None, 1, 1, None, 1, None, 16, None, 1, 0, 1e-6, 1, None, None, None, None,
                         None) == lib.MNF_EINVAL
    assert L.ptycho_descend(None, None, 1, 1, None, 1, None, 16, None, 1, 0, 1e-6, 1, 1, 0.0, 0.0, 1, None, None,
                            None) == lib.MNF_EINVAL
