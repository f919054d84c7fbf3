"""C-ABI library checks that need no GPU: it loads, exports every symbol that
include/corrx.h declares, and rejects bad arguments / a missing device cleanly.
No compute call is made here."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "corrx.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(corr_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def cx():
    from paper_1501_05992_amd import corrx

    if not os.path.exists(corrx.LIB_PATH):
        from paper_1501_05992_amd import build

        build.build()
    return corrx


def test_header_declares_the_binding_symbols(cx):
    assert _declared() == sorted(cx.SYMBOLS)


def test_library_exports_every_declared_symbol(cx):
    L = cx.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert L.corr_abi_version() == 1


def test_strerror(cx):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert cx.corr_strerror(code)
    assert cx.corr_strerror(-99) == "unknown status"


def test_create_rejects_bad_arguments_before_touching_the_device(cx):
    L = cx.lib()
    h = ctypes.c_void_p(123)
    for args in [(0, 1, 1, 0), (5000, 1, 1, 0), (4, 0, 1, 0), (4, 1, 0, 0), (4, 1, 1, 7),
                 (4096, 65536, 65536, 0)]:
        assert L.corr_create(*args, ctypes.byref(h)) == cx.CORRX_EINVAL
        assert h.value is None
    assert L.corr_create(4, 1, 1, 0, None) == cx.CORRX_EINVAL


def test_null_handle_calls(cx):
    L = cx.lib()
    assert L.corr_xmac(None, None, None, None) == cx.CORRX_EINVAL
    assert L.corr_zero(None, None, None) == cx.CORRX_EINVAL
    assert L.corr_dump(None, None, 0, 0, None, None) == cx.CORRX_EINVAL
    assert L.corr_set_engine(None, 0) == cx.CORRX_EINVAL
    assert L.corr_acc_bytes(None) == 0
    assert L.corr_destroy(None) == cx.CORRX_OK
    assert L.corr_batch_xmac(None, None, None, None) in (cx.CORRX_EINVAL, cx.CORRX_EUNSUPPORTED)
    assert L.corr_batch_samples(None, 0) == cx.CORRX_EINVAL


def test_noalloc_rejects_bad_arguments_before_touching_the_device(cx):
    L = cx.lib()
    p = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation
    assert L.corr_xmac_noalloc(None, p, 4, 1, 1, 0, 0, None) == cx.CORRX_EINVAL
    assert L.corr_xmac_noalloc(p, None, 4, 1, 1, 0, 0, None) == cx.CORRX_EINVAL
    assert L.corr_xmac_noalloc(p, p, 4, 1, 1, 0, 2, None) == cx.CORRX_EINVAL
    for args in [(0, 1, 1, 0), (5000, 1, 1, 0), (4, 0, 1, 0), (4, 1, 0, 0), (4, 1, 1, 7)]:
        assert L.corr_xmac_noalloc(p, p, *args, 0, None) == cx.CORRX_EINVAL
    assert L.corr_xmac_noalloc(p, p, 4, 1, 21913099, 0, 1, None) == cx.CORRX_EOVERFLOW


def test_no_gpu_means_edevice(cx):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert cx.lib().corr_create(256, 8, 2000, 0, ctypes.byref(h)) == cx.CORRX_EDEVICE
    with pytest.raises(cx.CorrxError):
        cx.corr_create(256, 8, 2000)


def test_header_is_plain_c_and_links(cx, tmp_path):
    # a C99 caller compiles against the header and links the library (not run)
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    src = tmp_path / "caller.c"
    src.write_text(
        '#include "corrx.h"\n'
        "int main(void) {\n"
        "  corrx_t h = 0;\n"
        "  void *in = 0, *acc = 0, *vis = 0, *stream = 0;\n"
        "  if (corr_create(256, 3072, 10000, CORRX_LAYOUT_TFI, &h) != CORRX_OK) return 1;\n"
        "  corr_zero(h, acc, stream);\n"
        "  corr_xmac(h, in, acc, stream);\n"
        "  corr_dump(h, acc, CORRX_TRI_STATION_POL, CORRX_F32, vis, stream);\n"
        "  return corr_destroy(h) == CORRX_OK && corr_strerror(0) != 0 ? 0 : 1;\n"
        "}\n")
    lib_dir = os.path.dirname(cx.LIB_PATH)
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                        "-o", str(tmp_path / "caller"), "-L", lib_dir, "-l:libcorrx.so",
                        "-Wl,--unresolved-symbols=ignore-in-shared-libs"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
