"""The C-ABI library loads and exports every function include/extrass.h declares
(no GPU needed: nothing is called that touches a device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2511_07539_amd", "libextrass.so")
HEADER = os.path.join(ROOT, "include", "extrass.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(extrass_[a-z0-9_]+)\s*\(", text)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libextrass.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libextrass.so not built")
def test_error_strings_and_null_arguments():
    lib = ctypes.CDLL(LIB)
    lib.extrass_error_string.restype = ctypes.c_char_p
    assert lib.extrass_error_string(0) == b"ok"
    assert lib.extrass_error_string(-2) == b"workspace too small"
    # host-side argument checks fail before any device work
    lib.extrass_transport.argtypes = [ctypes.c_void_p] * 7 + [ctypes.c_size_t, ctypes.c_void_p]
    assert lib.extrass_transport(None, None, None, None, None, None, None, 0, None) == -1
    lib.extrass_create.argtypes = [ctypes.c_void_p, ctypes.c_int]
    assert lib.extrass_create(None, 0) == -1


def test_binding_names_match_header():
    src = open(os.path.join(ROOT, "paper_2511_07539_amd", "__init__.py")).read()
    for name in declared_functions():
        assert name in src, name


def test_header_is_plain_c99():
    """include/extrass.h compiles as plain C (no HIP or C++ types in the
    signatures), with every warning enabled."""
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "use.c")
        with open(src, "w") as f:
            f.write('#include "extrass.h"\nint main(void) { return extrass_error_string(0) ? 0 : 1; }\n')
        r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-c", src,
                            "-I", os.path.dirname(HEADER), "-o", os.path.join(d, "use.o")],
                           capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
