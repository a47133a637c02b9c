"""Host-side checks of the C interface that need no GPU: the library loads
and exports every function include/glm.h declares, and the binding names the
same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1310_1537_amd", "libglm_hip.so")


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:glm_status|const char\*|void)\s+(glm_\w+)\s*\(", src, re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("glm_create", "glm_destroy", "glm_dataset_register",
                     "glm_logpost_grad", "glm_logpost_grad_host", "glm_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_binding_covers_the_header():
    from paper_1310_1537_amd import glm
    assert sorted(glm.exported_symbols()) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_last_error_starts_empty():
    from paper_1310_1537_amd import glm
    assert glm.glm_last_error() == ""
