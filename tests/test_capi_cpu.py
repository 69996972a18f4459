"""CPU-only checks of the C-ABI library: it loads, exports every symbol the
public header declares, and fails cleanly where it needs a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2312_06484_amd import airpf
    if not os.path.exists(airpf.LIBPATH):
        pytest.skip("libairpf.so not built (run __graft_entry__.build())")
    return airpf


def test_header_symbols_exported():
    airpf = _lib()
    header = open(os.path.join(ROOT, "include", "airpf.h")).read()
    declared = set(re.findall(r"^\s*(?:airpf_status|const char\s*\*)\s*(airpf_\w+)\s*\(", header, re.M))
    assert declared == set(airpf.EXPORTS)
    raw = ctypes.CDLL(airpf.LIBPATH)
    for name in declared:
        assert hasattr(raw, name), name


def test_status_strings():
    airpf = _lib()
    assert airpf.status_str(airpf.OK) == "ok"
    assert "domain" in airpf.status_str(airpf.E_DOMAIN)
    assert airpf.status_str(99) == "unknown status"


def test_null_arguments_rejected_without_device():
    airpf = _lib()
    L = airpf.lib()
    # a null context is rejected before any device call
    st = L.airpf_run(None, None, None, 0, None, 0, 0, 0, 0, None, None, None)
    assert st == airpf.E_INVALID_ARG
    assert L.airpf_ctx_destroy(None) == airpf.E_INVALID_ARG
    assert L.airpf_ctx_create(0, None, None) == airpf.E_INVALID_ARG


def test_product_path_does_not_import_oracle():
    # the binding and kernels never reach the checker
    for f in os.listdir(os.path.join(ROOT, "paper_2312_06484_amd")):
        if f.endswith(".py"):
            src = open(os.path.join(ROOT, "paper_2312_06484_amd", f)).read()
            assert "oracle" not in re.sub(r"#.*|\"\"\"[\s\S]*?\"\"\"", "", src), f
