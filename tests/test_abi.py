"""CPU checks of the C ABI: the library loads and exports every symbol that
include/tls.h declares, and the struct layouts of the binding match the
header's field lists. No compute calls (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tls.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^TLS_API[^(]*?\b(tls_\w+)\(", txt, flags=re.M)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("tls_factor_precond", "tls_rqi_solve", "tls_pcg_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2305_19028_amd import tls
    if not os.path.exists(tls.LIB_PATH):
        pytest.skip("libtls.so not built")
    L = ctypes.CDLL(tls.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    # the binding wraps every declared symbol
    assert set(_declared()) <= set(tls._SIGS)


def _struct_fields(name):
    txt = open(HEADER).read()
    end = re.search(r"\}\s*" + name + r";", txt).start()
    start = txt.rfind("typedef struct {", 0, end) + len("typedef struct {")
    body = re.sub(r"/\*.*?\*/", "", txt[start:end], flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        parts = decl.replace("*", " ").split()
        for item in " ".join(parts[1:]).split(","):
            item = item.strip().split("[")[0]
            if item and item not in ("const", "int32_t", "double", "int64_t"):
                fields.append(item.split()[-1])
    return fields


@pytest.mark.parametrize("cname,pyname", [
    ("tls_matrix", "c_matrix"), ("tls_gate_report", "c_gate_report"),
    ("tls_rqi_opts", "c_rqi_opts"), ("tls_rqi_stats", "c_rqi_stats"),
])
def test_struct_field_order_matches_header(cname, pyname):
    from paper_2305_19028_amd import tls
    py = [f for f, _ in getattr(tls, pyname)._fields_]
    assert _struct_fields(cname) == py


def test_library_version_and_error_string():
    from paper_2305_19028_amd import tls
    if not os.path.exists(tls.LIB_PATH):
        pytest.skip("libtls.so not built")
    L = tls.lib()
    assert b"gfx950" in L.tls_version()
    assert isinstance(L.tls_last_error(), bytes)
    # a size query with an invalid matrix returns 0 (no device work)
    A = tls.c_matrix(0, 0, 3, 5, 3, 0, None, None, None)
    assert L.tls_factor_workspace_size(ctypes.byref(A), 0) == 0
