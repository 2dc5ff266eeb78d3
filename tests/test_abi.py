"""CPU checks of the C-ABI library: it loads, exports every function declared in
include/cds.h, and rejects bad handles without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cds.h")
LIB = os.path.join(ROOT, "paper_1511_07174_amd", "libcds.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(?:cds_status_t|const char\s*\*)\s+(cds_\w+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1511_07174_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["cds_dgetrf", "cds_dgetrs", "cds_dpotrf", "cds_dpotrs", "cds_dgesv_mixed",
                     "cds_dposv_mixed_vbatched", "cds_create", "cds_set_workspace"]:
        assert required in names
    assert len(names) >= 30


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    import paper_1511_07174_amd.cds as b
    assert sorted(set(b.EXPORTED)) == declared_functions()


def test_null_handle_is_rejected_before_any_work(lib):
    lib.cds_dgetrf.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                               ctypes.c_void_p]
    lib.cds_dgetrf.restype = ctypes.c_int
    assert lib.cds_dgetrf(None, 4, None, 4, None, None) == 2     # CDS_NOT_INITIALIZED
    lib.cds_status_string.restype = ctypes.c_char_p
    lib.cds_status_string.argtypes = [ctypes.c_int]
    assert lib.cds_status_string(1) == b"CDS_INVALID_VALUE"
    assert lib.cds_status_string(99) == b"CDS_UNKNOWN_STATUS"


def test_create_without_gpu_reports_an_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    lib.cds_create.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    lib.cds_create.restype = ctypes.c_int
    assert lib.cds_create(ctypes.byref(h)) in (3, 4)   # CDS_HIP_ERROR or CDS_ARCH_MISMATCH
    assert not h.value


def test_product_path_refuses_to_run_without_the_library(tmp_path, monkeypatch):
    import paper_1511_07174_amd.cds as b
    monkeypatch.setattr(b, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(b, "_lib", None)
    with pytest.raises(b.CdsError):
        b.lib()


def test_colmajor_always_copies():
    """The functional API factors and solves on copies: colmajor must not alias its argument,
    also when the argument is already column-major."""
    import torch
    from paper_1511_07174_amd.cds import colmajor
    a = torch.arange(12.0, dtype=torch.float64).reshape(3, 4)
    f = colmajor(a)
    assert f.stride() == (1, 3) and torch.equal(f, a)
    g = colmajor(f)
    assert g.stride() == (1, 3) and torch.equal(g, f)
    assert g.data_ptr() != f.data_ptr()
    g[0, 0] = 99.0
    assert f[0, 0] == 0.0


def _tune_check(lib, path):
    lib.cds_tune_check.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)]
    lib.cds_tune_check.restype = ctypes.c_int
    n = ctypes.c_int64(-1)
    st = lib.cds_tune_check(os.fsencode(str(path)), ctypes.byref(n))
    return st, n.value


def test_tune_table_reader(lib, tmp_path):
    """cds_tune's file reader (host only): the shipped table parses; malformed files, unknown keys,
    values cds_tune_set would refuse and tables of another device are rejected."""
    import json
    shipped = os.path.join(ROOT, "paper_1511_07174_amd", "tune_gfx950.json")
    st, n = _tune_check(lib, shipped)
    assert st == 0 and n == len(json.load(open(shipped))["entries"])
    good = {"arch": "gfx950:sramecc+:xnack-", "note": "x \"quoted\" \\u00e9",
            "entries": [{"key": "getrf_nb", "dtype": "f64", "n_max": 8192, "value": 256},
                        {"key": "vbatch_tile", "dtype": "f32", "n_max": 1024, "value": 32, "extra": [1, {"a": None}]}],
            "timings": [{"ms": 1.5e-3, "ok": True}]}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(good))
    assert _tune_check(lib, p) == (0, 2)
    cases = [
        ({**good, "arch": "gfx942"}, 4),                                       # another device
        ({**good, "entries": [{"key": "getrf_nb", "dtype": "f64", "n_max": 8, "value": 1000}]}, 1),
        ({**good, "entries": [{"key": "vbatch_tile", "dtype": "f32", "n_max": 8, "value": 48}]}, 1),
        ({**good, "entries": [{"key": "nb", "dtype": "f64", "n_max": 8, "value": 128}]}, 1),
        ({**good, "entries": [{"key": "getrf_nb", "dtype": "f16", "n_max": 8, "value": 128}]}, 1),
        ({**good, "entries": [{"key": "getrf_nb", "dtype": "f64", "n_max": 8.5, "value": 128}]}, 1),
        ({**good, "entries": [{"key": "getrf_nb", "dtype": "f64", "value": 128}]}, 1),
        ({"arch": "gfx950"}, 1),                                               # no entries
    ]
    for table, status in cases:
        p.write_text(json.dumps(table))
        assert _tune_check(lib, p)[0] == status, table
    for text in ['{"entries": [', '[]', '{"entries": []} x', '{"entries": [{"key": "getrf_nb",}]}', '']:
        p.write_text(text)
        assert _tune_check(lib, p)[0] == 1, text
    p.write_text('{"entries": []}')
    assert _tune_check(lib, p) == (0, 0)
    assert _tune_check(lib, tmp_path / "missing.json")[0] == 1
