"""The C ABI library loads and exports every entry point include/hawkes.h declares
(no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:hawkes_status|int64_t|int|void|double)\s+(\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_symbols()
    for required in ("hawkes_plan_create", "hawkes_eval", "hawkes_loglik", "hawkes_grad", "hawkes_hessdiag",
                     "hawkes_plan_status"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2103_03348_amd", "libhawkes.so"))
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_match_header():
    from paper_2103_03348_amd import _lib
    assert set(_lib.SIGNATURES) == set(declared_symbols())
