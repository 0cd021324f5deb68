"""The C-ABI library loads and exports every function include/ddeig.h declares,
and the binding marshals arguments without a GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ddeig.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ddeig_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for f in ("ddeig_assemble", "ddeig_cell_shift", "ddeig_apply_op", "ddeig_apply_precond",
              "ddeig_pcg_solve", "ddeig_inverse_iteration"):
        assert f in names


def test_library_exports_every_declared_symbol():
    import paper_2311_08757_amd as dd
    lib = dd.load_library()
    for f in _declared():
        assert hasattr(lib, f), f
    assert sorted(dd.EXPORTS) == _declared()


def test_status_strings_and_null_handling():
    import paper_2311_08757_amd as dd
    lib = dd.load_library()
    assert dd.status_string(0) == "ok"
    assert dd.status_string(-4).startswith("operator or preconditioner")
    # argument validation happens before any HIP call
    out = ctypes.c_void_p()
    st = lib.ddeig_assemble(None, 0.1, None, 1, None, None, ctypes.byref(out))
    assert st == -1
    assert b"NULL" in lib.ddeig_last_error()
    assert lib.ddeig_query(None, None, None, None) == -1


@pytest.mark.parametrize("kw,msg", [
    (dict(p=1, q=0), b"p >= 1"), (dict(h=0.3), b"1/h"), (dict(overlap=5), b"overlap"),
    (dict(L=0), b"L must"), (dict(ell=0.55), b"ell"), (dict(h=float("nan")), b"h must")])
def test_assemble_rejects_invalid_geometry(kw, msg):
    import paper_2311_08757_amd.ddeig as B
    lib = B.load_library()
    a = dict(p=1, q=1, L=4, ell=1.0, h=0.125, overlap=2)
    a.update(kw)
    geom = B.Geometry(a["p"], a["q"], a["L"], a["ell"])
    V, keep = B._potential({"kind": "const", "c": 0.0})
    out = ctypes.c_void_p()
    st = lib.ddeig_assemble(ctypes.byref(geom), a["h"], ctypes.byref(V), a["overlap"], None,
                            None, ctypes.byref(out))
    assert st == -1
    assert msg in lib.ddeig_last_error()
    assert not out.value
