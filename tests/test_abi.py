"""The C ABI library loads on a machine without a GPU and exports every
function include/mtp.h declares (no compute call is made here)."""
import ctypes

from paper_2007_08555_amd import _lib


def test_header_declares_the_entry_points():
    names = _lib.header_functions()
    for n in ("mtp_load", "mtp_eval", "mtp_grade", "mtp_grade_from_b", "mtp_set_active_set",
              "mtp_free", "mtp_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    missing = [n for n in _lib.header_functions() if not hasattr(L, n)]
    assert not missing, missing
    # every declared function has a ctypes signature in the binding
    assert set(_lib.header_functions()) <= set(_lib._SIGNATURES)


def test_last_error_is_empty_string_initially():
    assert isinstance(_lib.lib().mtp_last_error(), bytes)


def test_compiled_bases_match_the_library_enumerator():
    # the variants table names levels 2..16; the package enumerator gives their sizes
    from paper_2007_08555_amd import basis, codegen
    for L in codegen.LEVELS:
        assert len(basis.functions(L)) > 0


def test_load_of_missing_file_fails_cleanly():
    h = ctypes.c_void_p()
    rc = _lib.lib().mtp_load(b"/nonexistent/potential.mtp", 0, ctypes.byref(h))
    assert rc != 0 and not h.value
