"""CPU checks of the C-ABI library: it loads and exports every symbol include/sweep.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sweep.h")
LIB = os.path.join(ROOT, "paper_2207_12848_amd", "libsweep.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const char\*|sweep_status_t|size_t)\s+(sweep_\w+)\s*\(",
                                 text, flags=re.M)))


def test_header_declares_the_abi():
    names = _declared()
    for n in ("sweep_build_dag", "sweep_forward", "sweep_adjoint", "sweep_dag_info",
              "sweep_dag_export", "sweep_destroy_dag", "sweep_last_error", "sweep_saved_bytes"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsweep.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name
    from paper_2207_12848_amd import _binding
    assert set(_binding.EXPORTED) == set(_declared())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsweep.so not built")
def test_null_handles_are_rejected_without_a_gpu():
    from paper_2207_12848_amd import _binding as B
    lib = B.load()
    assert lib.sweep_forward(None, 1, None, None, None, None, None, None, None, 0, None) == -5
    assert b"DAG" in lib.sweep_last_error()
    assert lib.sweep_adjoint(None, 1, None, None, None, None, 0, None, None, None, None, None) == -5
    assert lib.sweep_dag_info(None, None) == -5
    assert lib.sweep_destroy_dag(None) == 0
    assert lib.sweep_saved_bytes(None, 1, None) == 0
    out = ctypes.c_void_p()
    assert lib.sweep_build_dag(None, 0, None, 0, None, None, ctypes.byref(out)) == -1
    assert lib.sweep_build_dag(None, 1, None, 0, None, None, None) == -1


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2207_12848_amd import _binding as B
    with pytest.raises(B.SweepLibraryError):
        B._lib_saved = B._lib
        try:
            B._lib = None
            B.load(str(tmp_path / "missing.so"))
        finally:
            B._lib = B._lib_saved
