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


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes struct of the binding has the C struct's size and field offsets
    (a small C program compiled with gcc against include/sweep.h prints them)."""
    import subprocess
    from paper_2207_12848_amd import _binding as B
    structs = [B.sweep_mesh_t, B.sweep_build_opts_t, B.sweep_dag_info_t, B.sweep_fwd_opts_t,
               B.sweep_ion_params_t]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "sweep.h"', "int main(void) {"]
    for st in structs:
        n = st.__name__
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (n, n))
        for f in st._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (n, f[0], n, f[0]))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().split("\n"):
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for st in structs:
        n = st.__name__
        assert got[(n, "size")] == ctypes.sizeof(st), n
        for f in st._fields_:
            assert got[(n, f[0])] == getattr(st, f[0]).offset, (n, f[0])


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; --gpus 2 exits with a message before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
