"""The C-ABI library loads and exports every symbol include/dvl.h declares
(no compute calls: these run without a GPU)."""
import ctypes as C
import os
import subprocess

import pytest


def test_library_exports_declared_symbols():
    from paper_2306_11612_amd import dvl
    L = dvl.lib()
    names = dvl.declared_symbols()
    assert len(names) >= 10
    missing = [s for s in names if not hasattr(L, s)]
    assert not missing, missing
    # and nm agrees that they are exported, unmangled, from libdvl.so
    out = subprocess.run(["nm", "-D", "--defined-only", dvl.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    assert set(names) <= exported


def test_host_only_entry_points():
    from paper_2306_11612_amd import dvl
    L = dvl.lib()
    # argument validation happens before any device work
    out = C.c_void_p()
    st = L.dvl_build_order(0, None, None, None, None, 1, 0, None, None, C.byref(out))
    assert st == dvl.E_INVALID and not out.value
    assert b"n_cells" in L.dvl_last_error()
    st = L.dvl_build_order(10, None, None, None, None, 0, 0, None, None, C.byref(out))
    assert st == dvl.E_INVALID
    st = L.dvl_build_order(10, None, None, None, None, 2, 9, None, None, C.byref(out))
    assert st == dvl.E_INVALID
    assert L.dvl_update_workspace_bytes(0, 4, 10) == 0
    w = L.dvl_update_workspace_bytes(500_000_000, 4, 1920)
    # per tile: prefixes, bin indices and cell-range records (48 B), whatever W and M
    assert 3e6 < w < 12e6
    assert L.dvl_update_workspace_bytes(500_000_000, 16, 1920) == w
    assert L.dvl_num_cells(None) == 0
    L.dvl_destroy(None)


def test_header_is_plain_c():
    """The header compiles as C99 with no C++ or HIP types in signatures."""
    from paper_2306_11612_amd import dvl
    src = '#include "dvl.h"\nint main(void){return 0;}\n'
    inc = os.path.dirname(dvl.HEADER)
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", inc, "-x", "c", "-", "-o", os.devnull],
                       input=src, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_product_path_has_no_oracle_dependency():
    """Neither the binding nor the HIP sources refer to the oracle."""
    import paper_2306_11612_amd
    root = os.path.dirname(paper_2306_11612_amd.__file__)
    for dirpath, _, files in os.walk(root):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "dvl_oracle" not in text and "ora_" not in text, f
