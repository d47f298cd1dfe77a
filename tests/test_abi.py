"""Host-side checks of the C ABI: the library loads, exports every declared symbol, and
rejects invalid configurations before touching the GPU."""
import ctypes
import os
import re

import pytest

import stmg_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "stmg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(stmg_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2408_04372_amd import _lib
    lib = _lib.load()
    names = _declared()
    assert "stmg_create" in names and "stmg_solve" in names
    for n in names:
        assert getattr(lib, n) is not None, n
    assert set(_lib.exported_symbols()) <= set(names)


def test_struct_layout_matches_header():
    # compile a tiny host program against the header and compare sizes/offsets with ctypes
    import subprocess
    import tempfile
    from paper_2408_04372_amd._lib import CConfig, Info, SolveInfo
    src = r'''
#include <stddef.h>
#include <stdio.h>
#include "stmg.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(stmg_config), sizeof(stmg_info), sizeof(stmg_solve_info),
         offsetof(stmg_config, rtol), offsetof(stmg_info, omega), offsetof(stmg_solve_info, cnn_used));
  return 0;
}'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(v) for v in subprocess.check_output([exe]).split()]
    want = [ctypes.sizeof(CConfig), ctypes.sizeof(Info), ctypes.sizeof(SolveInfo),
            CConfig.rtol.offset, Info.omega.offset, SolveInfo.cnn_used.offset]
    assert got == want


@pytest.mark.parametrize("field,value", [("dim", 4), ("p", 0), ("p", 7), ("k", -1), ("tau", 0.0),
                                         ("n_time_cells", 0), ("restart", 0), ("rtol", 0.0),
                                         ("precision", 5), ("n_smooth", 0), ("time_mg", 2),
                                         ("asm_variant", 3), ("asm_variant", -1), ("gram_schmidt", 3), ("kernel_path", 3),
                                         ("kernel_path", -1)])
def test_invalid_config_rejected_on_host(field, value):
    from paper_2408_04372_amd import _lib
    lib = _lib.load()
    cfg = _lib.c_config(si.paper_config(1), **{field: value})
    h = ctypes.c_void_p()
    code = lib.stmg_create(ctypes.byref(cfg), None, None, None, ctypes.byref(h))
    assert code in (1, 6)
    assert h.value is None
    assert len(lib.stmg_last_error()) > 0


def test_abi_version_and_null_arguments():
    from paper_2408_04372_amd import _lib
    lib = _lib.load()
    cfg = _lib.c_config(si.paper_config(1))
    cfg.abi_version = 99
    h = ctypes.c_void_p()
    assert lib.stmg_create(ctypes.byref(cfg), None, None, None, ctypes.byref(h)) == 1
    assert lib.stmg_create(None, None, None, None, ctypes.byref(h)) == 1
    assert lib.stmg_vmult(None, 0, 0, None, None) == 1
    assert lib.stmg_vmult_noalloc(None, 0, 0, None, None) == 1
    assert lib.stmg_solve(None, None, None, None) == 1
    lib.stmg_destroy(None)


def test_inverted_cell_rejected():
    import numpy as np
    from paper_2408_04372_amd import _lib
    lib = _lib.load()
    c = si.Config(dim=2, p=1, n_cells=(2, 2, 1), perturb=0.1, seed=1)
    v, _ = si.draw_problem(c)
    v = v.copy()
    v[1, 1] = [1.2, 0.5]      # pull the centre vertex across the mesh
    cfg = _lib.c_config(c)
    h = ctypes.c_void_p()
    vp = v.ctypes.data_as(ctypes.c_void_p)
    assert lib.stmg_create(ctypes.byref(cfg), vp, None, None, ctypes.byref(h)) == 1
    assert b"inverted" in lib.stmg_last_error()
