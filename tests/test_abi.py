"""The C-ABI library loads on the CPU and exports every declared function.

No compute call is made here (there is no GPU in the CPU test run); the
checks are: every function declared in include/*.h is exported, the ctypes
signatures of the binding cover exactly those functions, and the calls that
validate arguments before touching the device return the documented error
codes."""
import ctypes
import glob
import os
import re

import pytest

from paper_2407_07411_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for path in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(?:dmrg_status|void|const char\*|int64_t|double)\s+(dmrg_\w+)\s*\(", text):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2407_07411_amd.build import build
        build()
    return _lib.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names == set(_lib.SIGNATURES), names ^ set(_lib.SIGNATURES)


def test_argument_errors_need_no_device(lib):
    out = ctypes.c_void_p()
    assert lib.dmrg_ctx_create(0, None, None) == -1
    assert b"NULL" in lib.dmrg_last_error()
    assert lib.dmrg_basis_create(None, 1, None, None, ctypes.byref(out)) == -1
    assert lib.dmrg_heff_apply(None, None, None) == -1
    assert lib.dmrg_heff_diag(None, None) == -1
    assert lib.dmrg_heff_flops(None, None, None) == -1
    assert lib.dmrg_heff_size(None) == -1
    assert lib.dmrg_davidson(None, None, None, None) == -1
    assert lib.dmrg_davidson_step(None, None) == -1
    assert lib.dmrg_heff_apply_adjoint(None, None, None, None, None, None) == -1


def test_build_info(lib):
    assert b"gfx950" in lib.dmrg_build_info()
