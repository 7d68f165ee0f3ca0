"""The C-ABI library loads and exports every entry point include/tpsolve.h
declares (no GPU needed); argument errors surface as status codes."""
import ctypes as C
import os
import re

import pytest

from paper_1902_00095_amd import synth, tpsolve

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tpsolve.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_expected_calls():
    names = declared_functions()
    for n in ("assemble_tpfa", "amg_setup", "precond_apply", "fgmres_solve"):
        assert n in names
    assert set(names) == set(tpsolve.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = tpsolve.load()
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_argument_errors_before_any_device_call():
    with pytest.raises(tpsolve.TpError) as e:
        tpsolve.jacobian_sizes(synth.Grid(0, 4, 4, 1, 1, 1))
    assert e.value.code == tpsolve.TP_ERR_ARG
    assert tpsolve.jacobian_sizes(synth.Grid(64, 64, 32, 1, 1, 1)) == (131072, 901120)
    lib = tpsolve.load()
    # amg_setup rejects a null output handle
    assert lib.amg_setup(C.c_int32(4), None, None, None, None, None, None) == tpsolve.TP_ERR_ARG
