"""Host-side checks of the C-ABI library that need no GPU: the shared library
loads, exports every symbol the public header declares, and the binding's
parameter struct matches the header layout."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tbkrylov.h")
LIB = os.path.join(ROOT, "paper_0910_4497_amd", "libtbkrylov.so")


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(tb_[a-z_A-Z]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = declared_symbols()
    for must in ("tb_create", "tb_destroy", "tb_build_local_H", "tb_krylov_rho",
                 "tb_rho_layout", "tb_energy_forces", "tb_last_error"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_params_struct_layout():
    from paper_0910_4497_amd import inputs, tb
    p = tb.TBParams.from_dict(inputs.load_params())
    # int64 + 12 doubles + 4 + 7 + 4 + 5 doubles
    assert ctypes.sizeof(tb.TBParams) == 8 + 8 * (12 + 4 + 7 + 4 + 5)
    assert p.struct_size == ctypes.sizeof(tb.TBParams)
    assert p.rm == 2.6 and p.frep[4] == inputs.load_params()["frep"][4]


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_last_error_callable_without_device():
    from paper_0910_4497_amd import tb
    lib = tb.load_library()
    assert isinstance(lib.tb_last_error(), bytes)
    # a null context is rejected on the host, before any device call
    code = lib.tb_krylov_rho(None, 10, None, 0.1, float("nan"), 4.0, 0, None, None)
    assert code == -1
    assert b"null" in lib.tb_last_error()
    assert lib.tb_set_launch(None, 1) == -1
    assert lib.tb_autotune(None, 10, None, 0, None) == -1
    assert lib.tb_virial(None, None) == -1
    assert lib.tb_energy_backward(None, None, None) == -1
    assert lib.tb_energy_forces_static(None, None, None) == -1
    assert lib.tb_set_seeds(None, 1) == -1
    assert lib.tb_set_groups(None, 4) == -1
    assert lib.tb_set_shape(None, 1, 256, 4, 1, 1) == -1
    h = ctypes.c_void_p()
    for bad_hop in (0, 257):     # checked before any device call
        assert lib.tb_create_ex(ctypes.byref(h), 0, None, 10, 10, 10, bad_hop) == -1
        assert b"hop_max" in lib.tb_last_error()
