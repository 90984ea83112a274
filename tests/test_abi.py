"""The C-ABI library loads and exports every function include/hrx.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2210_05547_amd", "libhrx.so")


def declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(hrx_\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared()
    for n in ("hrx_create", "hrx_destroy", "hrx_rhs_eval", "hrx_rk_stage", "hrx_thermo_eval",
              "hrx_chem_source", "hrx_get_counters", "hrx_strerror", "hrx_get_reference"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhrx.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n
    lib.hrx_strerror.restype = ctypes.c_char_p
    assert lib.hrx_strerror(0) == b"ok"
    # argument errors are returned without touching the device
    lib.hrx_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.hrx_create(None, None) == -1


def test_binding_refuses_missing_library(tmp_path):
    from paper_2210_05547_amd import hrx
    with pytest.raises(hrx.HrxError):
        hrx._lib_backup = hrx._lib
        hrx._lib = None
        try:
            hrx.load(str(tmp_path / "missing.so"))
        finally:
            hrx._lib = hrx._lib_backup


def test_binding_refuses_non_contiguous_arrays():
    import torch
    from paper_2210_05547_amd import hrx
    t = torch.zeros((4, 3), dtype=torch.float64).t()
    with pytest.raises(hrx.HrxError):
        hrx._ptr(t)
    assert hrx._ptr(None) is None


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhrx.so not built")
def test_stefan_maxwell_outside_its_scope_refused():
    """Stefan-Maxwell diffusion needs species (5-species air); other gases are refused
    before anything touches the device."""
    import dataclasses
    from paper_2210_05547_amd import fields, hrx
    for cfg in (dataclasses.replace(fields.get_config("c1"), diffusion=1),
                dataclasses.replace(fields.get_config("c1t"), diffusion=1)):
        x, y, z = fields.grid(cfg)
        with pytest.raises(hrx.HrxError):
            hrx.Context(cfg, x, y, z)
