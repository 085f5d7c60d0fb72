"""The C-ABI library loads and exports every function include/cfdmi.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os

import pytest

from paper_2504_03697_amd import _lib


def test_library_built():
    assert os.path.exists(_lib.LIB_PATH), "run python -m paper_2504_03697_amd.build"


def test_every_declared_symbol_is_exported():
    lib = _lib.load()
    names = _lib.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header_sizes():
    # cfd_grid: 3 int32 + pad + double; solve opts/info are 8-byte aligned
    assert ctypes.sizeof(_lib.CfdGrid) == 24
    assert ctypes.sizeof(_lib.CfdSolveOpts) == 64
    assert ctypes.sizeof(_lib.CfdSolveInfo) == 72


def test_param_count_is_host_only():
    lib = _lib.load()
    # 27 * (1*16 + 16*16 + 16*16 + 16*1)
    assert lib.cfd_net_param_count(16, 4) == 14688
    assert lib.cfd_net_param_count(3, 4) == 27 * (3 + 9 + 9 + 3)


def test_no_oracle_in_product_tree():
    root = os.path.dirname(_lib.HERE)
    pkg = _lib.HERE
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "cfd_oracle" not in text, f
    assert os.path.isdir(os.path.join(root, "oracle"))


def test_host_side_argument_checks():
    """Arguments the library rejects on the host, before any device call
    (this runs without a GPU): null pointers, empty grids, a non-positive
    cell size, an out-of-range pin, and a grid whose CSR would overflow the
    32-bit indices (N = 700: 7*700^3 > 2^31)."""
    lib = _lib.load()
    out = ctypes.c_void_p()
    g = _lib.CfdGrid(4, 4, 4, 0.25)
    assert lib.cfd_assemble(None, 0, None, ctypes.byref(out)) == _lib.CFD_EINVAL
    assert lib.cfd_assemble(ctypes.byref(g), 0, None, None) == _lib.CFD_EINVAL
    for bad in (_lib.CfdGrid(0, 4, 4, 0.25), _lib.CfdGrid(4, 4, -1, 0.25), _lib.CfdGrid(4, 4, 4, 0.0)):
        assert lib.cfd_assemble(ctypes.byref(bad), 0, None, ctypes.byref(out)) == _lib.CFD_EINVAL
    assert lib.cfd_assemble(ctypes.byref(g), 64, None, ctypes.byref(out)) == _lib.CFD_EINVAL
    big = _lib.CfdGrid(700, 700, 700, 1.0 / 700)
    assert lib.cfd_assemble(ctypes.byref(big), 0, None, ctypes.byref(out)) == _lib.CFD_EINVAL
    assert b"32-bit" in lib.cfd_last_error()
    assert not out.value
    info = _lib.CfdSolveInfo()
    assert lib.cfd_solve(None, None, None, 1e-10, None, None, ctypes.byref(info), None) == _lib.CFD_EINVAL
    assert lib.cfd_spmv(None, 0, None, None, None) == _lib.CFD_EINVAL
    assert lib.cfd_spmv_sym(None, 0, None, None, None) == _lib.CFD_EINVAL
