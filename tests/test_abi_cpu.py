"""The C-ABI library loads on a CPU-only host and exports every function include/lbmib.h declares.

No compute call is made here; lbm_workspace_bytes is a pure host function.
"""
import ctypes
import os
import re

import pytest

from paper_2607_07432_amd import lbmib, workloads

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), 'include')
HEADERS = [os.path.join(INCLUDE, h) for h in ('lbmib.h', 'lbmib_nn.h')]


def declared_functions():
    names = set()
    for path in HEADERS:
        text = open(path).read()
        text = re.sub(r'/\*.*?\*/', '', text, flags=re.S)
        names |= set(re.findall(r'\b((?:lbm|ib|nn)_[a-z_0-9]+)\s*\(', text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ('lbm_init_grid', 'ib_set_markers', 'lbm_step', 'ib_wall_loads', 'lbm_fields'):
        assert must in names
    assert sorted(names) == sorted(lbmib.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = lbmib.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_workspace_bytes_is_pure_and_validates():
    lib = lbmib.load_library()
    case = workloads.config1()
    p = lbmib.params_from_case(case, precision=64)
    n64 = lib.lbm_workspace_bytes(ctypes.byref(p))
    p32 = lbmib.params_from_case(case, precision=32)
    n32 = lib.lbm_workspace_bytes(ctypes.byref(p32))
    N = 200 * 100
    # two states of (Q + 1 + D - 1) values plus the working area of (D + 2 + Q) values per node
    assert n64 >= N * 8 * (2 * 11 + 13) and n32 >= N * 4 * (2 * 11 + 13)
    assert n64 > n32
    bad = lbmib.params_from_case(case)
    bad.precision = 16
    assert lib.lbm_workspace_bytes(ctypes.byref(bad)) == 0
    bad = lbmib.params_from_case(case)
    bad.mu = -1.0
    assert lib.lbm_workspace_bytes(ctypes.byref(bad)) == 0
    assert lib.lbm_workspace_bytes(None) == 0
    # every active axis needs two nodes (x: five) and 2D grids have nz = 1
    for nx, ny, nz, dim, ok in ((5, 2, 1, 2, True), (4, 8, 1, 2, False), (6, 1, 1, 2, False), (6, 4, 2, 2, False),
                                (5, 2, 2, 3, True), (6, 5, 1, 3, False), (6, 1, 5, 3, False)):
        q = lbmib.params_from_case(case)
        q.nx, q.ny, q.nz, q.dim = nx, ny, nz, dim
        assert (lib.lbm_workspace_bytes(ctypes.byref(q)) > 0) == ok, (nx, ny, nz, dim)


def test_binding_fails_loudly_without_library(tmp_path):
    saved = lbmib._lib
    try:
        lbmib._lib = None
        with pytest.raises(RuntimeError):
            lbmib.load_library(str(tmp_path / 'missing.so'))
    finally:
        lbmib._lib = saved


def test_network_size_functions_are_pure():
    from oracle import unet
    lib = lbmib.load_library()
    assert lib.nn_unet_param_count() == unet.param_count()
    assert lib.nn_unet_workspace_bytes(4, 128, 256) > 0
    assert lib.nn_unet_workspace_bytes(4, 120, 256) == 0      # H % 16
    assert lib.nn_unet_workspace_bytes(4, 128, 200) == 0      # W % 128
    assert lib.nn_unet_workspace_bytes(0, 128, 256) == 0
