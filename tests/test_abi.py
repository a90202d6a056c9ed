"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function that include/adscl.h declares,
and reject invalid configurations in adscl_create before it touches a GPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1706_07413_amd import adscl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "adscl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(adscl_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(adscl.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = adscl.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


@pytest.mark.parametrize("n_grid", [[16], [15], [65539], [16386], [513, 514], [1]])
def test_create_rejects_bad_grid_sizes_before_touching_the_gpu(n_grid):
    L = adscl.lib()
    N = np.asarray(n_grid, np.int32)
    cfg = adscl.Config(len(N), N.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 0.25, 0.5, 0.01, 0, 0, 0)
    h = ctypes.c_void_p()
    rc = L.adscl_create(ctypes.byref(cfg), None, ctypes.byref(h))
    assert rc == adscl.EINVAL
    assert h.value is None
    assert b"N=" in L.adscl_last_error(None)


@pytest.mark.parametrize("field,value", [("cfl", 0.0), ("cfl", 2.0), ("a_collapse", -0.1), ("gauge", 7),
                                         ("n_modes", 200), ("flags", 8), ("n_inst", 0)])
def test_create_rejects_bad_parameters(field, value):
    L = adscl.lib()
    N = np.asarray([65], np.int32)
    cfg = adscl.Config(1, N.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 0.25, 0.5, 0.01, 0, 0, 0)
    setattr(cfg, field, value)
    h = ctypes.c_void_p()
    assert L.adscl_create(ctypes.byref(cfg), None, ctypes.byref(h)) == adscl.EINVAL
    assert L.adscl_create(None, None, ctypes.byref(h)) == adscl.EINVAL


@pytest.mark.parametrize("rk,K,flags,N,code", [(5, 0, 0, 65, -1), (1, 0, 0, 65, -1), (3, -1, 0, 65, -1),
                                               (4, 8, 1, 65, -1)])
def test_create_rejects_bad_scheme_options_before_touching_the_gpu(rk, K, flags, N, code):
    L = adscl.lib()
    Ns = np.asarray([N], np.int32)
    cfg = adscl.Config(1, Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 0.25, 0.5, 0.01, 0, 0, flags, rk, K)
    h = ctypes.c_void_p()
    assert L.adscl_create(ctypes.byref(cfg), None, ctypes.byref(h)) == code
    assert h.value is None


def test_null_context_calls_fail_cleanly():
    L = adscl.lib()
    assert L.adscl_sync(None) == adscl.EINVAL
    assert L.adscl_step(None, 1, 1.0, 0, 0, None, 0) == adscl.EINVAL
    assert L.adscl_status(None, None, None, None, None, None) == adscl.EINVAL
    assert L.adscl_spectrum(None, 4, None, None, None, 0) == adscl.EINVAL
    assert L.adscl_spectrum_snaps(None, 4, 1, None, None, None, None, 0) == adscl.EINVAL
    assert L.adscl_adjoint(None, None, None, 4, 4, 1.0, 8, None, None, None, 0) == adscl.EINVAL
    assert L.adscl_descend(None, None, None, 4, 4, 1.0, 8, 2, 0.05, 0, None, None, 0) == adscl.EINVAL
    assert L.adscl_constraints(None, None, 0) == adscl.EINVAL
    assert L.adscl_get_state(None, None, None, None, None, None, 0) == adscl.EINVAL
    assert L.adscl_kernel_stats(None, 0, None, None, None, None, None, None) == adscl.EINVAL
    assert L.adscl_last_error(None) is not None


def test_create_accepts_large_grids_before_touching_the_gpu():
    """N above 4097 (up to 65537) passes validation; with no GPU here the call
    then fails on the device, not on the arguments."""
    L = adscl.lib()
    N = np.asarray([16385, 65537], np.int32)
    cfg = adscl.Config(len(N), N.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 0.25, 0.5, 0.01, 0, 0, 0)
    h = ctypes.c_void_p()
    rc = L.adscl_create(ctypes.byref(cfg), None, ctypes.byref(h))
    assert rc != adscl.EINVAL, L.adscl_last_error(None)
    if rc == adscl.OK:
        L.adscl_destroy(h)


@pytest.mark.parametrize("n_grid,n,steps", [([1025], 0, 8), ([1025], 1, 0), ([1024], 1, 8), ([4099], 1, 8),
                                            ([15], 1, 8), ([513, 16385], 2, 8)])
def test_autotune_rejects_bad_arguments_before_touching_the_gpu(n_grid, n, steps):
    L = adscl.lib()
    N = np.asarray(n_grid, np.int32)
    assert L.adscl_autotune(N.ctypes.data, n, steps, 0, None, None, None) == adscl.EINVAL
    assert L.adscl_autotune(None, 1, 8, 0, None, None, None) == adscl.EINVAL
    L.adscl_autotune_clear()
