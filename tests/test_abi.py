"""The C-ABI library loads on the CPU and exports every function include/gmg.h declares.

No compute call is made here (there is no GPU); gmg_default_options and
gmg_status_string touch no device state.
"""
import ctypes
import os
import subprocess

import pytest

from paper_1604_07163_amd import gmg


def test_library_is_built_and_loads():
    assert os.path.exists(gmg.LIB_PATH), "run `python -m paper_1604_07163_amd.build`"
    gmg.lib()


def test_every_declared_symbol_is_exported():
    names = gmg.declared_functions()
    assert len(names) >= 15
    L = gmg.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", gmg.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    assert set(names) <= exported


def test_default_options_and_status_strings():
    L = gmg.lib()
    o = gmg.Options()
    L.gmg_default_options(ctypes.byref(o), 257)
    assert (o.n, o.levels, o.cheb_degree, o.cheb_lo, o.cheb_hi) == (257, 8, 2, 0.25, 2.0)
    assert o.switch_n == 0 and o.precision == gmg.FP64 and o.coarse_rule == gmg.COARSE_ARITHMETIC
    L.gmg_default_options(ctypes.byref(o), 33)
    assert o.levels == 5
    for code, name in gmg.STATUS.items():
        assert L.gmg_status_string(code).decode() == name
    # with no handle: the message of the last gmg_solve_static call on this device (none yet)
    assert L.gmg_last_error(None).decode() == ""


def test_create_rejects_null_arguments_without_touching_the_device():
    L = gmg.lib()
    o = gmg.Options()
    L.gmg_default_options(ctypes.byref(o), 17)
    h = ctypes.c_void_p()
    assert L.gmg_create(ctypes.byref(o), None, None, None, None, ctypes.byref(h)) == 1
    assert L.gmg_create(None, None, None, None, None, ctypes.byref(h)) == 1
    assert not h.value


def test_create_rejects_grids_beyond_the_32_bit_chunk_offsets():
    """The one-sweep kernels address a z-chunk through 32-bit buffer offsets;
    gmg_create refuses an n whose planes cannot fit that range (GMG_ERR_DIMS)
    before it reads the coefficient pointers or touches the device."""
    L = gmg.lib()
    o = gmg.Options()
    L.gmg_default_options(ctypes.byref(o), 5441)
    o.levels = 7              # 5440 = 64 * 85
    o.coarse_solver = 1       # inexact coarse CG: no limit on the coarsest level
    o.switch_n = 0
    dummy = ctypes.c_void_p(256)  # never dereferenced: the option check comes first
    h = ctypes.c_void_p()
    assert L.gmg_create(ctypes.byref(o), dummy, dummy, dummy, None, ctypes.byref(h)) == 2
    assert not h.value


def test_header_cites_no_missing_type():
    src = open(gmg.HEADER).read()
    for t in ("gmg_options", "gmg_info", "gmg_status", "gmg_handle"):
        assert t in src


def test_kernel_class_names_match_binding():
    L = gmg.lib()
    assert [L.gmg_kernel_class_name(i).decode() for i in range(len(gmg.KERNEL_CLASSES))] == gmg.KERNEL_CLASSES
    assert L.gmg_kernel_class_name(len(gmg.KERNEL_CLASSES)).decode() == "unknown"
    assert L.gmg_calibration_copy(None, None, 16, 1, None) == 1
