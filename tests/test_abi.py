"""CPU checks of the C ABI boundary: the library loads and exports every
function that include/*.h declares (no compute calls: there is no GPU here)."""
import ctypes
import glob
import os
import re

import pytest

import paper_1904_12759_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(mc_\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_core_entry_points():
    names = _declared_functions()
    for core in ("mc_expmv_create", "mc_expmv_entries", "mc_expmv_full", "mc_expmv_destroy",
                 "mc_expmv_set_proposal", "mc_expmv_sync", "mc_expmv_stats"):
        assert core in names


@pytest.mark.parametrize("name", _declared_functions())
def test_library_exports_declared_symbol(name):
    lib = pkg.load()
    assert hasattr(lib, name), name


def test_binding_covers_every_declared_function():
    assert set(_declared_functions()) <= set(pkg._SIGS)


def test_status_strings_and_default_opts():
    lib = pkg.load()
    for code in range(10):
        assert lib.mc_expmv_status_string(code)
    o = pkg.default_opts()
    assert o.struct_size == ctypes.sizeof(pkg.mc_expmv_opts)
    assert o.mode == pkg.EXACT and o.walkers_per_block == 64 and o.dt == 0.03125
    assert o.task_walkers == 0 and o.slot_rows == 0
    b = pkg.mc_batch_opts()
    lib.mc_batch_default_opts(ctypes.byref(b))
    assert b.struct_size == ctypes.sizeof(pkg.mc_batch_opts) and b.slot_rows == 0


def test_create_rejects_bad_host_arguments_without_gpu():
    """Argument checks happen before any device call."""
    lib = pkg.load()
    h = ctypes.c_void_p()
    # null output handle, negative sizes, null rowptr, bad t, bad options
    assert lib.mc_expmv_create(None, 1, 0, None, None, None, 1.0, 1, None) == 1
    assert lib.mc_expmv_create(ctypes.byref(h), -1, 0, None, None, None, 1.0, 1, None) == 1
    assert lib.mc_expmv_create(ctypes.byref(h), 4, 0, None, None, None, 1.0, 1, None) == 1
    dummy = ctypes.c_void_p(16)
    assert lib.mc_expmv_create(ctypes.byref(h), 4, 0, dummy, None, None, -1.0, 1, None) == 1
    assert lib.mc_expmv_create(ctypes.byref(h), 4, 0, dummy, None, None, float("nan"), 1,
                               None) == 1
    o = pkg.default_opts(mode=7)
    assert lib.mc_expmv_create(ctypes.byref(h), 4, 0, dummy, None, None, 1.0, 1,
                               ctypes.byref(o)) == 1
    o = pkg.default_opts(walkers_per_block=100)
    assert lib.mc_expmv_create(ctypes.byref(h), 4, 0, dummy, None, None, 1.0, 1,
                               ctypes.byref(o)) == 1
    o = pkg.default_opts(mode=pkg.STRANG, dt=0.0)
    assert lib.mc_expmv_create(ctypes.byref(h), 4, 0, dummy, None, None, 1.0, 1,
                               ctypes.byref(o)) == 1
    assert not h.value


def test_null_handle_calls_are_rejected():
    lib = pkg.load()
    assert lib.mc_expmv_entries(None, None, None, 0, 1, None, None) == 1
    assert lib.mc_expmv_full(None, None, 1, None, None) == 1
    assert lib.mc_expmv_sync(None) == 1
    lib.mc_expmv_destroy(None)
    assert lib.mc_expmv_entries_multi(None, None, None, 1, None, None, None) == 1
    assert lib.mc_expmv_entries_to_target(None, None, None, 1, 100, 1e-3, 1.2, 2, 1000,
                                          None, None, None) == 1
    assert lib.mc_expmv_get_stencil(None, None, None, None, None) == 1
