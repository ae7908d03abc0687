"""CPU-side checks of the boundary: the library loads, exports every function that
include/tagi.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tagi.h")
LIB = os.path.join(ROOT, "paper_2003_01833_amd", "libtagi.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tagi_[a-z_]+)\s*\(", src)))


def _lib():
    if not os.path.exists(LIB):
        from paper_2003_01833_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("tagi_tree_build", "tagi_upward", "tagi_convolve", "tagi_direct"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in _declared():
        assert hasattr(lib, name), name


def test_validation_rejects_before_any_device_work():
    lib = _lib()
    lib.tagi_last_error.restype = ctypes.c_char_p
    vp = ctypes.c_void_p
    out = vp()
    bogus = vp(0x1000)  # never dereferenced: every call below fails validation first
    lib.tagi_tree_build.argtypes = [vp, vp, vp, ctypes.c_int64, vp, ctypes.c_int, vp,
                                    ctypes.POINTER(vp)]
    assert lib.tagi_tree_build(None, bogus, bogus, 10, None, 4, None, ctypes.byref(out)) == -1
    assert lib.tagi_tree_build(bogus, bogus, bogus, 0, None, 4, None, ctypes.byref(out)) == -1
    assert lib.tagi_tree_build(bogus, bogus, bogus, 10, None, 0, None, ctypes.byref(out)) == -1
    assert b"leaf_size" in lib.tagi_last_error()
    lib.tagi_upward.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
    assert lib.tagi_upward(None, bogus, bogus, 1, 4, None) == -1
    lib.tagi_convolve.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_int, vp, vp]
    assert lib.tagi_convolve(None, None, 0, None, 1.0, 0.5, 4, 0, bogus, None) == -1
    lib.tagi_direct.argtypes = [vp] * 5 + [ctypes.c_int64] + [vp] * 4 + [ctypes.c_int64, ctypes.c_int,
                                                                        ctypes.c_double, ctypes.c_double,
                                                                        vp, vp]
    # Yukawa with kappa <= 0, and a missing tf for a subtracted kernel
    assert lib.tagi_direct(bogus, bogus, bogus, bogus, bogus, 4, bogus, bogus, bogus, bogus, 4,
                           0, 0.0, 1.0, bogus, None) == -1
    assert lib.tagi_direct(bogus, bogus, bogus, bogus, bogus, 4, bogus, bogus, bogus, None, 4,
                           1, 1.0, 1.0, bogus, None) == -1
    assert lib.tagi_direct(bogus, bogus, bogus, bogus, bogus, 4, bogus, bogus, bogus, bogus, 4,
                           7, 1.0, 1.0, bogus, None) == -1
    lib.tagi_tree_set_orbital_block.argtypes = [vp, ctypes.c_int]
    assert lib.tagi_tree_set_orbital_block(None, 4) == -1
    i32, dbl = ctypes.c_int, ctypes.c_double
    lib.tagi_autotune.argtypes = [vp, vp, vp, vp, ctypes.c_int64, vp, vp, i32, i32, vp, dbl, dbl,
                                  i32, i32, vp, i32, vp, i32, vp, i32, vp, i32, i32, vp, vp, vp]
    leafs = (ctypes.c_int * 2)(500, 0)
    obs = (ctypes.c_int * 1)(3)
    items = (ctypes.c_int * 2)(0, 100)
    var = (ctypes.c_int * 2)(1, 4)
    best = (ctypes.c_int * 4)()
    # a leaf size of 0, then an orbital block of 3, then 100 schedule items, then
    # kernel variant 4
    assert lib.tagi_autotune(bogus, bogus, bogus, bogus, 10, None, bogus, 1, 0, bogus, 1.0, 0.5, 4,
                             0, leafs, 2, obs, 1, items, 1, var, 1, 1, best, None, None) == -1
    assert b"leaf_sizes[1]" in lib.tagi_last_error()
    assert lib.tagi_autotune(bogus, bogus, bogus, bogus, 10, None, bogus, 1, 0, bogus, 1.0, 0.5, 4,
                             0, leafs, 1, obs, 1, items, 1, var, 1, 1, best, None, None) == -1
    assert b"obs[0]" in lib.tagi_last_error()
    ob4 = (ctypes.c_int * 1)(4)
    assert lib.tagi_autotune(bogus, bogus, bogus, bogus, 10, None, bogus, 1, 0, bogus, 1.0, 0.5, 4,
                             0, leafs, 1, ob4, 1, items, 2, var, 1, 1, best, None, None) == -1
    assert b"items[1]" in lib.tagi_last_error()
    assert lib.tagi_autotune(bogus, bogus, bogus, bogus, 10, None, bogus, 1, 0, bogus, 1.0, 0.5, 4,
                             0, leafs, 1, ob4, 1, items, 1, var, 2, 1, best, None, None) == -1
    assert b"variants[1]" in lib.tagi_last_error()
    lib.tagi_autotune_learned.argtypes = [vp, vp, vp, vp, ctypes.c_int64, vp, vp, ctypes.c_int,
                                          ctypes.c_int, vp, ctypes.c_double, vp, vp, vp,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int, vp,
                                          ctypes.c_int, vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    assert lib.tagi_autotune_learned(bogus, bogus, bogus, bogus, 10, None, bogus, 1, 0, bogus,
                                     1.0, None, bogus, bogus, 0.9, 0.7, 8, 1, leafs, 1, ob4, 1,
                                     items, 1, var, 1, 1, best, None, None) == -1
    assert b"null selector argument" in lib.tagi_last_error()
    assert lib.tagi_autotune_learned(bogus, bogus, bogus, bogus, 10, None, bogus, 1, 0, bogus,
                                     1.0, bogus, bogus, bogus, 0.9, 0.7, 8, 1, leafs, 1, ob4, 1,
                                     items, 1, var, 2, 1, best, None, None) == -1
    assert b"tagi_autotune_learned: variants[1]" in lib.tagi_last_error()
    lib.tagi_tree_set_schedule_items.argtypes = [vp, ctypes.c_int]
    assert lib.tagi_tree_set_schedule_items(None, 4096) == -1
    lib.tagi_tree_set_kernel_variant.argtypes = [vp, ctypes.c_int]
    assert lib.tagi_tree_set_kernel_variant(None, 1) == -1
    lib.tagi_green_step.argtypes = [vp, vp, vp, vp, i32, vp, dbl, i32, i32, vp, vp, vp]
    eps = (ctypes.c_double * 1)(-1.0)
    assert lib.tagi_green_step(None, bogus, bogus, bogus, 1, eps, 0.7, 6, 0, bogus, None, None) == -1
    lib.tagi_green_step_learned.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp, dbl, dbl, i32,
                                            i32, vp, vp, vp]
    tol = (ctypes.c_double * 1)(1e-6)
    assert lib.tagi_green_step_learned(None, bogus, bogus, bogus, 1, eps, bogus, bogus, tol, 0.9,
                                       0.7, 8, 0, bogus, None, None) == -1
    assert b"tree is NULL" in lib.tagi_last_error()
    assert lib.tagi_tree_destroy(None) == 0


def test_workspace_held_reports_nothing_before_device_work():
    lib = _lib()
    lib.tagi_workspace_held.argtypes = [ctypes.c_void_p]
    lib.tagi_last_error.restype = ctypes.c_char_p
    held = ctypes.c_int64(-1)
    assert lib.tagi_workspace_held(ctypes.byref(held)) == 0 and held.value == 0
    assert lib.tagi_workspace_held(None) == -1
    assert b"bytes is NULL" in lib.tagi_last_error()


@pytest.mark.parametrize("value,limit", [("1", 1), ("3K", 3 << 10), ("2m", 2 << 20)])
def test_workspace_limit_refuses_the_first_allocation(monkeypatch, value, limit):
    # a tree needs far more than these limits: its first buffer is refused before
    # any device allocation is attempted, with the limit read back in the message
    lib = _lib()
    vp = ctypes.c_void_p
    lib.tagi_tree_build.argtypes = [vp, vp, vp, ctypes.c_int64, vp, ctypes.c_int, vp,
                                    ctypes.POINTER(vp)]
    lib.tagi_last_error.restype = ctypes.c_char_p
    monkeypatch.setenv("TAGI_WORKSPACE_LIMIT", value)
    n = 1 << 20
    bogus = ctypes.c_void_p(0x1000)  # never dereferenced: the limit stops the call first
    tree = vp()
    assert lib.tagi_tree_build(bogus, bogus, bogus, n, None, 64, None, ctypes.byref(tree)) == -3
    msg = lib.tagi_last_error().decode()
    assert "TAGI_WORKSPACE_LIMIT = %d bytes" % limit in msg and not tree.value
