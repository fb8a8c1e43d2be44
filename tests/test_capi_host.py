"""CPU tests of the C ABI: the library loads, exports every symbol that
include/psc.h declares, and validates descriptors synchronously (no device
work is issued by psc_init_patches)."""
import ctypes as C
import os
import re

import pytest

from paper_1310_7866_amd import cases, psc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(psc.LIB_PATH):
        pytest.skip("libpsc.so not built")
    return psc.load_library()


def test_header_symbols_exported():
    L = _lib()
    header = open(os.path.join(ROOT, "include", "psc.h")).read()
    declared = set(re.findall(r"^(?:psc_status|const char \*)\s*(psc_\w+)\s*\(", header, re.M))
    assert declared, "no declarations parsed"
    assert declared == set(psc.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def _init(desc, chunk=0):
    L = _lib()
    ctx = C.c_void_p()
    arr = (psc.RunDesc * 1)(desc)
    st = L.psc_init_patches(arr, 1, chunk, C.byref(ctx))
    if st == 0:
        size = C.c_size_t()
        L.psc_destroy(ctx)
    return st


def test_valid_descriptor_accepted():
    c = cases.thermal2d(ny=16, nz=12, ppc=2, patch=8)
    assert _init(psc.run_desc(c)) == 0


def test_cfl_violation_rejected():
    c = cases.thermal2d(ny=16, nz=12, ppc=2, patch=8)
    d = psc.run_desc(c)
    d.dt = 1.0 / (1.0 / 0.1 ** 2 + 1.0 / 0.1 ** 2) ** 0.5 * 1.001
    assert _init(d) == 2


def test_bad_geometry_rejected():
    c = cases.thermal2d(ny=16, nz=12, ppc=2, patch=8)
    d = psc.run_desc(c)
    d.gdims[0] = 2                      # 2-d needs nx == 1
    assert _init(d) == 1
    d = psc.run_desc(c)
    d.patch[1] = 17                     # patch larger than the grid
    assert _init(d) == 1
    d = psc.run_desc(c)
    d.gdims[2] = 2                      # fewer than 3 cells along an active axis
    d.patch[2] = 2
    assert _init(d) == 1
    d = psc.run_desc(c)
    d.order = 3
    assert _init(d) == 1


def test_capacity_limit():
    # the byte offsets of a species' arrays stay below 2^32 (the kernels
    # address them as a base plus a 32-bit offset)
    c = cases.thermal2d(ny=16, nz=12, ppc=2, patch=8)
    d = psc.run_desc(c)
    d.capacity[0] = (1 << 30) - 1024
    assert _init(d) == 0
    d.capacity[0] = (1 << 30) - 1023
    assert _init(d) == 1


def test_patches_narrower_than_the_current_halo_rejected():
    """The current fold reads a cell's own patch and its two neighbours: with
    more than three patches along a dimension, a patch (or the truncated last
    one) narrower than order + 1 cells would drop current.  Init refuses it."""
    for order, patch, n, ok in ((2, 2, 16, False), (2, 3, 15, True), (1, 2, 16, True), (1, 1, 16, False),
                                (2, 8, 26, False), (2, 8, 27, True), (2, 2, 6, True)):
        c = cases.thermal2d(ny=n, nz=12, ppc=1, patch=8, order=order)
        d = psc.run_desc(c)
        d.patch[1] = patch
        want = 0 if ok else 1
        assert _init(d) == want, (order, patch, n)


def test_vb_flag_rules():
    """The Villasenor-Buneman deposit is a 1st-order option without the adjoint."""
    d = psc.run_desc(cases.thermal2d(ny=16, nz=12, ppc=1, patch=8, order=1))
    d.flags = psc.RUN_VB
    assert _init(d) == 0
    d = psc.run_desc(cases.thermal2d(ny=16, nz=12, ppc=1, patch=8, order=2))
    d.flags = psc.RUN_VB
    assert _init(d) == 7
    d = psc.run_desc(cases.thermal2d(ny=16, nz=12, ppc=1, patch=8, order=1))
    d.flags = psc.RUN_VB | psc.RUN_ADJOINT
    assert _init(d) == 7


def test_lds_overflow_rejected():
    c = cases.thermal2d(ny=128, nz=128, ppc=1, patch=64, order=2)
    assert _init(psc.run_desc(c)) == 3


def test_mixed_orders_unsupported():
    L = _lib()
    a = psc.run_desc(cases.thermal2d(ny=16, nz=16, ppc=1, patch=8, order=1))
    b = psc.run_desc(cases.thermal2d(ny=16, nz=16, ppc=1, patch=8, order=2))
    ctx = C.c_void_p()
    arr = (psc.RunDesc * 2)(a, b)
    assert L.psc_init_patches(arr, 2, 0, C.byref(ctx)) == 7


def test_status_strings():
    L = _lib()
    for s in range(9):
        assert L.psc_status_string(s)
