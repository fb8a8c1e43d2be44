"""CPU tests of the patch order along the Hilbert-Peano curve (section
"Dynamic load balancing using space filling curves"), a host function of
the library (psc_hilbert_order).

The curve is pinned by what defines it rather than by a second
implementation: it visits every patch once (bijection); consecutive patches
are face neighbours (continuity); and, on a cube of side 2^k, every aligned
sub-cube of side 2^j is one contiguous segment of the curve (the recursive
quadrant/octant structure that separates a Hilbert curve from a serpentine
row order, which is continuous too).  The section's own example -- 16 x 16
patches on 16 processes give the same 4 x 4 blocks as the standard
decomposition -- is the j = 2 case in 2-d.
"""
import itertools

import numpy as np
import pytest

from paper_1310_7866_amd import psc


def _lib_or_skip():
    import os
    if not os.path.exists(psc.LIB_PATH):
        pytest.skip("libpsc.so not built")


def coords(order, np_):
    o = np.asarray(order, dtype=np.int64)
    return np.stack([o % np_[0], (o // np_[0]) % np_[1], o // (np_[0] * np_[1])], axis=1)


def jumps(order, np_):
    c = coords(order, np_)
    d = np.abs(np.diff(c, axis=0)).sum(axis=1)
    return int((d != 1).sum())


def cut_size(order, np_, n_seg):
    """Face-neighbour pairs of patches (non-periodic) that lie in different
    segments when the order is split into n_seg equal consecutive parts."""
    n = len(order)
    seg = np.empty(n, np.int64)
    seg[np.asarray(order)] = np.arange(n) * n_seg // n
    g = seg.reshape(np_[2], np_[1], np_[0])
    cut = 0
    for ax in range(3):
        if g.shape[ax] > 1:
            a = np.take(g, range(1, g.shape[ax]), axis=ax)
            b = np.take(g, range(0, g.shape[ax] - 1), axis=ax)
            cut += int((a != b).sum())
    return cut


SHAPES = [(2, (1, 16, 16)), (2, (1, 32, 16)), (2, (1, 16, 32)), (2, (1, 13, 7)), (2, (1, 5, 3)),
          (2, (1, 1, 9)), (2, (1, 64, 32)), (3, (8, 8, 8)), (3, (4, 8, 8)), (3, (8, 4, 4)),
          (3, (6, 5, 7)), (3, (3, 3, 3)), (3, (32, 32, 32))]


@pytest.mark.parametrize("dim,np_", SHAPES)
def test_bijection(dim, np_):
    _lib_or_skip()
    o = psc.hilbert_order(dim, np_)
    assert sorted(o.tolist()) == list(range(np_[0] * np_[1] * np_[2]))


@pytest.mark.parametrize("dim,np_", [(2, (1, 2, 2)), (2, (1, 16, 16)), (2, (1, 64, 64)), (3, (2, 2, 2)),
                                     (3, (8, 8, 8)), (3, (32, 32, 32))])
def test_power_of_two_cube_is_a_hilbert_curve(dim, np_):
    """Continuity, and every aligned sub-cube of side 2^j is a contiguous
    segment of the curve."""
    _lib_or_skip()
    o = psc.hilbert_order(dim, np_)
    assert jumps(o, np_) == 0
    c = coords(o, np_)
    side = max(np_)
    act = [0, 1, 2] if dim == 3 else [1, 2]
    s = 2
    while s <= side:
        block = np.zeros(len(o), np.int64)
        for k, a in enumerate(act):
            block = block * (side // s) + c[:, a] // s
        seglen = s ** len(act)
        segs = block.reshape(-1, seglen)
        assert (segs == segs[:, :1]).all(), f"sub-cubes of side {s} are not contiguous"
        assert len(np.unique(segs[:, 0])) == len(segs)
        s *= 2


def test_paper_example_16x16_patches_on_16_processes():
    """Splitting the 256-patch curve into 16 segments of 16 patches gives
    the 4 x 4 blocks of the standard decomposition."""
    _lib_or_skip()
    np_ = (1, 16, 16)
    c = coords(psc.hilbert_order(2, np_), np_)
    blocks = set()
    for seg in range(16):
        cs = c[16 * seg:16 * (seg + 1)]
        ys, zs = set(cs[:, 1] // 4), set(cs[:, 2] // 4)
        assert len(ys) == 1 and len(zs) == 1
        assert len(set(map(tuple, cs[:, 1:] % 4))) == 16
        blocks.add((ys.pop(), zs.pop()))
    assert len(blocks) == 16


@pytest.mark.parametrize("dim,np_", [(2, (1, 32, 16)), (2, (1, 16, 32)), (3, (8, 4, 4)), (3, (4, 8, 4)),
                                     (3, (8, 8, 4)), (3, (4, 8, 8))])
def test_boxes_filling_a_leading_part_of_the_curve_are_continuous(dim, np_):
    """2:1 boxes in 2-d (the Harris workload's 32 x 16 patches) and 2:1:1 or
    2:2:1 boxes in 3-d are a leading part of the enclosing cube's curve."""
    _lib_or_skip()
    assert jumps(psc.hilbert_order(dim, np_), np_) == 0


@pytest.mark.parametrize("dim,np_", [(2, (1, 13, 7)), (2, (1, 5, 3)), (2, (1, 63, 17)), (3, (6, 5, 7)),
                                     (3, (3, 3, 3)), (3, (5, 9, 3))])
def test_ragged_grids_keep_locality(dim, np_):
    """Grids that are not a leading part of a power-of-two curve keep most
    consecutive pairs adjacent."""
    _lib_or_skip()
    o = psc.hilbert_order(dim, np_)
    n = len(o)
    assert jumps(o, np_) <= max(2, n // 10)


@pytest.mark.parametrize("dim,np_,n_seg", [(2, (1, 32, 16), 8), (3, (32, 32, 32), 8), (2, (1, 16, 16), 16),
                                           (3, (8, 8, 8), 64), (2, (1, 13, 7), 8)])
def test_segments_are_more_compact_than_row_major(dim, np_, n_seg):
    """Equal segments of the curve (one per XCD queue, or per rank) share
    fewer patch faces with each other than equal row-major strips."""
    _lib_or_skip()
    o = psc.hilbert_order(dim, np_)
    rm = np.arange(len(o))
    assert cut_size(o, np_, n_seg) < cut_size(rm, np_, n_seg)


def test_invalid_sizes_rejected():
    _lib_or_skip()
    L = psc.load_library()
    import ctypes as C
    out = np.zeros(64, np.int32)
    for dim, n in [(2, (2, 4, 4)), (4, (1, 4, 4)), (3, (0, 4, 4)), (2, (1, -1, 4))]:
        a = np.asarray(n, np.int32)
        st = L.psc_hilbert_order(dim, a.ctypes.data_as(C.POINTER(C.c_int32)),
                                 out.ctypes.data_as(C.POINTER(C.c_int32)))
        assert st == 1
