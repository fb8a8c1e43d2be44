"""Why particles are stored as an integer cell plus a float32 offset.

The paper notes that single precision loses position resolution far from the
origin when positions are absolute (section on the particle data layout:
integer cell index plus in-cell offset).  This CPU ablation moves the same
particles by the same float32 displacements in both representations and
compares with the exact float64 result.  Along the 1024-cell y axis of the
Harris workload an absolute float32 position carries the spacing of floats
near 1024 (2^-13 cells), while an in-cell offset in [0, 1) keeps 2^-24 at
every cell.
"""
import numpy as np


def _absolute_f32(x0, d):
    return (x0.astype(np.float32) + d).astype(np.float64)


def _cell_offset_f32(x0, d):
    cell = np.floor(x0).astype(np.int64)
    off = (x0 - cell).astype(np.float32)
    o1 = off + d                                 # float32 arithmetic
    s = np.floor(o1).astype(np.int64)
    o1 = (o1 - s.astype(np.float32)).astype(np.float32)
    s = s + (o1 >= 1.0)                          # a sum that rounds up to 1 moves on
    o1 = np.where(o1 >= 1.0, np.float32(0.0), o1)
    return (cell + s).astype(np.float64) + o1.astype(np.float64)


def test_cell_offset_keeps_resolution_across_the_grid():
    rng = np.random.default_rng(1310)
    n = 200_000
    # cells across a 1024-cell axis; offsets representable in float32
    x0 = rng.integers(0, 1024, n) + rng.random(n).astype(np.float32).astype(np.float64)
    d = (rng.standard_normal(n) * 0.1).clip(-0.9, 0.9).astype(np.float32)
    exact = x0 + d.astype(np.float64)
    e_abs = np.abs(_absolute_f32(x0, d) - exact)
    e_cel = np.abs(_cell_offset_f32(x0, d) - exact)
    far = x0 >= 512
    # in-cell offsets: one rounding of a value below 2, at most 2^-23 cells
    assert e_cel.max() <= 2.0 ** -23
    # absolute float32 positions near 512..1025: storing the start rounds by
    # up to half a spacing of 2^-14, the sum by up to half of 2^-13
    assert e_abs[far].max() >= 2.0 ** -16
    assert e_abs[far].max() <= 2.0 ** -15 + 2.0 ** -14
    assert e_abs[far].mean() > 100 * e_cel[far].mean()


def test_many_steps_drift():
    """A particle crossing many cells: 2000 steps of a fixed float32
    displacement starting near cell 1000; the error of each representation
    against the exact sum."""
    x0 = np.array([1000.3], dtype=np.float64)
    d = np.array([0.0123], dtype=np.float32)
    xa = x0.copy()
    xc = x0.copy()
    for k in range(2000):
        xa = _absolute_f32(xa, d)
        xc = _cell_offset_f32(xc, d)
    exact = x0[0] + 2000 * float(d[0])
    err_a, err_c = abs(xa[0] - exact), abs(xc[0] - exact)
    print(f"2000 steps: absolute float32 error {err_a:.3e} cells, cell + offset {err_c:.3e}")
    assert err_c <= 2000 * 2.0 ** -24
    assert err_a > 100 * err_c
