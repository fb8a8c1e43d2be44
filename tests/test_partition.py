"""The greedy partition of App. A ("Load balancing algorithm").

Checked against a direct Python transcription of the appendix's description
(walk the space-filling curve, fill each rank up to T_hat * C_r, keep or pass
on the boundary patch by which side lands closer to the target, give one
patch to each remaining rank once patches run short, the last rank takes the
rest) and against the properties any such partition has: every patch is
assigned once, in order, and with at least as many patches as ranks no rank
is empty.  Pure host code: runs without a GPU.
"""
import numpy as np
import pytest

from paper_1310_7866_amd import psc


def reference(L, C):
    P, R = len(L), len(C)
    T = sum(L) / sum(C)
    N = [0] * R
    r, n, load = 0, 0, 0.0
    for p in range(P):
        load += L[p]
        n += 1
        if r < R - 1:
            target = T * C[r]
            if load > target or R - r >= P - p:
                over = load - target
                under = target - (load - L[p])
                if over > under and n > 1:
                    N[r], n, load = n - 1, 1, L[p]
                else:
                    N[r], n, load = n, 0, 0.0
                r += 1
        if p == P - 1:
            N[R - 1] += n
    return N


def _lib_or_skip():
    import os
    if not os.path.exists(psc.LIB_PATH):
        pytest.skip("libpsc.so not built")


@pytest.mark.parametrize("seed", range(8))
def test_partition_matches_reference(seed):
    _lib_or_skip()
    rng = np.random.default_rng(seed)
    P = int(rng.integers(1, 300))
    R = int(rng.integers(1, 40))
    L = rng.gamma(2.0, 50.0, P) + 10
    C = rng.choice([1.0, 1.0, 1.0, 60.0], R) if seed % 2 else np.ones(R)
    got = psc.partition(L, C)
    assert list(got) == reference(list(L), list(C))
    assert got.sum() == P
    if P >= R:
        assert (got >= 1).all()


def test_partition_uniform_and_skewed():
    _lib_or_skip()
    # uniform loads split evenly
    got = psc.partition(np.ones(64), np.ones(16))
    assert (got == 4).all()
    # a rank 60x as capable (the paper's GPU-vs-core capability) gets ~60x load
    L = np.ones(610)
    C = np.array([60.0] + [1.0] * 10)
    got = psc.partition(L, C)
    T = L.sum() / C.sum()               # 610 / 70
    assert abs(got[0] - 60 * T) <= 0.5  # 523 patches
    loads = np.add.reduceat(L, np.concatenate([[0], np.cumsum(got)[:-1]]))
    # each rank but the last lands within half a patch of its target; the
    # greedy walk leaves the accumulated rounding to the last rank
    assert np.all(np.abs(loads[:-1] - T * C[:-1]) <= 0.5 * L.max() + 1e-9)
    assert got.sum() == L.size
