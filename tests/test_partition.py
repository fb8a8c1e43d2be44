"""The greedy partition of App. A ("Load balancing algorithm").

Checked against a direct Python transcription of the appendix (walk the
space-filling curve adding patches to rank r; the running load is never reset
between ranks, so it is compared with the cumulative target T_hat * (C_0 +
... + C_r); at the crossing patch keep it on r or open r + 1 with it,
whichever lands closer to the target; give one patch to each remaining rank
once patches run short; the last rank takes the rest) and against the
properties such a partition has: every patch is assigned once, in order,
with at least as many patches as ranks no rank is empty, every boundary lies
within half a patch of its cumulative target, so no rank (the last one
included) is off its target by more than one patch.  Pure host code: runs
without a GPU.
"""
import numpy as np
import pytest

from paper_1310_7866_amd import psc


def reference(L, C):
    P, R = len(L), len(C)
    T = sum(L) / sum(C)
    N = [0] * R
    r, n, load, target = 0, 0, 0.0, 0.0
    for p in range(P):
        load += L[p]
        n += 1
        if r < R - 1:
            t = target + T * C[r]
            if load > t or R - r >= P - p:
                over = load - t
                under = t - (load - L[p])
                if over > under and n > 1:
                    N[r], n = n - 1, 1
                else:
                    N[r], n = n, 0
                target = t
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
    assert np.all(np.abs(loads - T * C) <= L.max() + 1e-9)
    assert got.sum() == L.size


@pytest.mark.parametrize("R", [7, 256, 300, 512])
def test_partition_does_not_drift(R):
    """Uneven loads over many ranks: boundaries stay within half a patch of
    the cumulative targets, so the last rank is not left with the rounding of
    all earlier boundaries."""
    _lib_or_skip()
    rng = np.random.default_rng(R)
    L = rng.uniform(40000, 110000, 1024)
    C = np.ones(R)
    got = psc.partition(L, C)
    assert got.sum() == L.size and (got >= 1).all()
    bounds = np.cumsum(got)[:-1]
    cum = np.cumsum(L)[bounds - 1]
    T = L.sum() / C.sum()
    assert np.all(np.abs(cum - T * np.arange(1, R)) <= 0.5 * L.max() + 1e-6)
    loads = np.add.reduceat(L, np.concatenate([[0], bounds]))
    assert loads.max() <= T + L.max() + 1e-6
