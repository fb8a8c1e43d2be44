"""Pins of the oracle's shape functions and interpolation.

B-splines: the printed b1/b2 are checked against the recursive definition
(b_{n+1} is b_n folded with the flat-top b0, section "Time integration of the
quasi-particle equations of motion") by numerical quadrature, and against
their moments.  Interpolation (eq. E_interp with piecewise-constant fields,
which gives B-spline weights one order up) is pinned by exactness on
constant and linear fields.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as O


def b0(s):
    return 1.0 if abs(s) < 0.5 else 0.0


@pytest.mark.parametrize("order", [1, 2])
def test_bspline_is_fold_of_lower_order(order):
    rng = np.random.default_rng(11)
    for s in rng.uniform(-2.0, 2.0, 25):
        # (b0 * b_{order-1})(s) = int b0(s - t) b_{order-1}(t) dt, integrand supported on |s-t| < 1/2
        val, _ = integrate.quad(lambda t: O.bspline(order - 1, t), s - 0.5, s + 0.5,
                                points=[-1.5, -1.0, -0.5, 0.0, 0.5, 1.0, 1.5], limit=200)
        assert abs(val - O.bspline(order, s)) < 1e-10


@pytest.mark.parametrize("order", [1, 2])
def test_bspline_moments(order):
    rng = np.random.default_rng(12)
    nodes = np.arange(-5, 6)
    for xi in rng.uniform(-1.0, 1.0, 200):
        w = np.array([O.bspline(order, xi - n) for n in nodes])
        assert abs(w.sum() - 1.0) < 1e-14                      # partition of unity
        assert abs((w * nodes).sum() - xi) < 1e-14             # first moment
        second = (w * (nodes - xi) ** 2).sum()
        if order == 2:
            assert abs(second - 0.25) < 1e-14                 # b2 variance = 1/12 + 1/6
        else:
            d = xi - np.floor(xi)
            assert abs(second - d * (1 - d)) < 1e-14


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("dim", [2, 3])
def test_interp_exact_on_linear_fields(order, dim):
    rng = np.random.default_rng(13 + dim * 7 + order)
    n = (16 if dim == 3 else 1, 20, 24)
    g = O.grid(dim, n, (0.3, 0.2, 0.25), 0.05, order)
    nc = n[0] * n[1] * n[2]
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    for stag in list(O.STAG_E) + list(O.STAG_B):
        a, b = rng.normal(size=4), rng.normal(size=1)
        F = (a[0] + a[1] * (i + stag[0]) * (dim == 3) + a[2] * (j + stag[1]) + a[3] * (k + stag[2])).ravel()
        for _ in range(10):
            xi = np.array([rng.uniform(5, n[0] - 5) if dim == 3 else 0.0,
                           rng.uniform(5, n[1] - 5), rng.uniform(5, n[2] - 5)])
            want = a[0] + a[1] * xi[0] * (dim == 3) + a[2] * xi[1] + a[3] * xi[2]
            assert abs(O.interp(g, F, xi, stag) - want) < 1e-12 * (1 + abs(want))
        G = np.full(nc, b[0])
        xi = np.array([1.3, 0.01, n[2] - 0.02])   # next to the periodic seam
        assert abs(O.interp(g, G, xi, stag) - b[0]) < 1e-14
