"""Pins of the oracle's Esirkepov current deposit.

* Discrete charge continuity (rho^{n+1/2} - rho^{n-1/2})/dt + div^- J = 0
  (section "FDTD method", continuity equation) by brute force on random
  single-particle moves with and without cell crossings, 2-d and 3-d, both
  orders; rho comes from an independent node deposit of the shape.
* Total current: the sum of J_d over the grid equals q w v_d (first moment).
* Moves inside one cell at order 1: in-plane components equal the
  Villasenor-Buneman area weighting; the 3-d components and the 2-d
  out-of-plane J_x equal the exact time average of the linear weights along
  the straight path, computed here by quadrature.
* A particle at rest deposits nothing.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as O


def _grid(dim, order):
    n = (9 if dim == 3 else 1, 10, 11)
    return O.grid(dim, n, (0.3, 0.2, 0.25), 0.04, order), n


def _rand_move(rng, dim, n, cross):
    lo = 1.0
    x0 = np.array([rng.uniform(lo, n[0] - lo) if dim == 3 else 0.0,
                   rng.uniform(lo, n[1] - lo), rng.uniform(lo, n[2] - lo)])
    if not cross:
        # stay inside the starting cell
        x0 = np.floor(x0) + rng.uniform(0.1, 0.9, 3)
        if dim == 2:
            x0[0] = 0.0
        f = np.floor(x0)
        x1 = f + rng.uniform(0.0, 1.0, 3) * 0.999
    else:
        x1 = x0 + rng.uniform(-0.99, 0.99, 3)
    if dim == 2:
        x1[0] = x0[0]
    return x0, x1


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("cross", [False, True])
def test_continuity(dim, order, cross):
    g, n = _grid(dim, order)
    nc = n[0] * n[1] * n[2]
    rng = np.random.default_rng(100 * dim + 10 * order + cross)
    qw = -0.37
    for _ in range(30):
        x0, x1 = _rand_move(rng, dim, n, cross)
        J = O.deposit(g, x0, x1, qw, 0.123)
        r0 = O.rho_of(g, x0, qw)
        r1 = O.rho_of(g, x1, qw)
        # discrete div^- of J at nodes (E-like staggering)
        div = O.div_e(g, J)
        res = (r1 - r0) / g.dt + div
        assert np.abs(res).max() < 1e-12 * abs(qw) / g.dt


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("order", [1, 2])
def test_total_current_and_rest(dim, order):
    g, n = _grid(dim, order)
    nc = n[0] * n[1] * n[2]
    rng = np.random.default_rng(7 * dim + order)
    qw, vx = 0.8, -0.31
    for _ in range(20):
        x0, x1 = _rand_move(rng, dim, n, True)
        J = O.deposit(g, x0, x1, qw, vx).reshape(3, nc)
        d = np.array([g.d[0], g.d[1], g.d[2]])
        for c in range(3):
            if dim == 2 and c == 0:
                want = qw * vx
            else:
                want = qw * (x1[c] - x0[c]) * d[c] / g.dt
            assert abs(J[c].sum() - want) < 1e-12 * (1 + abs(want))
        J0 = O.deposit(g, x0, x0, qw, 0.0)
        assert np.abs(J0).max() == 0.0


def _lin_weights(x):
    f = np.floor(x)
    return f, 1.0 - (x - f), x - f


def test_order1_inside_cell_2d_matches_area_weighting_and_time_average():
    g, n = _grid(2, 1)
    nc = n[0] * n[1] * n[2]
    rng = np.random.default_rng(5)
    qw, vx = 0.6, 0.27
    for _ in range(20):
        x0, x1 = _rand_move(rng, 2, n, False)
        J = O.deposit(g, x0, x1, qw, vx).reshape(3, n[2], n[1])
        j, k = int(np.floor(x0[1])), int(np.floor(x0[2]))
        ym, zm = 0.5 * (x0[1] + x1[1]) - j, 0.5 * (x0[2] + x1[2]) - k
        vy = (x1[1] - x0[1]) * g.d[1] / g.dt
        vz = (x1[2] - x0[2]) * g.d[2] / g.dt
        ref = np.zeros((3, n[2], n[1]))
        ref[1, k, j] = qw * vy * (1 - zm)
        ref[1, k + 1, j] = qw * vy * zm
        ref[2, k, j] = qw * vz * (1 - ym)
        ref[2, k, j + 1] = qw * vz * ym

        def shape(t, a, b):
            y = x0[1] + t * (x1[1] - x0[1]) - j
            z = x0[2] + t * (x1[2] - x0[2]) - k
            return (y if a else 1 - y) * (z if b else 1 - z)

        for a in (0, 1):
            for b in (0, 1):
                avg, _ = integrate.quad(shape, 0, 1, args=(a, b))
                ref[0, k + b, j + a] = qw * vx * avg
        assert np.abs(J - ref).max() < 1e-13


def test_order1_inside_cell_3d_matches_time_average():
    g, n = _grid(3, 1)
    rng = np.random.default_rng(6)
    qw = -0.45
    for _ in range(10):
        x0, x1 = _rand_move(rng, 3, n, False)
        J = O.deposit(g, x0, x1, qw, 0.0).reshape(3, n[2], n[1], n[0])
        c0 = np.floor(x0).astype(int)
        v = (x1 - x0) * np.array([g.d[0], g.d[1], g.d[2]]) / g.dt
        for comp in range(3):
            others = [d for d in range(3) if d != comp]
            for a in (0, 1):
                for b in (0, 1):
                    def shape(t):
                        p = x0 + t * (x1 - x0) - c0
                        wa = p[others[0]] if a else 1 - p[others[0]]
                        wb = p[others[1]] if b else 1 - p[others[1]]
                        return wa * wb
                    avg, _ = integrate.quad(shape, 0, 1)
                    idx = list(c0)
                    idx[others[0]] += a
                    idx[others[1]] += b
                    got = J[comp, idx[2], idx[1], idx[0]]
                    assert abs(got - qw * v[comp] * avg) < 1e-12
