"""Pins of the oracle's Villasenor-Buneman deposit (the paper's scheme for
1st-order particles, section "Time integration of the quasi-particle
equations of motion").

* Discrete charge continuity (rho^{n+1/2} - rho^{n-1/2})/dt + div^- J = 0 by
  brute force on random moves with cell crossings (up to three pieces in
  2-d, four in 3-d), rho from the independent node deposit of the linear
  shape.
* Total current q w v_d per component.
* Moves inside one cell: in 3-d, and for the in-plane components in 2-d, the
  current equals the Esirkepov deposit (both are the exact flux of the
  linear cloud); the 2-d out-of-plane J_x is q w v_x times the linear weights
  at the midpoint (Esirkepov instead averages them along the path: the two
  differ by q w v_x dy dz / 12 at each node, with alternating sign).
* A move across one face equals the sum of two in-cell moves cut at the
  face, computed here by hand from the in-cell current of each piece.
"""
import numpy as np
import pytest

from oracle import oracle as O


def _grid(dim):
    n = (9 if dim == 3 else 1, 10, 11)
    return O.grid(dim, n, (0.3, 0.2, 0.25), 0.04, 1), n


def _move(rng, dim, n, cross):
    x0 = np.array([rng.uniform(1, n[0] - 1) if dim == 3 else 0.0, rng.uniform(1, n[1] - 1), rng.uniform(1, n[2] - 1)])
    if cross:
        x1 = x0 + rng.uniform(-0.99, 0.99, 3)
    else:
        x0 = np.floor(x0) + rng.uniform(0.05, 0.95, 3)
        x1 = np.floor(x0) + rng.uniform(0.0, 0.999, 3)
    if dim == 2:
        x0[0] = x1[0] = 0.0
    return x0, x1


@pytest.mark.parametrize("dim", [2, 3])
def test_continuity_with_crossings(dim):
    g, n = _grid(dim)
    rng = np.random.default_rng(400 + dim)
    qw = 0.61
    crossed = 0
    for _ in range(60):
        x0, x1 = _move(rng, dim, n, True)
        crossed += int(np.any(np.floor(x0) != np.floor(x1)))
        J = O.deposit_vb(g, x0, x1, qw, 0.2)
        res = (O.rho_of(g, x1, qw) - O.rho_of(g, x0, qw)) / g.dt + O.div_e(g, J)
        assert np.abs(res).max() < 1e-12 * qw / g.dt
    assert crossed > 30


@pytest.mark.parametrize("dim", [2, 3])
def test_total_current(dim):
    g, n = _grid(dim)
    nc = n[0] * n[1] * n[2]
    rng = np.random.default_rng(410 + dim)
    qw, vx = -0.8, 0.37
    for _ in range(30):
        x0, x1 = _move(rng, dim, n, True)
        J = O.deposit_vb(g, x0, x1, qw, vx).reshape(3, nc)
        for c in range(3):
            want = qw * vx if (dim == 2 and c == 0) else qw * (x1[c] - x0[c]) * g.d[c] / g.dt
            assert abs(J[c].sum() - want) < 1e-12 * (1 + abs(want))


@pytest.mark.parametrize("dim", [2, 3])
def test_in_cell_moves_against_esirkepov(dim):
    g, n = _grid(dim)
    nc = n[0] * n[1] * n[2]
    rng = np.random.default_rng(420 + dim)
    qw, vx = 0.5, -0.9
    for _ in range(30):
        x0, x1 = _move(rng, dim, n, False)
        Jv = O.deposit_vb(g, x0, x1, qw, vx).reshape(3, nc)
        Je = O.deposit(g, x0, x1, qw, vx).reshape(3, nc)
        comps = (0, 1, 2) if dim == 3 else (1, 2)
        for c in comps:
            assert np.abs(Jv[c] - Je[c]).max() < 1e-12 * (1 + np.abs(Je[c]).max())
        if dim == 2:
            # out of plane: midpoint weights vs the path average
            m = 0.5 * (x0 + x1)
            j0, k0 = int(np.floor(m[1])), int(np.floor(m[2]))
            dy, dz = x1[1] - x0[1], x1[2] - x0[2]
            for b in (0, 1):
                for e in (0, 1):
                    wy = m[1] - j0 if b else 1 - (m[1] - j0)
                    wz = m[2] - k0 if e else 1 - (m[2] - k0)
                    node = (j0 + b) + n[1] * (k0 + e)
                    assert abs(Jv[0][node] - qw * vx * wy * wz) < 1e-13
                    sg = 1.0 if b == e else -1.0
                    assert abs(Je[0][node] - Jv[0][node] - qw * vx * sg * dy * dz / 12.0) < 1e-13


def test_one_face_crossing_is_two_pieces_2d():
    g, n = _grid(2)
    nc = n[1] * n[2]
    qw, vx = 1.0, 0.25
    x0 = np.array([0.0, 3.8, 5.3])
    x1 = np.array([0.0, 4.4, 5.5])          # crosses y = 4 at t = 1/3
    t = (4.0 - x0[1]) / (x1[1] - x0[1])
    xm = x0 + t * (x1 - x0)
    Jv = O.deposit_vb(g, x0, x1, qw, vx).reshape(3, nc)
    want = np.zeros((3, nc))
    for a, b, frac in ((x0, xm, t), (xm, x1, 1 - t)):
        mid = 0.5 * (a + b)
        j0, k0 = int(np.floor(mid[1])), int(np.floor(mid[2]))
        my, mz = mid[1] - j0, mid[2] - k0
        dy, dz = b[1] - a[1], b[2] - a[2]
        fy, fz = qw * g.d[1] / g.dt, qw * g.d[2] / g.dt
        want[1][j0 + n[1] * k0] += fy * dy * (1 - mz)
        want[1][j0 + n[1] * (k0 + 1)] += fy * dy * mz
        want[2][j0 + n[1] * k0] += fz * dz * (1 - my)
        want[2][j0 + 1 + n[1] * k0] += fz * dz * my
        for bb, wy in ((0, 1 - my), (1, my)):
            for ee, wz in ((0, 1 - mz), (1, mz)):
                want[0][j0 + bb + n[1] * (k0 + ee)] += qw * vx * frac * wy * wz
    assert np.abs(Jv - want).max() < 1e-12
