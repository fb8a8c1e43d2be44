"""Pins of the oracle's Yee FDTD update.

* div^+ curl^+ = 0 and div^- curl^- = 0 (section "FDTD method"): a field
  update leaves the matching divergence unchanged to roundoff.
* curl^+ and curl^- are transposes on a periodic grid (dot-product test).
* A single standing Fourier mode obeys the leap-frog recurrence
  E^{n+1} + E^{n-1} = 2 cos(omega dt) E^n with the discrete vacuum
  dispersion sin^2(omega dt/2)/dt^2 = sum_d sin^2(k_d dx_d/2)/dx_d^2.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O


def _g(dim):
    n = (6 if dim == 3 else 1, 12, 10)
    return O.grid(dim, n, (0.3, 0.2, 0.25), 0.05, 1), n


@pytest.mark.parametrize("dim", [2, 3])
def test_divergence_free_updates(dim):
    g, n = _g(dim)
    nc = n[0] * n[1] * n[2]
    rng = np.random.default_rng(dim)
    E = rng.normal(size=3 * nc)
    B = rng.normal(size=3 * nc)
    db0, de0 = O.div_b(g, B), O.div_e(g, E)
    O.push_b(g, E, B, 0.37)
    assert np.abs(O.div_b(g, B) - db0).max() < 1e-12 * np.abs(db0).max()
    O.push_e(g, E, B, None, 0.41)
    assert np.abs(O.div_e(g, E) - de0).max() < 1e-12 * np.abs(de0).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_curls_are_transposes(dim):
    g, n = _g(dim)
    nc = n[0] * n[1] * n[2]
    rng = np.random.default_rng(10 + dim)
    E = rng.normal(size=3 * nc)
    B = rng.normal(size=3 * nc)
    zero = np.zeros(3 * nc)
    cE = zero.copy()
    O.push_b(g, E, cE, -1.0)          # cE = curl^+ E
    cB = zero.copy()
    O.push_e(g, cB, B, None, 1.0)     # cB = curl^- B
    assert abs(cE @ B - E @ cB) < 1e-11 * np.abs(cE @ B)


@pytest.mark.parametrize("dim", [2, 3])
def test_standing_mode_dispersion(dim):
    g, n = _g(dim)
    nc = n[0] * n[1] * n[2]
    mx, my, mz = (1 if dim == 3 else 0), 2, 1
    kd = [2 * math.pi * mx / n[0], 2 * math.pi * my / n[1], 2 * math.pi * mz / n[2]]
    d = [g.d[0], g.d[1], g.d[2]]
    s2 = sum(math.sin(kd[a] / 2) ** 2 / d[a] ** 2 for a in range(3) if (dim == 3 or a > 0))
    cos_w = 1 - 2 * g.dt ** 2 * s2
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    E = np.zeros(3 * nc)
    B = np.zeros(3 * nc)
    # a transverse mode: E along a direction with zero discrete divergence
    if dim == 2:
        E[:nc] = (np.cos(kd[1] * j) * np.cos(kd[2] * k)).ravel()   # E_x, out of plane
    else:
        E[:nc] = (np.cos(kd[0] * (i + 0.5)) * np.cos(kd[1] * j) * np.cos(kd[2] * k)).ravel()
        E[:nc] *= 0  # keep the test to a pure single-component transverse mode
        E[2 * nc:] = (np.cos(kd[0] * i) * np.cos(kd[1] * j)).ravel()    # E_z(x,y), kz = 0
        s2 = sum(math.sin(kd[a] / 2) ** 2 / d[a] ** 2 for a in (0, 1))
        cos_w = 1 - 2 * g.dt ** 2 * s2
    hist = []
    for _ in range(40):
        hist.append(E.copy())
        O.push_b(g, E, B, 0.5 * g.dt)
        O.push_b(g, E, B, 0.5 * g.dt)
        O.push_e(g, E, B, None, g.dt)
    hist = np.array(hist)
    res = hist[2:] + hist[:-2] - 2 * cos_w * hist[1:-1]
    assert np.abs(res).max() < 1e-12
