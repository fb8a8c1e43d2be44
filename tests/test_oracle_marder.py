"""Pins of the oracle's Marder cleaning step (the iterative method the paper
names for dissipating violations of Gauss's law in long single-precision
runs): E += d dt grad^+ F with F the Gauss residual less its reference.

* A residual that is one Fourier mode is scaled by exactly
  1 + d dt lambda, lambda = -sum_d (4 / dx_d^2) sin^2(theta_d / 2), the
  eigenvalue of the discrete Laplacian div^- grad^+ (the particles do not
  move, so rho is unchanged).
* The step changes only the longitudinal part of E: curl^+ E (what drives B)
  is unchanged to round-off, since curl^+ grad^+ = 0 on the Yee grid.
* It is a no-op when the residual equals its reference.
* Repeated steps inside the stability bound d dt sum(4/dx^2) <= 2 drive a
  planted residual towards zero.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_1310_7866_amd import cases


def _sim(seed=7, ny=16, nz=12):
    c = cases.thermal2d(ny=ny, nz=nz, ppc=3, order=2, patch=4, seed=seed)
    cases.random_fields(c, 0.05, 0.3, seed=seed + 1)
    return c, O.OracleSim(c)


def _curl_plus(sim):
    """curl^+ E through the oracle's own B update: B change of a unit step."""
    B0 = sim.B.copy()
    E = sim.E.copy()
    Bz = np.zeros_like(B0)
    O.push_b(sim.g, E, Bz, 1.0)     # Bz = -curl^+ E
    return -Bz


def test_single_mode_scaled_by_laplacian_eigenvalue():
    c, sim = _sim()
    ny, nz = c.gdims[1], c.gdims[2]
    dy, dz = c.dx[1], c.dx[2]
    G0 = sim.gauss()
    my, mz = 3, 2
    ty, tz = 2 * math.pi * my / ny, 2 * math.pi * mz / nz
    j = np.arange(ny)[None, :]
    k = np.arange(nz)[:, None]
    nc = sim.nc
    E = sim.E.reshape(3, nz, ny)
    E[1] += 0.01 * np.cos(ty * (j + 0.5) + tz * k)     # E_y at (j + 1/2, k)
    E[2] += 0.02 * np.cos(ty * j + tz * (k + 0.5))     # E_z at (j, k + 1/2)
    F = sim.gauss() - G0
    assert np.abs(F).max() > 1e-3
    mode = np.sin(ty * j + tz * k).ravel()
    amp = F @ mode / (mode @ mode)
    assert np.abs(F - amp * mode).max() <= 1e-12 * np.abs(F).max()   # one mode
    d = 0.4 / (c.dt * (4 / dy ** 2 + 4 / dz ** 2))
    sim.marder(d, G0)
    F1 = sim.gauss() - G0
    lam = -(4 / dy ** 2) * math.sin(ty / 2) ** 2 - (4 / dz ** 2) * math.sin(tz / 2) ** 2
    assert np.abs(F1 - (1 + d * c.dt * lam) * F).max() <= 1e-11 * np.abs(F).max()


def test_transverse_part_unchanged():
    c, sim = _sim(seed=9)
    G0 = sim.gauss()
    rng = np.random.default_rng(5)
    sim.E += 0.01 * rng.standard_normal(sim.E.shape)
    curl0 = _curl_plus(sim)
    d = 0.5 / (c.dt * (4 / c.dx[1] ** 2 + 4 / c.dx[2] ** 2))
    sim.marder(d, G0, iters=3)
    assert np.abs(_curl_plus(sim) - curl0).max() <= 1e-12 * np.abs(curl0).max()


def test_no_op_without_drift():
    c, sim = _sim(seed=11)
    G0 = sim.gauss()
    E0 = sim.E.copy()
    sim.marder(1.0 / (c.dt * (4 / c.dx[1] ** 2 + 4 / c.dx[2] ** 2)), G0, iters=2)
    assert np.array_equal(sim.E, E0)


def test_planted_residual_decays():
    c, sim = _sim(seed=13)
    G0 = sim.gauss()
    rng = np.random.default_rng(6)
    sim.E += 0.01 * rng.standard_normal(sim.E.shape)
    d = 0.9 / (c.dt * (4 / c.dx[1] ** 2 + 4 / c.dx[2] ** 2))   # below the bound 2
    norms = []
    for _ in range(200):
        norms.append(np.linalg.norm(sim.gauss() - G0))
        sim.marder(d, G0)
    norms.append(np.linalg.norm(sim.gauss() - G0))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(norms, norms[1:]))
    # only the mean-free part can be removed; a periodic residual has zero mean
    assert norms[-1] < 0.1 * norms[0]
