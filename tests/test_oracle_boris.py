"""Pins of the oracle's relativistic Boris push (closed forms).

Boris' splitting (half E kick, rotation by B, half E kick; section "Time
integration of the quasi-particle equations of motion"):
  * pure magnetic field: |u| is invariant and each step rotates u about B by
    exactly theta = 2 arctan(|q| B dt / (2 m gamma)), clockwise for q > 0;
  * pure electric field: u gains exactly q E dt / m;
  * crossed fields: the guiding centre drifts with E x B / B^2.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O


@pytest.mark.parametrize("q,m,u0", [(1.0, 1.0, 0.1), (-1.0, 1.0, 0.3), (1.0, 25.0, 2.0), (-1.0, 1.0, 10.0)])
def test_gyration_angle_and_speed(q, m, u0):
    dt, Bz = 0.1, 0.7
    u = np.array([u0, 0.0, 0.37 * u0])
    gam = math.sqrt(1 + u @ u)
    theta = 2 * math.atan(abs(q) * Bz * dt / (2 * m * gam))
    for _ in range(50):
        un = O.boris(u, [0, 0, 0], [0, 0, Bz], q * dt / (2 * m))
        assert abs(np.linalg.norm(un) - np.linalg.norm(u)) < 1e-14 * np.linalg.norm(u)
        assert abs(un[2] - u[2]) < 1e-15 * abs(u0)
        ang = math.atan2(u[0] * un[1] - u[1] * un[0], u[0] * un[0] + u[1] * un[1])
        # q > 0 in B along +z turns clockwise (negative angle)
        assert abs(ang + math.copysign(theta, q)) < 1e-13
        u = un


def test_pure_electric_kick():
    rng = np.random.default_rng(3)
    for _ in range(20):
        u = rng.normal(size=3)
        E = rng.normal(size=3)
        q, m, dt = rng.choice([-1.0, 1.0]), rng.uniform(1, 30), 0.07
        un = O.boris(u, E, [0, 0, 0], q * dt / (2 * m))
        assert np.allclose(un, u + q * E * dt / m, rtol=0, atol=1e-15)


def test_exb_drift():
    # E = 0.01 B: drift speed 0.01 c along E x B = +x for E = E0 y, B = B0 z
    q, m, dt = -1.0, 1.0, 0.05
    B0, E0 = 1.0, 0.01
    u = np.zeros(3)
    x = np.zeros(3)
    period = 2 * math.pi * m / (abs(q) * B0)
    nsteps = int(round(40 * period / dt))
    xs = []
    for _ in range(nsteps):
        u = O.boris(u, [0, E0, 0], [0, 0, B0], q * dt / (2 * m))
        gam = math.sqrt(1 + u @ u)
        x = x + dt * u / gam
        xs.append(x.copy())
    xs = np.array(xs)
    t = dt * np.arange(1, nsteps + 1)
    slope = np.polyfit(t, xs[:, 0], 1)[0]
    assert abs(slope - E0 / B0) < 2e-3 * E0 / B0
    assert abs(np.polyfit(t, xs[:, 1], 1)[0]) < 1e-3 * E0 / B0
