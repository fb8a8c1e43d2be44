"""Edge cases of the GPU path against the oracle: an empty species, a grid
whose particles sit in a few cells (most patches and cells empty), particles
exactly on cell edges and at rest, and a cell with more particles than the
16-bit per-(cell, move) counters hold (refused with a device flag, never
mis-sorted).

Tolerances as in test_gpu_parity: one push <= 1e-6 cells / 1e-5 relative
momentum / 2e-5 of max|J|; three steps <= 1e-5 / 1e-4.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1310_7866_amd import cases
from tests.helpers import particle_errors

pytestmark = pytest.mark.gpu


def _sim(case):
    from paper_1310_7866_amd.psc import PscSim
    print(f"[gpu] edges {case.name} gdims={case.gdims} n={[s.n for s in case.species]}", flush=True)
    return PscSim(case)


def _check_against_oracle(c, steps=3):
    sim = _sim(c)
    ora = O.OracleSim(c)
    sim.push_fields(0)
    sim.push_particles()
    sim.deposit_current()
    assert sim.check() == 0
    ora.push_b_half()
    ora.push_particles()
    for s, sp in enumerate(c.species):
        if sp.n == 0:
            continue
        dpos, du = particle_errors(c, sim.front_buffer(0, s), ora, s, max(float(np.std(sp.u)), 1e-3))
        assert dpos <= 1e-6 and du <= 1e-5
    _, _, J = sim.field_arrays(0)
    jmax = max(np.abs(ora.J).max(), 1e-30)
    assert np.abs(J.ravel() - ora.J).max() <= 2e-5 * jmax
    sim2 = _sim(c)
    ora2 = O.OracleSim(c)
    for _ in range(steps):
        sim2.step(1)
        ora2.step(1)
    assert sim2.check() == 0
    for s, sp in enumerate(c.species):
        if sp.n == 0:
            continue
        dpos, du = particle_errors(c, sim2.particles(0, s), ora2, s, max(float(np.std(sp.u)), 1e-3))
        assert dpos <= 1e-5 and du <= 1e-4
    E, B, _ = sim2.field_arrays(0)
    assert np.abs(E.ravel() - ora2.E).max() <= 1e-4 * max(np.abs(ora2.E).max(), 1e-30)


@pytest.mark.parametrize("order", [1, 2])
def test_empty_species(order):
    c = cases.thermal2d(ny=20, nz=12, ppc=6, order=order, patch=8, seed=91)
    cases.random_fields(c, 0.05, 0.3, seed=92)
    sp = c.species[1]
    c.species[1] = cases.Species(sp.name, sp.q, sp.m, sp.w, sp.cell[:0].copy(), sp.off[:, :0].copy(),
                                 sp.u[:, :0].copy())
    _check_against_oracle(c)


@pytest.mark.parametrize("order", [1, 2])
def test_few_occupied_cells(order):
    """All particles in a 3x2 block of cells of a 32x24 grid (8x8 patches):
    most patches empty, the occupied cells dense and every wave one cell."""
    c = cases.thermal2d(ny=32, nz=24, ppc=4, order=order, patch=8, seed=93)
    cases.random_fields(c, 0.05, 0.3, seed=94)
    rng = np.random.default_rng(95)
    ny = c.gdims[1]
    for s in c.species:
        j = rng.integers(13, 16, s.n)
        k = rng.integers(9, 11, s.n)
        s.cell[:] = (j + ny * k).astype(np.int32)
    _check_against_oracle(c)


def test_particles_on_cell_edges_and_at_rest():
    """Offsets exactly 0 and the largest float below 1, momenta zero for a
    third of the particles: the edges of the weight formulas and moves of
    length zero."""
    c = cases.thermal2d(ny=16, nz=12, ppc=8, order=2, patch=8, seed=96)
    cases.random_fields(c, 0.05, 0.3, seed=97)
    below1 = np.nextafter(np.float32(1.0), np.float32(0.0))
    for s in c.species:
        s.off[0, 0::4] = 0.0
        s.off[1, 1::4] = 0.0
        s.off[0, 2::4] = below1
        s.off[1, 3::4] = below1
        s.u[:, 0::3] = 0.0
    _check_against_oracle(c, steps=2)


def test_overfull_cell_refused():
    """65,600 particles in one cell exceed the 16-bit per-(cell, move)
    counters: loading sets the overfull flag and psc_check reports it."""
    from paper_1310_7866_amd.psc import PscError
    c = cases.thermal2d(ny=8, nz=8, ppc=1, order=1, patch=8, seed=98)
    sp = c.species[0]
    n = 65600
    rng = np.random.default_rng(99)
    c.species[0] = cases.Species(sp.name, sp.q, sp.m, sp.w, np.full(n, 9, np.int32),
                                 rng.random((2, n)).astype(np.float32), np.zeros((3, n), np.float32))
    with pytest.raises(PscError):   # the constructor's final psc_check reports the flag
        sim = _sim(c)
        sim.check()


def test_load_sorted_restores_a_snapshot():
    """A snapshot in psc_get_particles order loaded back with psc_load_sorted
    (no sort) continues exactly as the run it was taken from."""
    c = cases.thermal2d(ny=24, nz=16, ppc=6, order=2, patch=8, seed=111)
    cases.random_fields(c, 0.05, 0.3, seed=112)
    sim = _sim(c)
    sim.step(2)
    snap = sim.snapshot()
    sim.step(2)
    ref = [sim.particles(0, s) for s in range(len(c.species))]
    E_ref = sim.field_arrays(0)[0]
    sim.restore(snap)
    sim.step(2)
    assert sim.check() == 0
    for s in range(len(c.species)):
        p = sim.particles(0, s)
        assert np.array_equal(p["key"], ref[s]["key"])
        assert np.array_equal(p["id"], ref[s]["id"])
        assert np.abs(p["u"] - ref[s]["u"]).max() <= 1e-6
    E = sim.field_arrays(0)[0]
    assert np.abs(E - E_ref).max() <= 1e-6 * np.abs(E_ref).max()
    sim.close()


def test_load_sorted_flags_unsorted_keys():
    """Keys in decreasing order are reported through the error word, not
    used: psc_load_sorted's offset pass checks every adjacent pair."""
    c = cases.thermal2d(ny=16, nz=16, ppc=2, order=1, patch=8, seed=113)
    sim = _sim(c)
    parts = [sim.device_particles(0, s) for s in range(len(c.species))]
    p = parts[0]
    sim.load_sorted(0, 0, p["key"].flip(0).contiguous(), p["off"], p["u"], p["id"])
    assert sim.error_word(clear=True) & 4   # PSC_DEV_KEY
    sim.close()
