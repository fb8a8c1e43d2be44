"""Full-size check in the launch configuration the benchmark times.

The 1024 x 512 double Harris sheet (29.2 M particles, 2nd order, 32 x 32
patches, default chunking) is advanced by the GPU; a seeded sample of
particles is recomputed one by one by the oracle from the same fields and
compared per particle (|dxi| <= 1e-6 cells, |du|/max(|u|, v_th) <= 1e-5).
Properties that hold at any size are checked on the whole state: the sort
is a permutation into non-decreasing keys with the right cell offsets, and
the total current equals sum(q w v) of the pushed particles.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O
from paper_1310_7866_amd import cases
from tests.helpers import periodic_diff

pytestmark = pytest.mark.gpu


def test_harris_full_size_sampled():
    from paper_1310_7866_amd.psc import PscSim
    c = cases.harris2d()
    print(f"[gpu] harris2d full size n={c.n_particles}", flush=True)
    sim = PscSim(c)
    sim.push_fields(0)
    sim.push_particles()
    sim.deposit_current()
    assert sim.check() == 0
    # oracle: fields after the B half step, in float64
    g = O.grid(c.dim, c.gdims, c.dx, c.dt, c.order)
    E = c.E.astype(np.float64).ravel().copy()
    B = c.B.astype(np.float64).ravel().copy()
    O.push_b(g, E, B, 0.5 * c.dt)
    rng = np.random.default_rng(2024)
    _, _, J = sim.field_arrays(0)
    jtot = np.zeros(3)
    for s, sp in enumerate(c.species):
        out = sim.front_buffer(0, s)
        ids = out["id"]
        sample = rng.choice(sp.n, 4000, replace=False)
        where = np.empty(sp.n, np.int64)
        where[ids] = np.arange(sp.n)
        nx, ny, nz = c.gdims
        cell = sp.cell[sample].astype(np.int64)
        xi = np.zeros((3, sample.size))
        xi[1] = cell % ny + sp.off[0, sample]
        xi[2] = cell // ny + sp.off[1, sample]
        u = sp.u[:, sample].astype(np.float64).copy()
        Jdummy = np.zeros(3 * c.ncell)
        xi = np.ascontiguousarray(xi)
        u = np.ascontiguousarray(u)
        O.lib().orc_push_particles(C.byref(g), sample.size, xi, u, E, B, Jdummy, sp.q, sp.m, sp.w)
        k = where[sample]
        gc = out["cell"][k].astype(np.int64)
        gxi = np.zeros((3, sample.size))
        gxi[1] = gc % ny + out["off"][0, k]
        gxi[2] = gc // ny + out["off"][1, k]
        dpos = max(np.abs(periodic_diff(gxi[1], xi[1], ny)).max(), np.abs(periodic_diff(gxi[2], xi[2], nz)).max())
        vth = float(np.std(sp.u))
        du = (np.linalg.norm(out["u"][:, k] - u, axis=0) / np.maximum(np.linalg.norm(u, axis=0), vth)).max()
        print(f"species {s}: sampled |dxi| {dpos:.2e}, rel |du| {du:.2e}")
        assert dpos <= 1e-6 and du <= 1e-5
        # total current of the species: q w sum(v) * ... (first-moment identity)
        uu = out["u"].astype(np.float64)
        gam = np.sqrt(1 + (uu ** 2).sum(0))
        jtot += sp.q * sp.w * (uu / gam).sum(1)
    # J summed over the grid equals sum q w v (in-plane via dxi*dx/dt, which is v)
    Jsum = J.astype(np.float64).sum(1)
    print(f"total current {Jsum} vs {jtot}")
    assert np.abs(Jsum - jtot).max() <= 1e-4 * np.abs(jtot).max() + 1e-3
    # sort properties on the whole state
    sim.push_fields(0)
    sim.push_fields(1)
    sim.sort()
    assert sim.check() == 0
    for s in range(2):
        f, _ = sim.front()
        n = c.species[s].n
        keys = sim.parts[0][s][f]["cell"][:n].cpu().numpy()
        perm, cst = sim.sort_view(0, s)
        assert np.array_equal(np.sort(perm), np.arange(n))
        sk = keys[perm]
        assert np.all(np.diff(sk) >= 0)
        counts = np.bincount(keys, minlength=c.ncell)
        assert np.array_equal(cst, np.concatenate([[0], np.cumsum(counts)]))
        # stability: within equal keys the original positions increase
        same = np.diff(sk) == 0
        assert np.all(np.diff(perm)[same] > 0)
