"""Full-size checks in the launch configuration the benchmark times.

Workloads: the 1024 x 512 double Harris sheet (29.2 M particles, 2nd order,
32 x 32 patches) and the 256^3 Weibel setup (536.9 M particles, 1st order,
8^3 patches, random smooth fields so that the gather and the Boris rotation
act), default launch shapes.  After one push and the current fold:

  * a seeded sample of particles is recomputed one by one by the oracle from
    the same fields and compared per particle (|dxi| <= 1e-6 cells,
    |du| / max(|u|, v_th) <= 1e-5, the one-push parity tolerances);
  * the current is compared element by element on a few 4-cell blocks
    (4x4 in 2-d, 4x4x4 in 3-d): the oracle pushes every particle within
    three cells of a block (a particle's current stencil reaches at most two
    cells below and three above its cell), and J inside the block must
    match to 2e-5 of the block's largest |J| (the one-deposit parity
    tolerance);
  * the total current equals sum(q w v) of the pushed particles.

Properties that hold at any size are checked on the whole state after the
sort: the permutation is a bijection into non-decreasing keys, stable, with
the right cell offsets.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O
from paper_1310_7866_amd import cases
from tests.helpers import periodic_diff

pytestmark = pytest.mark.gpu


def _positions(c, cell, off):
    """Absolute positions (3, n) in cell units from geometric cells and offsets."""
    nx, ny, nz = c.gdims
    cell = cell.astype(np.int64)
    xi = np.zeros((3, cell.size))
    if c.dim == 2:
        xi[1] = cell % ny + off[0]
        xi[2] = cell // ny + off[1]
    else:
        xi[0] = cell % nx + off[0]
        xi[1] = (cell // nx) % ny + off[1]
        xi[2] = cell // (nx * ny) + off[2]
    return xi


def _oracle_push(c, sp, idx, E, B, J):
    """The oracle's particle loop on particles `idx` of species `sp` (initial
    state), depositing into J (float64, 3 * ncell); returns (xi, u)."""
    g = O.grid(c.dim, c.gdims, c.dx, c.dt, c.order)
    xi = np.ascontiguousarray(_positions(c, sp.cell[idx], sp.off[:, idx].astype(np.float64)))
    u = np.ascontiguousarray(sp.u[:, idx].astype(np.float64))
    O.lib().orc_push_particles(C.byref(g), idx.size, xi, u, E, B, J, sp.q, sp.m, sp.w)
    return xi, u


def _device_rows(sim, s, slots):
    """Keys, geometric cells, offsets and momenta of (run 0, species s) at
    buffer slots `slots` of the set the last push wrote."""
    import torch
    f, _ = sim.front()
    t = sim.parts[0][s][f]
    n = sim.cases[0].species[s].n
    D = sim.cases[0].dim
    k = torch.from_numpy(slots).to(t["cell"].device)
    key = t["cell"][:n][k]
    out = dict(cell=sim.keys_to_cells(0, key.contiguous()).cpu().numpy(),
               off=t["off"][:D * n].view(D, n)[:, k].cpu().numpy(),
               u=t["u"][:3 * n].view(3, n)[:, k].cpu().numpy())
    return out


def _slots_of_ids(sim, s, ids):
    """Buffer slots (in the set the last push wrote) of particle ids `ids`."""
    import torch
    f, _ = sim.front()
    t = sim.parts[0][s][f]
    n = sim.cases[0].species[s].n
    where = torch.empty(n, dtype=torch.int64, device=t["id"].device)
    where[t["id"][:n].long()] = torch.arange(n, dtype=torch.int64, device=where.device)
    return where[torch.from_numpy(ids).to(where.device)].cpu().numpy()


def _check_sampled_particles(c, sim, E, B, rng, per_species=4000):
    for s, sp in enumerate(c.species):
        sample = np.sort(rng.choice(sp.n, per_species, replace=False))
        xi, u = _oracle_push(c, sp, sample, E, B, np.zeros(3 * c.ncell))
        rows = _device_rows(sim, s, _slots_of_ids(sim, s, sample))
        gxi = _positions(c, rows["cell"], rows["off"].astype(np.float64))
        dpos = max(np.abs(periodic_diff(gxi[d], xi[d], c.gdims[d])).max() for d in c.active_dims())
        vth = float(np.std(sp.u))
        du = (np.linalg.norm(rows["u"] - u, axis=0) / np.maximum(np.linalg.norm(u, axis=0), vth)).max()
        print(f"species {s}: sampled |dxi| {dpos:.2e}, rel |du| {du:.2e}", flush=True)
        assert dpos <= 1e-6 and du <= 1e-5


def _block_cells(c, lo, width):
    """Geometric indices of the cells of the block [lo, lo + width) per
    active dimension (periodic), as a (D-dim) grid flattened."""
    dims = c.active_dims()
    axes = [(np.arange(lo[d], lo[d] + width) % c.gdims[d]) if d in dims else np.zeros(1, np.int64) for d in range(3)]
    i, j, k = np.meshgrid(axes[0], axes[1], axes[2], indexing="ij")
    nx, ny, _ = c.gdims
    return (i + nx * (j + ny * k)).ravel()


def _check_block_currents(c, sim, E, B, rng, n_blocks=4, width=4, margin=3):
    """J on n_blocks blocks of width^D cells, element by element."""
    _, _, Jg = sim.field_arrays(0)
    dims = c.active_dims()
    for b in range(n_blocks):
        lo = [int(rng.integers(0, c.gdims[d])) if d in dims else 0 for d in range(3)]
        inner = _block_cells(c, lo, width)
        outer = _block_cells(c, [x - margin if d in dims else 0 for d, x in enumerate(lo)], width + 2 * margin)
        J = np.zeros(3 * c.ncell)
        npart = 0
        for sp in c.species:
            # particles are emitted cell by cell in increasing geometric index
            starts = np.searchsorted(sp.cell, outer, side="left")
            ends = np.searchsorted(sp.cell, outer, side="right")
            idx = np.concatenate([np.arange(a, e) for a, e in zip(starts, ends)]).astype(np.int64)
            npart += idx.size
            _oracle_push(c, sp, idx, E, B, J)
        Jo = J.reshape(3, -1)[:, inner]
        Jb = Jg[:, inner].astype(np.float64)
        scale = np.abs(Jo).max()
        err = np.abs(Jb - Jo).max()
        print(f"block {b} at {lo}: {npart} particles, max|J| {scale:.3e}, max|dJ| {err:.3e}", flush=True)
        assert scale > 0
        assert err <= 2e-5 * scale


def _check_total_current(c, sim):
    import torch
    _, _, J = sim.field_arrays(0)
    f, _ = sim.front()
    jtot = np.zeros(3)
    for s, sp in enumerate(c.species):
        t = sim.parts[0][s][f]
        u = t["u"][:3 * sp.n].view(3, sp.n).double()
        gam = torch.sqrt(1.0 + (u * u).sum(0))
        jtot += sp.q * sp.w * (u / gam).sum(1).cpu().numpy()
    # the Esirkepov current of one particle sums over the grid to q w v
    Jsum = J.astype(np.float64).sum(1)
    print(f"total current {Jsum} vs {jtot}", flush=True)
    assert np.abs(Jsum - jtot).max() <= 1e-4 * np.abs(jtot).max() + 1e-3


def _check_sort(c, sim):
    """Permutation, order, stability and offsets on the whole state (device)."""
    import torch
    for s, sp in enumerate(c.species):
        f, _ = sim.front()
        n = sp.n
        keys = sim.parts[0][s][f]["cell"][:n].long()
        perm = sim.get_perm(0, s).long()
        ones = torch.bincount(perm, minlength=n)
        assert int(ones.min()) == 1 and int(ones.max()) == 1            # a bijection
        sk = keys[perm]
        assert bool((sk[1:] >= sk[:-1]).all())                          # sorted
        same = sk[1:] == sk[:-1]
        assert bool((perm[1:][same] > perm[:-1][same]).all())           # stable
        _, cst = sim.sort_view(0, s)
        counts = torch.bincount(keys, minlength=c.ncell).cpu().numpy()
        assert np.array_equal(cst, np.concatenate([[0], np.cumsum(counts)]))
        del keys, perm, ones, sk, same


def _full_size(c, seed):
    from paper_1310_7866_amd.psc import PscSim
    print(f"[gpu] {c.name} full size {c.gdims} n={c.n_particles}", flush=True)
    sim = PscSim(c)
    sim.push_fields(0)
    sim.push_particles()
    sim.deposit_current()
    assert sim.check() == 0
    # oracle fields after the B half step, in float64
    g = O.grid(c.dim, c.gdims, c.dx, c.dt, c.order)
    E = c.E.astype(np.float64).ravel().copy()
    B = c.B.astype(np.float64).ravel().copy()
    O.push_b(g, E, B, 0.5 * c.dt)
    rng = np.random.default_rng(seed)
    _check_sampled_particles(c, sim, E, B, rng)
    _check_block_currents(c, sim, E, B, rng)
    _check_total_current(c, sim)
    sim.push_fields(0)
    sim.push_fields(1)
    sim.sort()
    assert sim.check() == 0
    _check_sort(c, sim)
    sim.close()


def test_harris_full_size_sampled():
    _full_size(cases.harris2d(), 2024)


def test_weibel_full_size_sampled():
    c = cases.weibel3d()
    cases.random_fields(c, 0.05, 0.3, seed=2025)
    _full_size(c, 2026)
