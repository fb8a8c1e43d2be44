"""Seeded synthetic workloads for the particle hot path.

Pure input generation: the positions, momenta and initial fields of the
plasma setups the particle-in-cell method is exercised on.  Nothing here
computes a step of the method (no shape weights, no gather, no particle
push, no current deposit, no field update, no sort).  Both the GPU binding
and the double-precision oracle used by the tests take their inputs from
these arrays, so both sides see bit-identical starting states.

Normalisation (the paper writes Maxwell's equations in SI form and fixes no
units): c = eps0 = 1, electron charge and mass 1, reference density 1, so
time is in 1/omega_pe and length in electron skin depths d_e.  Momenta are
u = gamma v / c.  A species of density-weight w contributes q*w to the
charge density per particle, so ``ppc`` particles of weight 1/ppc represent
density 1.

Layout of every array handed out:
  * grid: cells (nx, ny, nz); a 2-d case is the (y, z) plane with nx == 1.
  * fields: float32, shape (3, ncell), component-major, cell index
    ``i + nx*(j + ny*k)`` (x fastest).  Staggering follows the Yee cell:
    E_x at (i+1/2, j, k), E_y at (i, j+1/2, k), E_z at (i, j, k+1/2),
    B_x at (i, j+1/2, k+1/2), B_y at (i+1/2, j, k+1/2),
    B_z at (i+1/2, j+1/2, k); each stored at its lower integer index.
  * particles: ``cell`` int32 geometric cell index (same formula),
    ``off`` float32 (D, n) in-cell offsets in [0, 1) for the active
    dimensions ((y, z) in 2-d, (x, y, z) in 3-d), ``u`` float32 (3, n).
    Particles are emitted cell by cell in increasing geometric index.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

ONE_BELOW = np.float32(np.nextafter(np.float32(1.0), np.float32(0.0)))


@dataclasses.dataclass
class Species:
    name: str
    q: float
    m: float
    w: float
    cell: np.ndarray          # int32 (n,)
    off: np.ndarray           # float32 (D, n)
    u: np.ndarray             # float32 (3, n)

    @property
    def n(self) -> int:
        return int(self.cell.shape[0])


@dataclasses.dataclass
class Case:
    name: str
    dim: int                  # 2: (y,z) plane, 3: (x,y,z)
    gdims: tuple              # cells (nx, ny, nz)
    dx: tuple                 # cell sizes (dx, dy, dz)
    dt: float
    order: int                # 1 or 2 (b1 or b2 interpolation weights)
    patch: tuple              # patch size in cells (px, py, pz)
    steps: int
    seed: int
    species: List[Species]
    E: np.ndarray             # float32 (3, ncell)
    B: np.ndarray             # float32 (3, ncell)
    deposit: str = "esirkepov"   # or "vb": Villasenor-Buneman (1st order only)

    @property
    def ncell(self) -> int:
        return int(self.gdims[0] * self.gdims[1] * self.gdims[2])

    @property
    def n_particles(self) -> int:
        return sum(s.n for s in self.species)

    def active_dims(self) -> Sequence[int]:
        return (1, 2) if self.dim == 2 else (0, 1, 2)


def half_cfl_dt(dim: int, dx: Sequence[float]) -> float:
    """dt = 0.5 * CFL limit of the Yee scheme with c = 1."""
    active = (1, 2) if dim == 2 else (0, 1, 2)
    return 0.5 / math.sqrt(sum(1.0 / dx[d] ** 2 for d in active))


def _offsets(rng: np.random.Generator, ndim: int, n: int) -> np.ndarray:
    """Uniform in-cell offsets in [0, 1), rounded to float32 strictly below 1."""
    off = rng.random((ndim, n)).astype(np.float32)
    off[off >= np.float32(1.0)] = ONE_BELOW
    return off


def _maxwellian(rng: np.random.Generator, n: int, vth: Sequence[float],
                drift: Sequence[float]) -> np.ndarray:
    u = np.empty((3, n), dtype=np.float32)
    for c in range(3):
        u[c] = (drift[c] + vth[c] * rng.standard_normal(n)).astype(np.float32)
    return u


def _cells_from_counts(counts: np.ndarray) -> np.ndarray:
    """Repeat each geometric cell index by its particle count."""
    return np.repeat(np.arange(counts.size, dtype=np.int32), counts.ravel())


def _stochastic_round(rng: np.random.Generator, x: np.ndarray) -> np.ndarray:
    base = np.floor(x)
    return (base + (rng.random(x.shape) < (x - base))).astype(np.int64)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def thermal2d(ny: int = 64, nz: int = 64, dx: float = 0.1, ppc: int = 16,
              vth_e: float = 0.1, vth_i: float = 0.02, mi: float = 25.0,
              order: int = 1, patch: int = 32, steps: int = 100,
              seed: int = 1310) -> Case:
    """2-d periodic thermal electron-ion plasma.

    ``ppc`` electron-ion pairs per cell, each pair co-located (uniform in
    the cell), so the charge density vanishes identically and E = B = 0
    satisfies Gauss's law at t = 1/2.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ncell = ny * nz
    counts = np.full(ncell, ppc, dtype=np.int64)
    cell = _cells_from_counts(counts)
    n = cell.size
    off = _offsets(rng, 2, n)
    ue = _maxwellian(rng, n, (vth_e,) * 3, (0.0, 0.0, 0.0))
    ui = _maxwellian(rng, n, (vth_i,) * 3, (0.0, 0.0, 0.0))
    w = 1.0 / ppc
    sp = [Species("electron", -1.0, 1.0, w, cell, off, ue),
          Species("ion", 1.0, mi, w, cell.copy(), off.copy(), ui)]
    dxs = (1.0, dx, dx)
    E = np.zeros((3, ncell), np.float32)
    B = np.zeros((3, ncell), np.float32)
    return Case("thermal2d", 2, (1, ny, nz), dxs, half_cfl_dt(2, dxs), order,
                (1, patch, patch), steps, seed, sp, E, B)


def harris2d(ny: int = 1024, nz: int = 512, dx: float = 0.25, ppc: float = 100.0,
             mi: float = 25.0, ti_te: float = 5.0, nb: float = 0.2,
             half_thickness_di: float = 0.5, b0: float = 0.5, pert: float = 0.1,
             order: int = 2, patch: int = 32, steps: int = 1000,
             seed: int = 7866) -> Case:
    """Doubly periodic double Harris current sheet for reconnection.

    Sheets at z = Lz/4 and 3Lz/4 with
      B_y(z) = B0 [tanh((z - Lz/4)/L) - tanh((z - 3Lz/4)/L) - 1],
      n(z) = sech^2((z - Lz/4)/L) + sech^2((z - 3Lz/4)/L) + nb.
    Pressure balance n0 (Te + Ti) = B0^2/2 with Ti/Te = ti_te; the sheet
    populations drift along x with Vi = -(B0/L) Ti/(Te+Ti) and
    Ve = +(B0/L) Te/(Te+Ti) on the first sheet (signs flip on the second),
    so that J_x = (curl B)_x.  The background is at rest with the same
    temperatures.  Electron-ion pairs are co-located, so rho = 0 and E = 0.
    A flux perturbation dA_x = pert*B0*d_i*cos(2 pi y/Ly) sin(2 pi z/Lz) is
    added; its field is the exact face average of curl(dA_x x), i.e. the
    difference of A_x between the two nodes bounding each face.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ncell = ny * nz
    di = math.sqrt(mi)
    L = half_thickness_di * di
    Ly, Lz = ny * dx, nz * dx
    T = b0 * b0 / 2.0
    te = T / (1.0 + ti_te)
    ti = T - te
    vth_e = math.sqrt(te)
    vth_i = math.sqrt(ti / mi)
    vdi = (b0 / L) * ti / T
    vde = (b0 / L) * te / T

    zc = (np.arange(nz) + 0.5) * dx
    s1 = 1.0 / np.cosh((zc - Lz / 4) / L) ** 2
    s2 = 1.0 / np.cosh((zc - 3 * Lz / 4) / L) ** 2
    n1 = _stochastic_round(rng, np.broadcast_to(ppc * s1[:, None], (nz, ny)).copy())
    n2 = _stochastic_round(rng, np.broadcast_to(ppc * s2[:, None], (nz, ny)).copy())
    nbg = _stochastic_round(rng, np.full((nz, ny), ppc * nb))
    # per cell: [sheet1 | sheet2 | background], cells in geometric order
    counts = (n1 + n2 + nbg).ravel()
    cell = _cells_from_counts(counts)
    n = cell.size
    # population tag per particle: 0 sheet1, 1 sheet2, 2 background
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    rank = np.arange(n) - np.repeat(starts, counts)
    c1 = np.repeat(n1.ravel(), counts)
    c2 = np.repeat(n2.ravel(), counts)
    pop = np.where(rank < c1, 0, np.where(rank < c1 + c2, 1, 2))
    off = _offsets(rng, 2, n)
    sign = np.where(pop == 0, 1.0, np.where(pop == 1, -1.0, 0.0))
    ue = _maxwellian(rng, n, (vth_e,) * 3, (0.0, 0.0, 0.0))
    ui = _maxwellian(rng, n, (vth_i,) * 3, (0.0, 0.0, 0.0))
    ue[0] = (ue[0].astype(np.float64) + vde * sign).astype(np.float32)
    ui[0] = (ui[0].astype(np.float64) - vdi * sign).astype(np.float32)
    w = 1.0 / ppc
    sp = [Species("electron", -1.0, 1.0, w, cell, off, ue),
          Species("ion", 1.0, mi, w, cell.copy(), off.copy(), ui)]

    E = np.zeros((3, ncell), np.float32)
    B = np.zeros((3, nz, ny), np.float64)
    zh = (np.arange(nz) + 0.5) * dx       # B_y sits at (node y, half z)
    by = b0 * (np.tanh((zh - Lz / 4) / L) - np.tanh((zh - 3 * Lz / 4) / L) - 1.0)
    B[1] += by[:, None]
    # perturbation potential at nodes (A_x location in the plane)
    yn = np.arange(ny) * dx
    zn = np.arange(nz) * dx
    A = pert * b0 * di * np.cos(2 * np.pi * yn[None, :] / Ly) * np.sin(2 * np.pi * zn[:, None] / Lz)
    # face averages of (dA/dz, -dA/dy): endpoint differences along each face
    B[1] += (np.roll(A, -1, axis=0) - A) / dx
    B[2] -= (np.roll(A, -1, axis=1) - A) / dx
    dxs = (1.0, dx, dx)
    return Case("harris2d", 2, (1, ny, nz), dxs, half_cfl_dt(2, dxs), order,
                (1, patch, patch), steps, seed, sp, E,
                B.reshape(3, ncell).astype(np.float32))


def weibel3d(n: int = 256, dx: float = 0.1, ppc: int = 32, beam_v: float = 0.3,
             vth: float = 0.05, order: int = 1, patch: int = 8, steps: int = 200,
             seed: int = 2013, nxyz: Optional[Sequence[int]] = None) -> Case:
    """3-d periodic counter-streaming electron beams (Weibel instability).

    ``ppc`` electrons per cell, half drifting along +z and half along -z with
    velocity ``beam_v`` (u_d = beam_v / sqrt(1 - beam_v^2)) plus a thermal
    spread ``vth``.  Ions are immobile and are not stored; they sit at the
    electrons' initial positions, so the initial charge density vanishes and
    E = B = 0 satisfies Gauss's law at t = 1/2.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = (n, n, n) if nxyz is None else tuple(nxyz)
    ncell = nx * ny * nz
    ud = beam_v / math.sqrt(1.0 - beam_v * beam_v)
    counts = np.full(ncell, ppc, dtype=np.int64)
    cell = _cells_from_counts(counts)
    npart = cell.size
    off = _offsets(rng, 3, npart)
    u = np.empty((3, npart), np.float32)
    beam = np.where((np.arange(npart) % ppc) < ppc // 2, 1.0, -1.0)
    for c in range(3):
        u[c] = (vth * rng.standard_normal(npart) + (ud * beam if c == 2 else 0.0)).astype(np.float32)
    sp = [Species("electron", -1.0, 1.0, 1.0 / ppc, cell, off, u)]
    dxs = (dx, dx, dx)
    E = np.zeros((3, ncell), np.float32)
    B = np.zeros((3, ncell), np.float32)
    return Case("weibel3d", 3, (nx, ny, nz), dxs, half_cfl_dt(3, dxs), order,
                (patch, patch, patch), steps, seed, sp, E, B)


def twostream2d(ny: int, nz: int, ppc: int, dx: float = 0.1, beam_v: float = 0.2,
                vth: float = 0.02, order: int = 1, patch: int = 32, steps: int = 200,
                seed: int = 4064) -> Case:
    """2-d periodic electron two-stream run: beams at +-beam_v along y.

    ``ppc`` electrons per cell split evenly between the beams; ions are
    immobile, unstored and co-located with the initial electrons.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ncell = ny * nz
    counts = np.full(ncell, ppc, dtype=np.int64)
    cell = _cells_from_counts(counts)
    npart = cell.size
    off = _offsets(rng, 2, npart)
    ud = beam_v / math.sqrt(1.0 - beam_v * beam_v)
    beam = np.where((np.arange(npart) % ppc) < ppc // 2, 1.0, -1.0)
    u = np.empty((3, npart), np.float32)
    for c in range(3):
        u[c] = (vth * rng.standard_normal(npart) + (ud * beam if c == 1 else 0.0)).astype(np.float32)
    sp = [Species("electron", -1.0, 1.0, 1.0 / ppc, cell, off, u)]
    dxs = (1.0, dx, dx)
    E = np.zeros((3, ncell), np.float32)
    B = np.zeros((3, ncell), np.float32)
    return Case("twostream2d", 2, (1, ny, nz), dxs, half_cfl_dt(2, dxs), order,
                (1, min(patch, ny), min(patch, nz)), steps, seed, sp, E, B)


def twostream_batch(n_runs: int = 64, seed: int = 4064, steps: int = 200,
                    patch: int = 32, max_cells: Optional[int] = None) -> List[Case]:
    """Many independent two-stream runs of uneven size.

    Per run: ny log-uniform in [32, 512] and nz log-uniform in [32, 256],
    both rounded to multiples of 8 (so a 32x32 patch grid has ragged edge
    patches); particles per cell log-uniform in [8, 128], rounded to even.
    ``max_cells`` optionally rescales oversized draws (used for reduced
    test variants).
    """
    root = np.random.SeedSequence(seed)
    children = root.spawn(n_runs + 1)
    draw = np.random.Generator(np.random.PCG64(children[0]))
    cases = []
    for r in range(n_runs):
        ny = int(round(math.exp(draw.uniform(math.log(32), math.log(512))) / 8.0)) * 8
        nz = int(round(math.exp(draw.uniform(math.log(32), math.log(256))) / 8.0)) * 8
        ppc = int(round(math.exp(draw.uniform(math.log(8), math.log(128))) / 2.0)) * 2
        ny, nz, ppc = max(ny, 8), max(nz, 8), max(ppc, 2)
        if max_cells is not None:
            while ny * nz > max_cells:
                ny = max(8, (ny // 2) // 8 * 8)
                nz = max(8, (nz // 2) // 8 * 8)
        sub = int(children[r + 1].generate_state(1)[0])
        cases.append(twostream2d(ny, nz, ppc, patch=patch, steps=steps, seed=sub))
    return cases


def plasma_oscillation2d(ny: int = 8, nz: int = 8, dx: float = 0.1, side: int = 4,
                         uz: float = 1e-3, order: int = 1, patch: int = 8) -> Case:
    """Cold k = 0 electron oscillation with a quiet-start lattice.

    ``side`` x ``side`` electrons per cell at offsets (a + 1/2)/side, all
    with the same momentum u_z; immobile neutralising ions (unstored).
    """
    ncell = ny * nz
    per = side * side
    counts = np.full(ncell, per, dtype=np.int64)
    cell = _cells_from_counts(counts)
    n = cell.size
    a = (np.arange(per) % side + 0.5) / side
    b = (np.arange(per) // side + 0.5) / side
    off = np.empty((2, n), np.float32)
    off[0] = np.tile(a, ncell).astype(np.float32)
    off[1] = np.tile(b, ncell).astype(np.float32)
    u = np.zeros((3, n), np.float32)
    u[2] = np.float32(uz)
    sp = [Species("electron", -1.0, 1.0, 1.0 / per, cell, off, u)]
    dxs = (1.0, dx, dx)
    return Case("plasma_osc2d", 2, (1, ny, nz), dxs, half_cfl_dt(2, dxs), order,
                (1, patch, patch), 0, 0, sp,
                np.zeros((3, ncell), np.float32), np.zeros((3, ncell), np.float32))


def random_fields(case: Case, scale_e: float, scale_b: float, seed: int) -> None:
    """Overwrite E and B with smooth random periodic fields (test inputs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = case.gdims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for arr, scale in ((case.E, scale_e), (case.B, scale_b)):
        for c in range(3):
            f = np.zeros((nz, ny, nx))
            for _ in range(3):
                kx = rng.integers(0, 3) if nx > 1 else 0
                ky = rng.integers(0, 3)
                kz = rng.integers(0, 3)
                ph = rng.uniform(0, 2 * np.pi)
                amp = rng.uniform(0.3, 1.0)
                f += amp * np.cos(2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + ph)
            arr[c] = (scale * f.ravel()).astype(np.float32)


def thin(case: Case, keep_every: int) -> Case:
    """Return a copy keeping every ``keep_every``-th particle of each species."""
    sp = [Species(s.name, s.q, s.m, s.w, s.cell[::keep_every].copy(),
                  s.off[:, ::keep_every].copy(), s.u[:, ::keep_every].copy())
          for s in case.species]
    return dataclasses.replace(case, species=sp)
