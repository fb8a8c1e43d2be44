"""GPU parity: each C-ABI call against the double-precision oracle.

Tolerances (float32 kernels vs float64 oracle on identical float32 inputs):
  * per particle after one push: |dxi| <= 1e-6 cells and
    |du| / max(|u|, v_th) <= 1e-5;
  * fields after one update: |dF| <= 1e-6 * max|F| (one float32 stencil
    evaluation, a handful of roundings of O(max|F|) values);
  * current after one deposit: |dJ| <= 2e-5 * max|J| (sums of up to a few
    hundred float32 contributions of O(q w dx/dt) each);
  * sort permutation: bit-exact against the oracle's stable sort of the same
    keys.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1310_7866_amd import cases
from tests.helpers import by_id, gpu_positions, particle_errors, periodic_diff

pytestmark = pytest.mark.gpu


def _sim(case, **kw):
    from paper_1310_7866_amd.psc import PscSim
    print(f"[gpu] {case.name} dim={case.dim} order={case.order} gdims={case.gdims} patch={case.patch} "
          f"n={case.n_particles}", flush=True)
    return PscSim(case, **kw)


def _small_2d(order, seed=5, ny=20, nz=12, patch=8, ppc=6):
    c = cases.thermal2d(ny=ny, nz=nz, ppc=ppc, order=order, patch=patch, seed=seed)
    # separate the species so the charge density is non-trivial
    c.species[1].off = np.random.default_rng(seed + 1000).random(c.species[1].off.shape).astype(np.float32)
    cases.random_fields(c, 0.05, 0.3, seed=seed + 1)
    return c


def _small_3d(order, seed=8, nxyz=(10, 9, 7), patch=4, ppc=4):
    c = cases.weibel3d(ppc=ppc, order=order, patch=patch, seed=seed, nxyz=nxyz)
    cases.random_fields(c, 0.05, 0.3, seed=seed + 1)
    return c


CASES = [("2d", 1), ("2d", 2), ("3d", 1), ("3d", 2)]


def _make(kind, order):
    return _small_2d(order) if kind == "2d" else _small_3d(order)


@pytest.mark.parametrize("kind,order", CASES)
def test_fields_match_oracle(kind, order):
    c = _make(kind, order)
    sim = _sim(c)
    ora = O.OracleSim(c)
    sim.push_fields(0)
    ora.push_b_half()
    E, B, J = sim.field_arrays(0)
    assert np.abs(B.ravel() - ora.B).max() <= 1e-6 * np.abs(ora.B).max()
    sim.push_fields(1)
    ora.J[:] = 0
    ora.push_e_full()
    E, B, J = sim.field_arrays(0)
    assert np.abs(E.ravel() - ora.E).max() <= 1e-6 * max(np.abs(ora.E).max(), 1e-30)


@pytest.mark.parametrize("tile_fold", [False, True])
@pytest.mark.parametrize("kind,order", CASES)
def test_push_and_deposit_match_oracle(kind, order, tile_fold):
    # tile_fold: the current through per-patch tiles and the fold pass
    # instead of the particle kernel adding it into J
    c = _make(kind, order)
    sim = _sim(c, tile_fold=tile_fold)
    ora = O.OracleSim(c)
    sim.push_fields(0)
    sim.push_particles()
    sim.deposit_current()
    assert sim.check() == 0
    ora.push_b_half()
    ora.push_particles()
    for s, sp in enumerate(c.species):
        vth = float(np.std(sp.u))
        dpos, du = particle_errors(c, sim.front_buffer(0, s), ora, s, vth)
        print(f"species {s}: max |dxi| = {dpos:.3e} cells, max rel |du| = {du:.3e}")
        assert dpos <= 1e-6
        assert du <= 1e-5
    _, _, J = sim.field_arrays(0)
    err = np.abs(J.ravel() - ora.J).max()
    print(f"max |dJ| = {err:.3e}, max |J| = {np.abs(ora.J).max():.3e}")
    assert err <= 2e-5 * np.abs(ora.J).max()


@pytest.mark.parametrize("kind,order", CASES)
def test_sort_matches_stable_sort(kind, order):
    c = _make(kind, order)
    sim = _sim(c)
    for step in range(3):
        sim.step(1) if step else None
        sim.push_fields(0)
        sim.push_particles()
        sim.push_fields(0)
        sim.deposit_current()
        sim.push_fields(1)
        for s in range(len(c.species)):
            keys = sim.front_buffer(0, s)["key"]
        word_push = sim.error_word()
        sim.sort()
        word = sim.error_word()
        print(f"step {step}: error word after push {word_push:#x}, after sort {word:#x}", flush=True)
        assert word == 0
        for s in range(len(c.species)):
            f, _ = sim.front()
            n = c.species[s].n
            keys = sim.parts[0][s][f]["cell"][:n].cpu().numpy()
            perm, cst = sim.sort_view(0, s)
            want = O.stable_sort(keys, c.ncell)
            assert np.array_equal(perm, want)
            counts = np.bincount(keys, minlength=c.ncell)
            assert np.array_equal(cst, np.concatenate([[0], np.cumsum(counts)]))


# Sort workloads of different densities for the scatter pass (waves of 64
# cells in 3-d, 32 in 2-d, each walking its particles 64 at a time): groups
# spanning many cells, about one cell, a fraction of a cell, and one cell
# holding hundreds of particles.
SORT_LOADS = [("3d", 3, 0), ("3d", 20, 0), ("3d", 40, 0), ("3d", 45, 0), ("3d", 4, 400), ("2d", 40, 0),
              ("2d", 90, 0), ("2d", 5, 300)]


@pytest.mark.parametrize("kind,ppc,dense", SORT_LOADS)
def test_sort_scatter_paths_match_stable_sort(kind, ppc, dense):
    if kind == "3d":
        c = _small_3d(1, seed=91, nxyz=(8, 8, 12), patch=4, ppc=ppc)
    else:
        c = _small_2d(1, seed=92, ny=64, nz=16, patch=16, ppc=ppc)
    if dense:
        # `dense` particles of species 0 moved into one cell
        sp = c.species[0]
        sp.cell[:dense] = sp.cell[0]
    sim = _sim(c)
    for step in range(2):
        sim.push_fields(0)
        sim.push_particles()
        sim.push_fields(0)
        sim.deposit_current()
        sim.push_fields(1)
        sim.sort()
        assert sim.error_word() == 0
        for s in range(len(c.species)):
            f, _ = sim.front()
            n = c.species[s].n
            keys = sim.parts[0][s][f]["cell"][:n].cpu().numpy()
            perm, cst = sim.sort_view(0, s)
            assert np.array_equal(perm, O.stable_sort(keys, c.ncell)), (step, s)
            counts = np.bincount(keys, minlength=c.ncell)
            assert np.array_equal(cst, np.concatenate([[0], np.cumsum(counts)]))
            if dense and s == 0:
                assert counts.max() >= dense // 2   # the dense cell is still dense


@pytest.mark.parametrize("kind,order", CASES)
def test_steps_match_oracle(kind, order):
    c = _make(kind, order)
    sim = _sim(c)
    ora = O.OracleSim(c)
    for _ in range(5):
        sim.step(1)
        ora.step(1)
    assert sim.check() == 0
    for s, sp in enumerate(c.species):
        vth = float(np.std(sp.u))
        dpos, du = particle_errors(c, sim.particles(0, s), ora, s, vth)
        print(f"5 steps, species {s}: |dxi| {dpos:.3e}, rel |du| {du:.3e}")
        assert dpos <= 1e-5
        assert du <= 1e-4
    E, B, J = sim.field_arrays(0)
    assert np.abs(E.ravel() - ora.E).max() <= 1e-4 * np.abs(ora.E).max()
    assert np.abs(B.ravel() - ora.B).max() <= 1e-4 * np.abs(ora.B).max()


@pytest.mark.parametrize("order", [1, 2])
def test_steps_match_oracle_3d_patch_fold(order):
    # every patch 4 wide (at least the current halo at both orders): with
    # per-patch current tiles the 3-d run folds them by patch, which the
    # default 3-d case (with narrower last patches) does not reach
    c = _small_3d(order, seed=18, nxyz=(8, 8, 12), patch=4, ppc=3)
    sim = _sim(c, tile_fold=True)
    ora = O.OracleSim(c)
    for _ in range(3):
        sim.step(1)
        ora.step(1)
    assert sim.check() == 0
    for s, sp in enumerate(c.species):
        dpos, du = particle_errors(c, sim.particles(0, s), ora, s, float(np.std(sp.u)))
        assert dpos <= 1e-5 and du <= 1e-4, (s, dpos, du)
    E, B, J = sim.field_arrays(0)
    assert np.abs(J.ravel() - ora.J).max() <= 1e-4 * np.abs(ora.J).max()
    assert np.abs(E.ravel() - ora.E).max() <= 1e-4 * np.abs(ora.E).max()
    assert np.abs(B.ravel() - ora.B).max() <= 1e-4 * np.abs(ora.B).max()


@pytest.mark.parametrize("use_graph", [False, True])
def test_graph_replay_matches_eager(use_graph):
    c = _small_2d(2, seed=21)
    a = _sim(c)
    b = _sim(c)
    for k in range(4):
        a.step(1, use_graph=False)
        b.step(1, use_graph=use_graph)
        assert a.check() == 0 and b.check() == 0
        pa, pb = a.particles(0, 0), b.particles(0, 0)
        assert np.array_equal(pa["key"], pb["key"])
        assert np.abs(pa["u"] - pb["u"]).max() <= 1e-5
    Ea = a.field_arrays(0)[0]
    Eb = b.field_arrays(0)[0]
    assert np.abs(Ea - Eb).max() <= 1e-5 * np.abs(Ea).max()


@pytest.mark.parametrize("use_graph", [False, True])
def test_step_matches_separate_calls(use_graph):
    # psc_step (eager or replayed from a graph) against the separate entry
    # points called in the order of fig. psc_new: the same state (keys
    # exactly; values to the summation-order tolerance of the float tile
    # atomics)
    from paper_1310_7866_amd.psc import B_HALF, E_FULL
    c = _small_2d(2, seed=23, ny=40, nz=24)
    a = _sim(c)
    b = _sim(c)
    for k in range(4):
        a.step(1, use_graph=use_graph)
        b.push_fields(B_HALF)
        b.push_particles()
        b.push_fields(B_HALF)
        b.deposit_current()
        b.push_fields(E_FULL)
        b.sort()
        assert a.check() == 0 and b.check() == 0
        for s in range(len(c.species)):
            pa, pb = a.particles(0, s), b.particles(0, s)
            assert np.array_equal(pa["key"], pb["key"])
            assert np.abs(pa["u"] - pb["u"]).max() <= 1e-5
    for q in range(3):
        fa, fb = a.field_arrays(0)[q], b.field_arrays(0)[q]
        assert np.abs(fa - fb).max() <= 1e-5 * max(np.abs(fa).max(), 1e-30)


def test_nonfinite_momentum_flagged():
    c = _small_2d(1, seed=3)
    c.species[0].u[0, 5] = np.float32(np.nan)
    sim = _sim(c)
    sim.push_fields(0)
    sim.push_particles()
    word = sim.error_word(clear=True)
    assert word & 1
    assert sim.error_word() == 0


def test_superluminal_move_flagged():
    # u so large that dt*v/dx would exceed a cell only if v > c: here the
    # kernel must still keep every particle in bounds; a huge field makes
    # gamma large but |v| < c, so no flag; the flag path is driven through a
    # non-finite momentum instead (move of NaN length).
    c = _small_2d(1, seed=4)
    c.species[0].u[:, 7] = np.float32(np.inf)
    sim = _sim(c)
    sim.push_fields(0)
    sim.push_particles()
    word = sim.error_word(clear=True)
    assert word & (1 | 2)


@pytest.mark.parametrize("kind,order", CASES)
def test_dense_cells_deposit(kind, order):
    """Many particles per cell: long same-cell runs inside each wave (the
    wave-segmented current reduction), plus cell-crossers."""
    if kind == "2d":
        c = _small_2d(order, seed=41, ny=12, nz=10, patch=4, ppc=90)
    else:
        c = _small_3d(order, seed=42, nxyz=(6, 5, 4), patch=3, ppc=70)
    sim = _sim(c)
    ora = O.OracleSim(c)
    sim.push_fields(0)
    sim.push_particles()
    sim.deposit_current()
    assert sim.check() == 0
    ora.push_b_half()
    ora.push_particles()
    for s, sp in enumerate(c.species):
        dpos, du = particle_errors(c, sim.front_buffer(0, s), ora, s, float(np.std(sp.u)))
        assert dpos <= 1e-6 and du <= 1e-5
    _, _, J = sim.field_arrays(0)
    err = np.abs(J.ravel() - ora.J).max()
    print(f"dense: max |dJ| = {err:.3e}, max |J| = {np.abs(ora.J).max():.3e}")
    assert err <= 2e-5 * np.abs(ora.J).max()


# launch shapes: (mode, threads, particles per lane and round, chunk).  A lane
# that pushes several consecutive particles accumulates the current of those
# in its first particle's cell and queues the rest, so every shape must give
# the same particles and, up to summation order, the same current.
SHAPES = [(0, 256, 1, 512), (1, 512, 2, 1024), (1, 384, 2, 256), (2, 512, 2, 2048), (1, 512, 1, 4096),
          (2, 256, 2, 333)]


@pytest.mark.parametrize("kind,order", CASES)
@pytest.mark.parametrize("mode,threads,run,chunk", SHAPES)
def test_launch_shapes_match_oracle(kind, order, mode, threads, run, chunk):
    if kind == "2d":
        c = _small_2d(order, seed=43, ny=12, nz=10, patch=4, ppc=40)
    else:
        c = _small_3d(order, seed=44, nxyz=(6, 5, 4), patch=3, ppc=30)
    sim = _sim(c)
    print(f"[gpu] launch mode={mode} threads={threads} run={run} chunk={chunk}", flush=True)
    sim.set_launch(mode, chunk=chunk, threads=threads, run=run)
    ora = O.OracleSim(c)
    sim.push_fields(0)
    sim.push_particles()
    sim.deposit_current()
    assert sim.check() == 0
    ora.push_b_half()
    ora.push_particles()
    for s, sp in enumerate(c.species):
        dpos, du = particle_errors(c, sim.front_buffer(0, s), ora, s, float(np.std(sp.u)))
        assert dpos <= 1e-6 and du <= 1e-5
    _, _, J = sim.field_arrays(0)
    err = np.abs(J.ravel() - ora.J).max()
    print(f"one push: max |dJ| = {err:.3e}, max |J| = {np.abs(ora.J).max():.3e}")
    assert err <= 2e-5 * np.abs(ora.J).max()
    # three more whole steps: the push then reads through the sort permutation
    sim2 = _sim(c)
    sim2.set_launch(mode, chunk=chunk, threads=threads, run=run)
    ora2 = O.OracleSim(c)
    for _ in range(3):
        sim2.step(1)
        ora2.step(1)
    assert sim2.check() == 0
    for s, sp in enumerate(c.species):
        dpos, du = particle_errors(c, sim2.particles(0, s), ora2, s, float(np.std(sp.u)))
        print(f"3 steps, species {s}: |dxi| {dpos:.3e}, rel |du| {du:.3e}")
        assert dpos <= 1e-5 and du <= 1e-4
    E, B, _ = sim2.field_arrays(0)
    assert np.abs(E.ravel() - ora2.E).max() <= 1e-4 * np.abs(ora2.E).max()
    assert np.abs(B.ravel() - ora2.B).max() <= 1e-4 * np.abs(ora2.B).max()


@pytest.mark.parametrize("kind,order", [("2d", 2), ("3d", 1)])
def test_radix_sort_equals_counting_sort(kind, order):
    """psc_sort_radix (general multi-pass radix sort of the keys) gives the
    same stable permutation and cell offsets as psc_sort (move-code counting
    sort), and the steps that follow agree bit for bit."""
    c = _make(kind, order)
    a, b = _sim(c), _sim(c)
    for step in range(3):
        for sim in (a, b):
            sim.push_fields(0)
            sim.push_particles()
            sim.push_fields(0)
            sim.deposit_current()
            sim.push_fields(1)
        a.sort()
        b.sort_radix()
        assert a.check() == 0 and b.check() == 0
        for s in range(len(c.species)):
            pa, ca = a.sort_view(0, s)
            pb, cb = b.sort_view(0, s)
            assert np.array_equal(pa, pb), f"step {step} species {s}: permutations differ"
            assert np.array_equal(ca, cb)
    for s in range(len(c.species)):
        qa, qb = a.particles(0, s), b.particles(0, s)
        assert np.array_equal(qa["cell"], qb["cell"])
        assert np.array_equal(qa["u"], qb["u"])


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_vb_deposit_matches_oracle(kind):
    """1st-order runs with the Villasenor-Buneman deposit (PSC_RUN_VB): one
    push + deposit and three whole steps against the oracle's VB deposit, and
    the Gauss residual stays at its initial value (charge conservation)."""
    if kind == "2d":
        c = _small_2d(1, seed=81, ny=12, nz=10, patch=4, ppc=40)
    else:
        c = _small_3d(1, seed=82, nxyz=(6, 5, 4), patch=3, ppc=30)
    c.deposit = "vb"
    sim = _sim(c)
    ora = O.OracleSim(c)
    sim.push_fields(0)
    sim.push_particles()
    sim.deposit_current()
    assert sim.check() == 0
    ora.push_b_half()
    ora.push_particles()
    for s, sp in enumerate(c.species):
        dpos, du = particle_errors(c, sim.front_buffer(0, s), ora, s, float(np.std(sp.u)))
        assert dpos <= 1e-6 and du <= 1e-5
    _, _, J = sim.field_arrays(0)
    err = np.abs(J.ravel() - ora.J).max()
    print(f"vb {kind}: max |dJ| = {err:.3e}, max |J| = {np.abs(ora.J).max():.3e}")
    assert err <= 2e-5 * np.abs(ora.J).max()
    # the Esirkepov current differs for the same move (crossings, 2-d J_x)
    c2 = _small_2d(1, seed=81, ny=12, nz=10, patch=4, ppc=40) if kind == "2d" else \
        _small_3d(1, seed=82, nxyz=(6, 5, 4), patch=3, ppc=30)
    esk = O.OracleSim(c2)
    esk.push_b_half()
    esk.push_particles()
    assert np.abs(esk.J - ora.J).max() > 100 * err
    sim2 = _sim(c)
    ora2 = O.OracleSim(c)
    _, g0 = sim2.diagnostics(with_gauss=True)
    for _ in range(3):
        sim2.step(1)
        ora2.step(1)
    assert sim2.check() == 0
    for s, sp in enumerate(c.species):
        dpos, du = particle_errors(c, sim2.particles(0, s), ora2, s, float(np.std(sp.u)))
        assert dpos <= 1e-5 and du <= 1e-4
    E, _, _ = sim2.field_arrays(0)
    assert np.abs(E.ravel() - ora2.E).max() <= 1e-4 * np.abs(ora2.E).max()
    _, g3 = sim2.diagnostics(with_gauss=True)
    rho_scale = np.abs(ora2.rho()).max()
    print(f"vb {kind}: Gauss drift over 3 steps {np.abs(g3 - g0).max():.3e} (rho scale {rho_scale:.3e})")
    assert np.abs(g3 - g0).max() <= 1e-5 * rho_scale


@pytest.mark.parametrize("tile_fold", [False, True])
@pytest.mark.parametrize("order", [1, 2])
def test_3d_patch8_matches_oracle(order, tile_fold):
    """3-d with the Weibel workload's 8^3 patches (its LDS tile layout, its
    deposit, the current added into J with the halo wrapped or the per-patch
    fold at that size): full patches plus a ragged last patch of 4 cells
    along z, after one push and after five steps."""
    c = _small_3d(order, seed=61, nxyz=(16, 16, 20), patch=8, ppc=4)
    sim = _sim(c, tile_fold=tile_fold)
    ora = O.OracleSim(c)
    sim.push_fields(0)
    sim.push_particles()
    sim.deposit_current()
    assert sim.check() == 0
    ora.push_b_half()
    ora.push_particles()
    for s, sp in enumerate(c.species):
        dpos, du = particle_errors(c, sim.front_buffer(0, s), ora, s, float(np.std(sp.u)))
        print(f"one push, species {s}: |dxi| {dpos:.3e}, rel |du| {du:.3e}")
        assert dpos <= 1e-6 and du <= 1e-5
    _, _, J = sim.field_arrays(0)
    assert np.abs(J.ravel() - ora.J).max() <= 2e-5 * np.abs(ora.J).max()
    sim2 = _sim(c, tile_fold=tile_fold)
    ora2 = O.OracleSim(c)
    for _ in range(5):
        sim2.step(1)
        ora2.step(1)
    assert sim2.check() == 0
    for s, sp in enumerate(c.species):
        dpos, du = particle_errors(c, sim2.particles(0, s), ora2, s, float(np.std(sp.u)))
        print(f"5 steps, species {s}: |dxi| {dpos:.3e}, rel |du| {du:.3e}")
        assert dpos <= 1e-5 and du <= 1e-4
    E, B, J = sim2.field_arrays(0)
    assert np.abs(E.ravel() - ora2.E).max() <= 1e-4 * np.abs(ora2.E).max()
    assert np.abs(B.ravel() - ora2.B).max() <= 1e-4 * np.abs(ora2.B).max()
    assert np.abs(J.ravel() - ora2.J).max() <= 1e-4 * np.abs(ora2.J).max()
