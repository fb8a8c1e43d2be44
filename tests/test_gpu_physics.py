"""GPU physics checks against the oracle and against invariants.

* FP64 diagnostics (field/kinetic energy, charge, Gauss residual) equal the
  oracle's on the same float32 state to 1e-9 relative.
* Gauss invariant: max|G^n - G^0| stays at float32 roundoff
  (<= 1e-5 * max|rho_species|) over 50 steps (FDTD section: exact under
  discrete continuity).
* The 64x64 thermal workload, 100 steps: relative field-energy error <= 1e-4
  and relative kinetic-energy error <= 1e-5 against the oracle.
* k = 0 cold plasma oscillation: omega = (2/dt) asin(dt/2) to 1e-5.
* Batching: runs advanced in one context equal the same runs alone.
* Patch size does not change the physics (16x16 vs 8x8 patches).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1310_7866_amd import cases
from tests.helpers import particle_errors

pytestmark = pytest.mark.gpu


def _sim(case, **kw):
    from paper_1310_7866_amd.psc import PscSim
    name = case[0].name + f" x{len(case)}" if isinstance(case, list) else case.name
    print(f"[gpu] {name}", flush=True)
    return PscSim(case, **kw)


def _charged(order, seed=11, ny=24, nz=20, patch=8, ppc=8):
    c = cases.thermal2d(ny=ny, nz=nz, ppc=ppc, order=order, patch=patch, seed=seed)
    c.species[1].off = np.random.default_rng(seed + 1000).random(c.species[1].off.shape).astype(np.float32)
    cases.random_fields(c, 0.02, 0.2, seed=seed + 1)
    return c


@pytest.mark.parametrize("order", [1, 2])
def test_diagnostics_match_oracle(order):
    c = _charged(order)
    sim = _sim(c)
    ora = O.OracleSim(c)
    d, G = sim.diagnostics(with_gauss=True)
    we, wb = ora.field_energy()
    ke = ora.kinetic_energy()
    rho = ora.rho()
    dV = c.dx[1] * c.dx[2]
    assert abs(d[0, 0] - we) <= 1e-9 * max(we, 1e-30)
    assert abs(d[0, 1] - wb) <= 1e-9 * wb
    for s in range(2):
        assert abs(d[0, 2 + s] - ke[s]) <= 1e-9 * ke[s]
    g_ref = ora.div_e() - rho
    assert np.abs(G - g_ref).max() <= 1e-9 * np.abs(rho).max()
    assert abs(d[0, 6] - np.abs(g_ref).max()) <= 1e-9 * np.abs(rho).max()
    assert abs(d[0, 8] - rho.sum() * dV) <= 1e-9 * np.abs(rho).sum() * dV
    assert d[0, 9] == c.n_particles


@pytest.mark.parametrize("order", [1, 2])
def test_gauss_invariant_over_steps(order):
    """max|G^n - G^0| over 50 steps <= 1e-5 max_s max|rho_s|, G = div E - rho.

    The scheme keeps G exactly under discrete continuity, so only float32
    roundoff moves it: each step adds to E a float32 current whose
    contributions are of size q w dx/dt per particle, and div E differences
    float32 E values; rho itself is accumulated in float64 by the
    diagnostics.  Relative to the species densities rho_s the drift stays a
    few float32 ulps per step.  (An earlier bar of 1e-5 max|q w|, a single
    particle's charge, is 1/ppc of this one at density 1; the measured drift
    is printed against both.)"""
    c = _charged(order, seed=13)
    sim = _sim(c)
    _, G0 = sim.diagnostics(with_gauss=True)
    ora = O.OracleSim(c)
    rho_s = max(np.abs(O.rho_of(ora.g, sp.xi, sp.q * sp.w)).max() for sp in ora.species)
    qw = max(abs(sp.q * sp.w) for sp in c.species)
    worst = 0.0
    for k in range(50):
        sim.step(1)
        _, G = sim.diagnostics(with_gauss=True)
        worst = max(worst, np.abs(G - G0).max())
    sim.check()
    print(f"order {order}: max |G^n - G^0| over 50 steps = {worst:.3e}; 1e-5 max|rho_s| = {1e-5 * rho_s:.3e}, "
          f"1e-5 max|q w| = {1e-5 * qw:.3e}", flush=True)
    assert worst <= 1e-5 * rho_s


def test_thermal_workload_energies_100_steps():
    c = cases.thermal2d()   # 64x64 cells, 16 pairs/cell, order 1, seed 1310
    sim = _sim(c)
    ora = O.OracleSim(c)
    for _ in range(100):
        sim.step(1, use_graph=True)
    ora.step(100)
    sim.check()
    d = sim.diagnostics()
    we, wb = ora.field_energy()
    ke = ora.kinetic_energy()
    wf = we + wb
    rel_f = abs(d[0, 0] + d[0, 1] - wf) / wf
    rel_k = max(abs(d[0, 2 + s] - ke[s]) / ke[s] for s in range(2))
    print(f"thermal2d 100 steps: field energy {wf:.6e} rel err {rel_f:.2e}; kinetic rel err {rel_k:.2e}")
    assert rel_f <= 1e-4
    assert rel_k <= 1e-5


@pytest.mark.parametrize("order", [1, 2])
def test_plasma_frequency_gpu(order):
    c = cases.plasma_oscillation2d(order=order, patch=4)
    sim = _sim(c)
    hist = []
    for _ in range(300):
        sim.step(1)
        E, _, _ = sim.field_arrays(0)
        hist.append(float(E[2].astype(np.float64).mean()))
    e = np.array(hist)
    cw = (e[1:-1] @ (e[2:] + e[:-2])) / (2 * e[1:-1] @ e[1:-1])
    omega = math.acos(cw) / c.dt
    want = (2.0 / c.dt) * math.asin(c.dt / 2.0)
    print(f"order {order}: omega {omega:.8f} want {want:.8f}")
    assert abs(omega - want) <= 1e-5 * want


def _batch_vs_alone(runs, **kw):
    batch = _sim(runs, **kw)
    alone = [_sim(r, **kw) for r in runs]
    for _ in range(4):
        batch.step(1)
        for a in alone:
            a.step(1)
    batch.check()
    for r, a in enumerate(alone):
        a.check()
        for s in range(2):
            pb, pa = batch.particles(r, s), a.particles(0, s)
            assert np.array_equal(pb["key"], pa["key"])
            assert np.array_equal(pb["id"], pa["id"])
            assert np.abs(pb["u"] - pa["u"]).max() <= 1e-6
            assert np.abs(pb["off"] - pa["off"]).max() <= 1e-6
        Eb, Bb, _ = batch.field_arrays(r)
        Ea, Ba, _ = a.field_arrays(0)
        assert np.abs(Eb - Ea).max() <= 1e-6 * max(np.abs(Ea).max(), 1e-30)


def test_batch_equals_runs_alone():
    _batch_vs_alone([_charged(1, seed=20 + r, ny=16 + 8 * r, nz=12 + 4 * r, patch=8, ppc=4 + 2 * r)
                     for r in range(3)])


def test_batch_mixing_fold_paths_equals_runs_alone():
    # per-patch current tiles, order 2 (current halo 3 cells): 18 = 8 + 8 + 2
    # leaves a last patch narrower than the halo, folded with the alias
    # search; the other run's patches are all wide enough for the per-patch
    # fold.  One batch launches both fold kernels.
    _batch_vs_alone([_charged(2, seed=41, ny=18, nz=12, patch=8, ppc=6),
                     _charged(2, seed=42, ny=24, nz=16, patch=8, ppc=6)], tile_fold=True)


def test_patch_size_independence():
    a = _charged(2, seed=31, ny=32, nz=32, patch=16)
    b = _charged(2, seed=31, ny=32, nz=32, patch=8)
    sa, sb = _sim(a), _sim(b)
    for _ in range(3):
        sa.step(1)
        sb.step(1)
    for s in range(2):
        pa, pb = sa.particles(0, s), sb.particles(0, s)
        oa, ob = np.argsort(pa["id"]), np.argsort(pb["id"])
        assert np.array_equal(pa["cell"][oa], pb["cell"][ob])
        assert np.abs(pa["u"][:, oa] - pb["u"][:, ob]).max() <= 1e-6
    Ea, _, _ = sa.field_arrays(0)
    Eb, _, _ = sb.field_arrays(0)
    assert np.abs(Ea - Eb).max() <= 1e-6 * np.abs(Ea).max()


def _weibel_small():
    c = cases.weibel3d(ppc=16, order=1, patch=8, nxyz=(16, 16, 24), seed=19)
    cases.random_fields(c, 0.05, 0.3, seed=20)
    return c


REPEAT_CASES = {
    "harris2d": lambda: cases.harris2d(ny=128, nz=64, ppc=40, order=2, patch=32, seed=17),
    "weibel3d": _weibel_small,
}


@pytest.mark.parametrize("tile_fold", [False, True])
@pytest.mark.parametrize("name", sorted(REPEAT_CASES))
def test_repeat_runs_agree(name, tile_fold):
    """Run-to-run reproducibility: the same case advanced twice (several work
    items per patch, so that a patch's current is added to by several
    workgroups in an order that varies between runs) gives identical keys,
    ids and cell offsets.  With the current added into J by the particle
    kernel, in fixed point (integer sums), the whole state is bit for bit
    identical.  With per-patch float tiles (tile_fold) the tiles are summed
    with float atomics: momenta and offsets agree to 1e-6, fields to 2e-5 of
    their largest value (the one-deposit current tolerance)."""
    c = REPEAT_CASES[name]()
    a, b = _sim(c, chunk=1024, tile_fold=tile_fold), _sim(c, chunk=1024, tile_fold=tile_fold)
    for _ in range(10):
        a.step(1)
        b.step(1)
    a.check()
    b.check()
    ndiff = 0
    for s in range(len(c.species)):
        pa, pb = a.particles(0, s), b.particles(0, s)
        assert np.array_equal(pa["key"], pb["key"]) and np.array_equal(pa["id"], pb["id"])
        assert np.array_equal(a.sort_view(0, s)[1], b.sort_view(0, s)[1])
        assert np.abs(pa["u"] - pb["u"]).max(initial=0) <= 1e-6
        assert np.abs(pa["off"] - pb["off"]).max(initial=0) <= 1e-6
        ndiff += int((pa["u"] != pb["u"]).sum() + (pa["off"] != pb["off"]).sum())
    for fname, fa, fb in zip("EBJ", a.field_arrays(0), b.field_arrays(0)):
        rel = float(np.abs(fa - fb).max() / max(np.abs(fa).max(), 1e-30))
        print(f"{fname}: largest difference {rel:.2e} of max|{fname}|", flush=True)
        assert rel <= 2e-5
        ndiff += int((fa != fb).sum())
    print(f"{name}, 10 steps, two runs: {ndiff} float values differ (integer state identical)", flush=True)
    if not tile_fold:
        assert ndiff == 0


def test_sort_outputs_redirected_equal_workspace():
    """psc_set_sort_outputs: a run whose sorts write their permutation and
    cell offsets into caller arrays (switched every step, as the adjoint
    does, with the counting sort, the radix sort and graph replay) stays bit
    for bit equal to the same run on the workspace's arrays; the arrays hold
    that run's permutation and offsets; returning to the workspace keeps the
    state (the next steps stay equal too)."""
    import torch
    c = cases.harris2d(ny=64, nz=32, ppc=20, order=2, patch=16, seed=23)
    a, b = _sim(c, chunk=1024), _sim(c, chunk=1024)
    bufs = [[dict(perm=torch.empty(sp.n, dtype=torch.int32, device="cuda"),
                  cs=torch.empty(c.ncell + 1, dtype=torch.int32, device="cuda")) for _ in range(2)]
            for sp in c.species]
    from paper_1310_7866_amd.psc import B_HALF, E_FULL
    for k in range(6):
        for s in range(len(c.species)):
            b.set_sort_outputs(0, s, bufs[s][k % 2]["perm"], bufs[s][k % 2]["cs"])
        a.step(1)
        if k % 3 == 2:   # the general radix sort writes the same outputs
            b.push_fields(B_HALF)
            b.push_particles()
            b.push_fields(B_HALF)
            b.deposit_current()
            b.push_fields(E_FULL)
            b.sort_radix()
        else:
            b.step(1, use_graph=k == 4)
        for s in range(len(c.species)):
            assert torch.equal(a.get_perm(0, s), bufs[s][k % 2]["perm"])
            assert torch.equal(a.cell_offsets(0, s), bufs[s][k % 2]["cs"])
            assert torch.equal(b.get_perm(0, s), bufs[s][k % 2]["perm"])
    for s in range(len(c.species)):
        b.set_sort_outputs(0, s, None, None)
    for _ in range(3):
        a.step(1)
        b.step(1, use_graph=True)
    assert a.check() == 0 and b.check() == 0
    for s in range(len(c.species)):
        pa, pb = a.particles(0, s), b.particles(0, s)
        for key in ("key", "id", "off", "u"):
            assert np.array_equal(pa[key], pb[key]), key
        assert np.array_equal(a.sort_view(0, s)[1], b.sort_view(0, s)[1])
    for fa, fb in zip(a.field_arrays(0), b.field_arrays(0)):
        assert np.array_equal(fa, fb)
