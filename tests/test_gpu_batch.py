"""Batched runs and launch shapes of the particle kernel.

Many independent two-stream runs of uneven size (ragged edge patches) share
one context; every launch shape (one workgroup per work item, persistent
workgroups with per-XCD queues, persistent workgroups over the App. A
partition) and HIP-graph replay must give the same state, and each batched
run must equal the same run advanced alone.
"""
import numpy as np
import pytest

from paper_1310_7866_amd import cases

pytestmark = pytest.mark.gpu


def _batch(n=5):
    return cases.twostream_batch(n_runs=n, seed=4064, max_cells=96 * 64)


def _sim(cs, **kw):
    from paper_1310_7866_amd.psc import PscSim
    cl = cs if isinstance(cs, list) else [cs]
    print(f"[gpu] batch of {len(cl)}: {[c.gdims[1:] for c in cl]}", flush=True)
    return PscSim(cs, **kw)


def _state(sim):
    out = []
    for r, c in enumerate(sim.cases):
        for s in range(len(c.species)):
            p = sim.particles(r, s)
            out.append((p["key"], p["id"], p["u"], p["off"]))
        E, B, _ = sim.field_arrays(r)
        out.append((E, B))
    return out


def _same(a, b, tol=1e-6):
    for x, y in zip(a, b):
        if len(x) == 4:
            assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
            assert np.abs(x[2] - y[2]).max(initial=0) <= tol
            assert np.abs(x[3] - y[3]).max(initial=0) <= tol
        else:
            for f, g in zip(x, y):
                assert np.abs(f - g).max(initial=0) <= tol * max(np.abs(g).max(initial=0), 1e-30)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("graph", [False, True])
def test_launch_shapes_agree(mode, graph):
    cs = _batch()
    ref = _sim(cs)
    alt = _sim(cs)
    alt.set_launch(mode, chunk=1024)
    for _ in range(3):
        ref.step(1)
        alt.step(1, use_graph=graph)
    ref.check()
    alt.check()
    _same(_state(ref), _state(alt))


def test_rebalance_between_steps():
    cs = _batch(3)
    ref = _sim(cs)
    alt = _sim(cs)
    alt.set_launch(2, chunk=512, workers=64)
    for k in range(4):
        ref.step(1)
        alt.step(1)
        if k == 1:
            alt.balance(2.0)
    alt.check()
    _same(_state(ref), _state(alt))


def test_batched_runs_equal_alone_two_stream():
    cs = _batch(4)
    batch = _sim(cs)
    for _ in range(3):
        batch.step(1, use_graph=True)
    batch.check()
    for r, c in enumerate(cs):
        alone = _sim(c)
        for _ in range(3):
            alone.step(1)
        for s in range(len(c.species)):
            pb, pa = batch.particles(r, s), alone.particles(0, s)
            assert np.array_equal(pb["key"], pa["key"])
            assert np.abs(pb["u"] - pa["u"]).max() <= 1e-6
        Eb, _, _ = batch.field_arrays(r)
        Ea, _, _ = alone.field_arrays(0)
        assert np.abs(Eb - Ea).max() <= 1e-6 * max(np.abs(Ea).max(), 1e-30)


def _uneven_batch(order):
    """Four runs of one context: two-species thermal runs and a one-species
    two-stream run, different particles per cell, ragged last patches, and
    (at both orders) one run whose last patch is narrower than the current
    halo, so that with per-patch current tiles the batch folds by patch and
    with the alias search."""
    def charged(seed, ny, nz, patch, ppc):
        c = cases.thermal2d(ny=ny, nz=nz, ppc=ppc, order=order, patch=patch, seed=seed)
        c.species[1].off = np.random.default_rng(seed + 1000).random(c.species[1].off.shape).astype(np.float32)
        cases.random_fields(c, 0.02, 0.2, seed=seed + 1)
        return c
    ts = cases.twostream2d(ny=40, nz=20, ppc=10, order=order, patch=16, seed=77)
    cases.random_fields(ts, 0.02, 0.2, seed=78)
    narrow = 8 + 8 + order            # last patch of `order` cells: narrower than order + 1
    return [charged(51, narrow, 12, 8, 6), charged(52, 24, 16, 8, 3), ts, charged(53, 30, 22, 8, 9)]


# chunk per run of _uneven_batch (run 0 keeps the context's 512)
RUN_CHUNKS = {1: 128, 2: 333, 3: 2048}


def _run_chunks(sim):
    for r, ch in RUN_CHUNKS.items():
        sim.set_run_chunk(r, ch)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_per_run_chunks_agree(mode):
    """Different chunks per run hand the same particles to other work items:
    the same state as one chunk for every run (fields to the summation order
    of the current tiles)."""
    cs = _uneven_batch(1)
    a, b = _sim(cs), _sim(cs)
    a.set_launch(mode, chunk=512)
    b.set_launch(mode, chunk=512)
    _run_chunks(b)
    for k in range(3):
        a.step(1)
        b.step(1, use_graph=k > 0)
    a.check()
    b.check()
    _same(_state(a), _state(b))


@pytest.mark.parametrize("order,mode,tile_fold", [(1, 1, False), (1, 2, False), (2, 1, False), (2, 2, False),
                                                  (1, 1, True), (2, 2, True)])
def test_batch_matches_oracle(order, mode, tile_fold):
    """Every run of a batched context (a different chunk per run) against
    the double-precision oracle run alone: one push (the parity tolerances
    of single runs), then three whole steps replayed from a HIP graph.
    tile_fold: the current through per-patch tiles and both fold kernels
    instead of the particle kernel adding it into J."""
    from oracle import oracle as O
    from tests.helpers import particle_errors
    cs = _uneven_batch(order)
    sim = _sim(cs, tile_fold=tile_fold)
    sim.set_launch(mode, chunk=512)
    _run_chunks(sim)
    oras = [O.OracleSim(c) for c in cs]
    sim.push_fields(0)
    sim.push_particles()
    sim.deposit_current()
    assert sim.check() == 0
    for r, (c, ora) in enumerate(zip(cs, oras)):
        ora.push_b_half()
        ora.push_particles()
        for s, sp in enumerate(c.species):
            dpos, du = particle_errors(c, sim.front_buffer(r, s), ora, s, float(np.std(sp.u)))
            print(f"run {r} species {s}: one push |dxi| {dpos:.3e}, rel |du| {du:.3e}", flush=True)
            assert dpos <= 1e-6 and du <= 1e-5
        _, _, J = sim.field_arrays(r)
        assert np.abs(J.ravel() - ora.J).max() <= 2e-5 * np.abs(ora.J).max()
    sim2 = _sim(cs, tile_fold=tile_fold)
    sim2.set_launch(mode, chunk=512)
    _run_chunks(sim2)
    oras = [O.OracleSim(c) for c in cs]
    for _ in range(3):
        sim2.step(1, use_graph=True)
        for ora in oras:
            ora.step(1)
    assert sim2.check() == 0
    for r, (c, ora) in enumerate(zip(cs, oras)):
        for s, sp in enumerate(c.species):
            dpos, du = particle_errors(c, sim2.particles(r, s), ora, s, float(np.std(sp.u)))
            print(f"run {r} species {s}: 3 steps |dxi| {dpos:.3e}, rel |du| {du:.3e}", flush=True)
            assert dpos <= 1e-5 and du <= 1e-4
        E, B, _ = sim2.field_arrays(r)
        assert np.abs(E.ravel() - ora.E).max() <= 1e-4 * np.abs(ora.E).max()
        assert np.abs(B.ravel() - ora.B).max() <= 1e-4 * np.abs(ora.B).max()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_unit_orders_agree(mode):
    """Row-major and Hilbert unit orders hand the same work out in another
    order: the same particles, and fields to the summation order of the
    current tiles."""
    from paper_1310_7866_amd.psc import ORDER_HILBERT, ORDER_ROWMAJOR
    cs = _uneven_batch(2)
    a, b = _sim(cs), _sim(cs)
    a.set_launch(mode, chunk=512)
    b.set_launch(mode, chunk=512)
    b.set_unit_order(ORDER_HILBERT)   # the default is row-major
    for k in range(3):
        a.step(1)
        b.step(1, use_graph=k > 0)
    b.set_unit_order(ORDER_ROWMAJOR)
    b.step(1)
    a.step(1)
    a.check()
    b.check()
    _same(_state(a), _state(b))
