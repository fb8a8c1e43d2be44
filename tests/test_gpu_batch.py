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
