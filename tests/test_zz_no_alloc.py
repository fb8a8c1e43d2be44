"""psc_bind_static: the context bound to the library-held workspace (for
callers that cannot allocate device memory) gives the same state as the
same context bound to a caller workspace with psc_bind, on two binds in a
row (the second with a smaller input, so the array holds the first one's
leftovers), and refuses runs whose workspace exceeds the array.
"""
import numpy as np
import pytest

from paper_1310_7866_amd import cases

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 * 1024 * 1024   # PSC_STATIC_WORKSPACE_BYTES


def _state(sim):
    out = []
    for r, c in enumerate(sim.cases):
        for s in range(len(c.species)):
            p = sim.particles(r, s)
            out.append((p["key"], p["id"], p["u"], p["off"]))
        E, B, J = sim.field_arrays(r)
        out.append((E, B, J))
    return out


def _same(a, b, tol=1e-6):
    """Keys and ids bit-exact (integer work); offsets and momenta within
    1e-6 absolute, fields within 1e-6 of their largest value (the two binds
    run the same kernels; only the order of the float current additions
    between work items of a patch may differ)."""
    for x, y in zip(a, b):
        if len(x) == 4:
            assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
            assert np.abs(x[2] - y[2]).max(initial=0) <= tol
            assert np.abs(x[3] - y[3]).max(initial=0) <= tol
        else:
            for f, g in zip(x, y):
                assert np.abs(f - g).max(initial=0) <= tol * max(np.abs(g).max(initial=0), 1e-30)


def test_static_bind_equals_caller_workspace_twice():
    from paper_1310_7866_amd.psc import PscError, PscSim
    big = cases.thermal2d(ny=64, nz=48, ppc=8, order=2, patch=16, seed=901)
    cases.random_fields(big, 0.05, 0.3, seed=903)
    small = cases.thermal2d(ny=24, nz=16, ppc=4, order=1, patch=8, seed=902)
    cases.random_fields(small, 0.05, 0.3, seed=904)
    first = None
    for c in (big, small):
        print(f"[gpu] static bind: {c.gdims} order {c.order} {c.n_particles} particles", flush=True)
        st = PscSim(c, static_workspace=True)
        assert st.workspace is None and 0 < st.workspace_bytes <= STATIC_BYTES
        ref = PscSim(c)
        for k in range(3):
            st.step(1, use_graph=(k == 2))
            ref.step(1, use_graph=(k == 2))
        st.check()
        ref.check()
        _same(_state(st), _state(ref))
        if first is None:
            first = st          # keep it: the second static bind takes its array
        else:
            st.close()
        ref.close()
    # the first context lost the array to the second: it refuses to step
    with pytest.raises(PscError) as e:
        first.step(1)
    assert e.value.status == 8
    first.close()


def test_static_bind_refuses_oversized_runs():
    from paper_1310_7866_amd.psc import PscError, PscSim
    c = cases.thermal2d(ny=512, nz=512, ppc=16, order=1, patch=32, seed=905)
    print(f"[gpu] static bind oversize: {c.gdims} {c.n_particles} particles", flush=True)
    with pytest.raises(PscError) as e:
        PscSim(c, with_ids=False, static_workspace=True)
    assert e.value.status == 1 and "bytes of workspace" in str(e.value)
