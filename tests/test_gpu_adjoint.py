"""GPU adjoint (psc_adjoint_step driven with checkpoints) against the FP64
CPU adjoint of oracle/adjoint.py (autograd of the plain float64 step, itself
pinned to central finite differences of the C oracle).

Bar: relative L2 error of each gradient block (dW/dE0, dW/dB0, dW/du0 per
species) <= 1e-3 -- float32 forward and reverse arithmetic over the steps
against float64.
"""
import numpy as np
import pytest

from oracle import adjoint as A
from paper_1310_7866_amd import cases

pytestmark = pytest.mark.gpu


def _case(order, seed, ny=16, nz=12, ppc=6, patch=8):
    c = cases.harris2d(ny=ny, nz=nz, ppc=ppc, order=order, patch=patch, seed=seed, dx=0.25)
    cases.random_fields(c, 0.02, 0.1, seed=seed + 3)
    return c


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("order", [1, 2])
def test_adjoint_matches_fp64_oracle(order):
    from paper_1310_7866_amd.adjoint import energy_gradient
    c = _case(order, seed=50 + order)
    nsteps, every = 8, 3
    print(f"[gpu] adjoint order {order} gdims={c.gdims} n={c.n_particles}", flush=True)
    W, gE, gB, gU, fms, ams = energy_gradient(c, nsteps, every)
    Wo, oE, oB, oU = A.energy_gradient(c, nsteps)
    nx, ny, nz = c.gdims
    oE = oE.reshape(3, -1)
    oB = oB.reshape(3, -1)
    errs = dict(W=abs(W - Wo) / Wo, E=_rel(gE, oE), B=_rel(gB, oB))
    for s in range(len(gU)):
        errs[f"u{s}"] = _rel(gU[s], oU[s])
    print(f"order {order}: relative errors {errs}; forward {fms:.2f} ms, adjoint {ams:.2f} ms")
    assert errs["W"] <= 1e-5
    for k, v in errs.items():
        assert v <= 1e-3, (k, v)


def test_autograd_function_matches_driver():
    import torch
    from paper_1310_7866_amd.adjoint import energy_gradient, field_energy
    c = _case(2, seed=61)
    E0 = torch.tensor(c.E, requires_grad=True)
    B0 = torch.tensor(c.B, requires_grad=True)
    u0 = [torch.tensor(sp.u, requires_grad=True) for sp in c.species]
    W = field_energy(c, 6, 3, E0, B0, *u0)
    W.backward()
    W2, gE, gB, gU, _, _ = energy_gradient(c, 6, 3)
    assert abs(W.item() - W2) <= 1e-6 * W2
    assert _rel(E0.grad.numpy(), gE) <= 1e-4
    assert _rel(B0.grad.numpy(), gB) <= 1e-4
    for s in range(2):
        assert _rel(u0[s].grad.numpy(), gU[s]) <= 1e-4


def test_checkpoint_interval_does_not_change_gradient():
    from paper_1310_7866_amd.adjoint import energy_gradient
    c = _case(2, seed=71)
    _, a_E, a_B, a_U, _, _ = energy_gradient(c, 6, 6)
    _, b_E, b_B, b_U, _, _ = energy_gradient(c, 6, 2)
    assert _rel(a_E, b_E) <= 1e-4 and _rel(a_B, b_B) <= 1e-4
    for s in range(2):
        assert _rel(a_U[s], b_U[s]) <= 1e-4
