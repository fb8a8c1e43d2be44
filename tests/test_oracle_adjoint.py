"""Pins of the FP64 CPU adjoint (oracle/adjoint.py).

* Its forward equals the C oracle's forward after several steps (1e-12): the
  same step of fig. psc_new written twice, independently.
* Its gradient of the final field energy W = 1/2 sum(E^2 + B^2) dV with
  respect to the initial E, B and particle momenta equals central finite
  differences of the C oracle along random directions and single
  coordinates (2nd-order shapes, where the step is continuously
  differentiable), relative error <= 1e-6.
* Dot-product (transpose) identity of the discrete curls used by the reverse
  field update: <curl^+ E, B> = <E, curl^- B>.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import adjoint as A
from paper_1310_7866_amd import cases

torch = pytest.importorskip("torch")


def _case(dim, order, seed):
    if dim == 2:
        c = cases.thermal2d(ny=10, nz=9, ppc=3, order=order, patch=5, seed=seed)
        c.species[1].off = np.random.default_rng(seed + 1000).random(c.species[1].off.shape).astype(np.float32)
    else:
        c = cases.weibel3d(ppc=2, order=order, patch=3, seed=seed, nxyz=(5, 4, 6))
    cases.random_fields(c, 0.05, 0.3, seed=seed + 1)
    return c


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_torch_forward_equals_c_oracle(dim, order):
    c = _case(dim, order, 3)
    pic, E, B, sps = A.from_case(c)
    ora = O.OracleSim(c, sort_initial=False)
    for _ in range(4):
        E, B, sps = pic.step(E, B, sps)
        ora.step(1, sort=False)
    nx, ny, nz = c.gdims
    assert np.abs(E.numpy().reshape(-1) - ora.E).max() < 1e-12 * max(1.0, np.abs(ora.E).max())
    assert np.abs(B.numpy().reshape(-1) - ora.B).max() < 1e-12 * max(1.0, np.abs(ora.B).max())
    for s, sp in enumerate(sps):
        assert np.abs(sp["u"].numpy() - ora.species[s].u).max() < 1e-12
        dx = sp["x"].numpy() - ora.species[s].xi
        for d in range(3):
            dx[d] -= c.gdims[d] * np.round(dx[d] / c.gdims[d])
        assert np.abs(dx).max() < 1e-12


def _oracle_energy(c, nsteps, dE=None, dB=None, du=None, h=0.0):
    ora = O.OracleSim(c)
    if dE is not None:
        ora.E = ora.E + h * dE.reshape(-1)
    if dB is not None:
        ora.B = ora.B + h * dB.reshape(-1)
    if du is not None:
        for s, sp in enumerate(ora.species):
            sp.u = np.ascontiguousarray(sp.u + h * du[s][:, sp.ids])
    ora.step(nsteps)
    we, wb = ora.field_energy()
    return we + wb


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_matches_finite_differences(dim):
    c = _case(dim, 2, 7)
    nsteps = 4
    W, gE, gB, gU = A.energy_gradient(c, nsteps)
    assert abs(W - _oracle_energy(c, nsteps)) < 1e-12 * abs(W)
    rng = np.random.default_rng(11)
    h = 1e-6
    # central differences carry a roundoff floor of about eps*|W|/h
    floor = 8 * np.finfo(float).eps * abs(W) / h
    checks = []
    for k in range(6):
        dE = rng.normal(size=gE.shape) * (k % 3 == 0)
        dB = rng.normal(size=gB.shape) * (k % 3 == 1)
        du = [rng.normal(size=g.shape) * 0.05 * (k % 3 == 2) for g in gU]
        fd = (_oracle_energy(c, nsteps, dE, dB, du, h) - _oracle_energy(c, nsteps, dE, dB, du, -h)) / (2 * h)
        ad = (gE * dE).sum() + (gB * dB).sum() + sum((g * d).sum() for g, d in zip(gU, du))
        checks.append((fd, ad))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + floor, (k, fd, ad)
    # single coordinates: one momentum component of one particle, one field value
    i = int(np.argmax(np.abs(gU[0][2])))
    du = [np.zeros_like(g) for g in gU]
    du[0][2, i] = 1.0
    fd = (_oracle_energy(c, nsteps, None, None, du, h) - _oracle_energy(c, nsteps, None, None, du, -h)) / (2 * h)
    assert abs(fd - gU[0][2, i]) <= 1e-6 * abs(gU[0][2, i]) + floor
    j = int(np.argmax(np.abs(gB.reshape(-1))))
    dB = np.zeros(gB.size)
    dB[j] = 1.0
    fd = (_oracle_energy(c, nsteps, None, dB, None, h) - _oracle_energy(c, nsteps, None, dB, None, -h)) / (2 * h)
    assert abs(fd - gB.reshape(-1)[j]) <= 1e-6 * abs(gB.reshape(-1)[j]) + floor


@pytest.mark.parametrize("dim", [2, 3])
def test_curl_transpose(dim):
    c = _case(dim, 1, 5)
    pic, E, B, _ = A.from_case(c)
    rng = np.random.default_rng(2)
    e = torch.tensor(rng.normal(size=E.shape))
    b = torch.tensor(rng.normal(size=B.shape))
    lhs = (pic.curl_plus(e) * b).sum().item()
    rhs = (e * pic.curl_minus(b)).sum().item()
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
