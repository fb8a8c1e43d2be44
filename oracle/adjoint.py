"""Double-precision CPU adjoint of the PIC step (test infrastructure only).

The time step of fig. psc_new written out again with plain PyTorch float64
CPU operations -- B half step, gather with B-spline weights (eq. E_interp
and the b1/b2 definitions), Boris' split push, position update, Esirkepov
deposit (discrete continuity), B half step, E full step -- so that autograd
gives the exact gradient of any scalar of the final state with respect to
the initial fields and momenta.  The forward is pinned to the C oracle
(same state after several steps to 1e-12) and the gradient to central finite
differences of the C oracle; see tests/test_oracle_adjoint.py.

The sort only reorders particles and is omitted here.  Positions are
absolute, in cell units.  Shares nothing with the HIP library.
"""
from __future__ import annotations

from typing import Sequence

import torch

T = torch.float64


def bspline(order: int, s: torch.Tensor) -> torch.Tensor:
    a = s.abs()
    if order == 1:
        return torch.clamp(1.0 - a, min=0.0)
    inner = 0.75 - a * a
    outer = 0.5 * (1.5 - a) ** 2
    return torch.where(a <= 0.5, inner, torch.where(a <= 1.5, outer, torch.zeros_like(a)))


class TorchPIC:
    """Periodic run; fields (3, nz, ny, nx) float64, particles (3, n)."""

    STAG_E = ((0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5))
    STAG_B = ((0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0))

    def __init__(self, dim: int, n: Sequence[int], d: Sequence[float], dt: float, order: int):
        self.dim, self.n, self.d, self.dt, self.order = dim, tuple(n), tuple(d), float(dt), order
        self.active = (0, 1, 2) if dim == 3 else (1, 2)
        self.dV = d[1] * d[2] * (d[0] if dim == 3 else 1.0)

    # field arrays are indexed [c, k, j, i]; axis of dimension d is 3 - d
    def _shift(self, F, d, s):
        if d not in self.active:
            return F
        return torch.roll(F, shifts=-s, dims=F.dim() - 1 - d)

    def curl_plus(self, E):
        Ex, Ey, Ez = E[0], E[1], E[2]
        d = self.d
        def df(F, ax):   # forward difference along ax
            if ax not in self.active:
                return torch.zeros_like(F)
            return (self._shift(F, ax, 1) - F) / d[ax]
        return torch.stack([df(Ez, 1) - df(Ey, 2), df(Ex, 2) - df(Ez, 0), df(Ey, 0) - df(Ex, 1)])

    def curl_minus(self, B):
        Bx, By, Bz = B[0], B[1], B[2]
        d = self.d
        def db(F, ax):   # backward difference
            if ax not in self.active:
                return torch.zeros_like(F)
            return (F - self._shift(F, ax, -1)) / d[ax]
        return torch.stack([db(Bz, 1) - db(By, 2), db(Bx, 2) - db(Bz, 0), db(By, 0) - db(Bx, 1)])

    def _window(self, x, stag, width):
        """Node indices (width per active dim) and weights for positions x."""
        idx, w = [], []
        for d in range(3):
            if d not in self.active:
                idx.append(torch.zeros(1, x.shape[1], dtype=torch.long))
                w.append(torch.ones(1, x.shape[1], dtype=T))
                continue
            p = x[d] - stag[d]
            base = torch.floor(p.detach()).long() - (width // 2 - 1)
            nodes = base[None, :] + torch.arange(width)[:, None]
            w.append(bspline(self.order, p[None, :] - nodes.to(T)))
            idx.append(torch.remainder(nodes, self.n[d]))
        return idx, w

    def gather(self, F, x, stag):
        (ix, iy, iz), (wx, wy, wz) = self._window(x, stag, 4)
        out = 0.0
        for a in range(ix.shape[0]):
            for b in range(iy.shape[0]):
                for c in range(iz.shape[0]):
                    out = out + wx[a] * wy[b] * wz[c] * F[iz[c], iy[b], ix[a]]
        return out

    def boris(self, u, E, B, h):
        um = u + h * E
        gm = torch.sqrt(1.0 + (um * um).sum(0))
        t = h * B / gm
        s = 2.0 * t / (1.0 + (t * t).sum(0))
        up = um + torch.cross(um, t, dim=0)
        uq = um + torch.cross(up, s, dim=0)
        return uq + h * E

    def deposit(self, x0, x1, u, q, w):
        nz, ny, nx = self.n[2], self.n[1], self.n[0]
        J = torch.zeros(3, nz * ny * nx, dtype=T)
        L = 6
        S0, DS, ids = [], [], []
        for d in range(3):
            if d not in self.active:
                S0.append(torch.ones(1, x0.shape[1], dtype=T))
                DS.append(torch.zeros(1, x0.shape[1], dtype=T))
                ids.append(torch.zeros(1, x0.shape[1], dtype=torch.long))
                continue
            base = torch.floor(x0[d].detach()).long() - 2
            nodes = base[None, :] + torch.arange(L)[:, None]
            s0 = bspline(self.order, x0[d][None, :] - nodes.to(T))
            s1 = bspline(self.order, x1[d][None, :] - nodes.to(T))
            S0.append(s0)
            DS.append(s1 - s0)
            ids.append(torch.remainder(nodes, self.n[d]))
        qw = q * w
        gam = torch.sqrt(1.0 + (u * u).sum(0))
        def lin(i, j, k):
            return (ids[0][i] + nx * (ids[1][j] + ny * ids[2][k]))
        if self.dim == 3:
            comps = [(0, 1, 2), (1, 0, 2), (2, 0, 1)]
            for c, a, b in comps:
                f = -qw * self.d[c] / self.dt
                la, lb = S0[a].shape[0], S0[b].shape[0]
                for ia in range(la):
                    for ib in range(lb):
                        cross = (S0[a][ia] * S0[b][ib] + 0.5 * DS[a][ia] * S0[b][ib] +
                                 0.5 * S0[a][ia] * DS[b][ib] + DS[a][ia] * DS[b][ib] / 3.0)
                        Wc = DS[c] * cross[None, :]
                        acc = torch.cumsum(Wc, dim=0)
                        for ic in range(L):
                            sel = [0, 0, 0]
                            sel[c], sel[a], sel[b] = ic, ia, ib
                            J[c] = J[c].index_add(0, lin(*sel), f * acc[ic])
        else:
            fy = -qw * self.d[1] / self.dt
            fz = -qw * self.d[2] / self.dt
            for n_ in range(L):
                acc = torch.cumsum(DS[1] * (S0[2][n_] + 0.5 * DS[2][n_])[None, :], dim=0)
                for m in range(L):
                    J[1] = J[1].index_add(0, lin(0, m, n_), fy * acc[m])
            for m in range(L):
                acc = torch.cumsum(DS[2] * (S0[1][m] + 0.5 * DS[1][m])[None, :], dim=0)
                for n_ in range(L):
                    J[2] = J[2].index_add(0, lin(0, m, n_), fz * acc[n_])
            vx = u[0] / gam
            for m in range(L):
                for n_ in range(L):
                    sh = (S0[1][m] * S0[2][n_] + 0.5 * DS[1][m] * S0[2][n_] +
                          0.5 * S0[1][m] * DS[2][n_] + DS[1][m] * DS[2][n_] / 3.0)
                    J[0] = J[0].index_add(0, lin(0, m, n_), qw * vx * sh)
        return J.reshape(3, nz, ny, nx)

    def step(self, E, B, species):
        """species: list of dict(x, u, q, m, w); returns new E, B and species."""
        dt = self.dt
        B1 = B - 0.5 * dt * self.curl_plus(E)
        J = torch.zeros_like(E)
        out = []
        for sp in species:
            x, u = sp["x"], sp["u"]
            Ep = torch.stack([self.gather(E[c], x, self.STAG_E[c]) for c in range(3)])
            Bp = torch.stack([self.gather(B1[c], x, self.STAG_B[c]) for c in range(3)])
            u1 = self.boris(u, Ep, Bp, sp["q"] * dt / (2 * sp["m"]))
            gam = torch.sqrt(1.0 + (u1 * u1).sum(0))
            x1 = torch.stack([x[d] + dt * u1[d] / (gam * self.d[d]) if d in self.active else x[d]
                              for d in range(3)])
            J = J + self.deposit(x, x1, u1, sp["q"], sp["w"])
            xw = torch.stack([torch.remainder(x1[d], self.n[d]) if d in self.active else x1[d]
                              for d in range(3)])
            out.append(dict(sp, x=xw, u=u1))
        B2 = B1 - 0.5 * dt * self.curl_plus(E)
        E2 = E + dt * (self.curl_minus(B2) - J)
        return E2, B2, out

    def field_energy(self, E, B):
        return 0.5 * ((E * E).sum() + (B * B).sum()) * self.dV


def from_case(case):
    """TorchPIC and initial tensors (E, B, species) of a cases.Case."""
    import numpy as np
    nx, ny, nz = case.gdims
    pic = TorchPIC(case.dim, case.gdims, case.dx, case.dt, case.order)
    E = torch.tensor(case.E.astype(np.float64).reshape(3, nz, ny, nx))
    B = torch.tensor(case.B.astype(np.float64).reshape(3, nz, ny, nx))
    species = []
    for s in case.species:
        c = s.cell.astype(np.int64)
        xi = np.zeros((3, s.n))
        if case.dim == 2:
            xi[1] = (c // nx) % ny + s.off[0]
            xi[2] = c // (nx * ny) + s.off[1]
        else:
            xi[0] = c % nx + s.off[0]
            xi[1] = (c // nx) % ny + s.off[1]
            xi[2] = c // (nx * ny) + s.off[2]
        species.append(dict(x=torch.tensor(xi), u=torch.tensor(s.u.astype(np.float64)),
                            q=s.q, m=s.m, w=s.w))
    return pic, E, B, species


def energy_gradient(case, nsteps: int):
    """W = final field energy after nsteps; returns (W, dW/dE0, dW/dB0, [dW/du0 per species])."""
    pic, E, B, species = from_case(case)
    E.requires_grad_(True)
    B.requires_grad_(True)
    for sp in species:
        sp["u"].requires_grad_(True)
    u0 = [sp["u"] for sp in species]
    e, b, sps = E, B, species
    for _ in range(nsteps):
        e, b, sps = pic.step(e, b, sps)
    W = pic.field_energy(e, b)
    grads = torch.autograd.grad(W, [E, B] + u0)
    return W.item(), grads[0].numpy(), grads[1].numpy(), [g.numpy() for g in grads[2:]]
