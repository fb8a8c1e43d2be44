"""Gradient of the final field energy through the GPU time steps.

W = 1/2 sum(E^2 + B^2) dV after N steps.  The forward pass keeps a full
device snapshot every ``every`` steps; the reverse pass restores each
snapshot in turn, recomputes its segment while keeping every step's state and
sort permutation, and runs the hand-written reverse step (psc_adjoint_step)
backwards through the segment.  The result is dW/dE^{1/2}, dW/dB^0 and
dW/du^0 of every particle (in the case's particle order).

``FieldEnergy`` exposes the same computation as a torch.autograd.Function of
the initial fields and momenta.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .psc import PscSim


def _seed(sim):
    torch = sim.torch
    lam = []
    for r, c in enumerate(sim.cases):
        E, B, _ = sim.fields[r]
        dV = c.dx[1] * c.dx[2] * (c.dx[0] if c.dim == 3 else 1.0)
        lam.append(dict(lE=(E * dV).contiguous(), lB=(B * dV).contiguous(),
                        loff=[torch.zeros(c.dim * sp.n, dtype=torch.float32, device=sim.device) for sp in c.species],
                        lu=[torch.zeros(3 * sp.n, dtype=torch.float32, device=sim.device) for sp in c.species]))
    return lam


def _state(sim):
    st = []
    for r, c in enumerate(sim.cases):
        E, B, _ = sim.fields[r]
        st.append(dict(E=E.clone(), B=B.clone(),   # the reverse step reads no ids
                       parts=[sim.device_particles(r, s, ids=False) for s in range(len(c.species))]))
    return st


class EnergyGradient:
    """Forward with checkpoints, then reverse; timings in milliseconds."""

    def __init__(self, cases, nsteps: int, every: int = 10, chunk: int = 0):
        self.sim = PscSim(cases, adjoint=True, chunk=chunk)
        self.nsteps, self.every = int(nsteps), int(every)

    def forward(self):
        sim, torch = self.sim, self.sim.torch
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        self.ckpts = []
        for k in range(self.nsteps):
            if k % self.every == 0:
                self.ckpts.append((k, sim.snapshot()))
            sim.step(1)
        b.record()
        torch.cuda.synchronize()
        self.forward_ms = a.elapsed_time(b)
        sim.check()
        d = sim.diagnostics()
        self.W = d[:, 0] + d[:, 1]
        return self.W

    def backward(self):
        sim, torch = self.sim, self.sim.torch
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        lam = _seed(sim)
        for k0, snap in reversed(self.ckpts):
            k1 = min(k0 + self.every, self.nsteps)
            sim.restore(snap)
            states = []
            for _ in range(k0, k1):
                st = _state(sim)
                sim.step(1)
                for r, c in enumerate(sim.cases):
                    st[r]["perm"] = [sim.get_perm(r, s) for s in range(len(c.species))]
                states.append(st)
            for st in reversed(states):
                sim.adjoint_step(st, lam)
        b.record()
        torch.cuda.synchronize()
        self.adjoint_ms = a.elapsed_time(b)
        sim.check()
        # map particle adjoints from the initial sorted order to case order
        out = []
        snap0 = self.ckpts[0][1]
        for r, c in enumerate(sim.cases):
            gE = lam[r]["lE"].cpu().numpy().reshape(3, -1)
            gB = lam[r]["lB"].cpu().numpy().reshape(3, -1)
            gU = []
            for s, sp in enumerate(c.species):
                ids = snap0[r]["parts"][s]["id"].cpu().numpy()
                g = np.empty((3, sp.n), np.float32)
                g[:, ids] = lam[r]["lu"][s].cpu().numpy().reshape(3, sp.n)
                gU.append(g)
            out.append((gE, gB, gU))
        return out


def energy_gradient(case, nsteps: int, every: int = 10, chunk: int = 0):
    """(W, dW/dE0, dW/dB0, [dW/du0 per species], forward_ms, adjoint_ms) of one run."""
    eg = EnergyGradient(case, nsteps, every, chunk)
    W = eg.forward()
    (gE, gB, gU), = eg.backward()
    return float(W[0]), gE, gB, gU, eg.forward_ms, eg.adjoint_ms


def _torch_function():
    import torch

    class FieldEnergy(torch.autograd.Function):
        """W(E0, B0, u0 of each species) = final field energy after nsteps.

        Inputs are float32 tensors with the case's layouts: E0, B0 (3, ncell)
        and u0 (3, n) per species; positions come from ``case``."""

        @staticmethod
        def forward(ctx, case, nsteps, every, E0, B0, *u0):
            c = dataclasses.replace(
                case, E=E0.detach().cpu().numpy().astype(np.float32).reshape(3, -1).copy(),
                B=B0.detach().cpu().numpy().astype(np.float32).reshape(3, -1).copy(),
                species=[dataclasses.replace(sp, u=u.detach().cpu().numpy().astype(np.float32).copy())
                         for sp, u in zip(case.species, u0)])
            eg = EnergyGradient(c, nsteps, every)
            W = eg.forward()
            ctx.eg = eg
            return torch.tensor(float(W[0]), dtype=torch.float64)

        @staticmethod
        def backward(ctx, gW):
            (gE, gB, gU), = ctx.eg.backward()
            g = float(gW)
            grads = [torch.from_numpy(gE * g), torch.from_numpy(gB * g)] + [torch.from_numpy(x * g) for x in gU]
            return (None, None, None, *grads)

    return FieldEnergy


def field_energy(case, nsteps: int, every: int, E0, B0, *u0):
    """Differentiable final field energy (see FieldEnergy)."""
    return _torch_function().apply(case, nsteps, every, E0, B0, *u0)
