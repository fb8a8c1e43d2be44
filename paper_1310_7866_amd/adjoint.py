"""Gradient of the final field energy through the GPU time steps.

W = 1/2 sum(E^2 + B^2) dV after N steps.  The forward pass keeps a full
device snapshot every ``every`` steps; the reverse pass seeds the adjoint
state in the library (psc_adjoint_seed), restores each snapshot in turn,
recomputes its segment while keeping every step's state and sort
permutation, and runs the hand-written reverse step (psc_adjoint_step)
backwards through the segment.  The result is dW/dE^{1/2}, dW/dB^0 and
dW/du^0 of every particle (in the case's particle order).

``FieldEnergy`` exposes the same computation as a torch.autograd.Function of
the initial fields and momenta; it keeps one context per (case, steps,
checkpoint interval), loads new inputs into it on the device, and returns
the gradients on the inputs' device.
"""
from __future__ import annotations

import numpy as np

from .psc import PscSim


class EnergyGradient:
    """Forward with checkpoints, then reverse; timings in milliseconds."""

    def __init__(self, cases, nsteps: int, every: int = 10, chunk: int = 0):
        self.sim = PscSim(cases, adjoint=True, chunk=chunk)
        self.nsteps, self.every = int(nsteps), int(every)
        sim, torch = self.sim, self.sim.torch
        # positions of the initial particles (fixed inputs) for reloading
        # new momenta, and the adjoint state, allocated once
        self._pos, self.lam = [], []
        for r, c in enumerate(sim.cases):
            self._pos.append([(torch.from_numpy(np.ascontiguousarray(sp.cell, dtype=np.int32)).to(sim.device),
                               torch.from_numpy(np.ascontiguousarray(sp.off, dtype=np.float32).reshape(-1))
                               .to(sim.device)) for sp in c.species])
            f32 = torch.float32
            self.lam.append(dict(lE=torch.empty(3 * c.ncell, dtype=f32, device=sim.device),
                                 lB=torch.empty(3 * c.ncell, dtype=f32, device=sim.device),
                                 loff=[torch.empty(c.dim * max(sp.n, 1), dtype=f32, device=sim.device)
                                       for sp in c.species],
                                 lu=[torch.empty(3 * max(sp.n, 1), dtype=f32, device=sim.device)
                                     for sp in c.species]))

    def set_initial(self, E0, B0, u0):
        """Restart from new initial fields and momenta (device tensors, float32,
        per run: E0, B0 of 3 * ncell values, u0 a list of (3, n) per species),
        positions as in the case."""
        sim, torch = self.sim, self.sim.torch
        for r, c in enumerate(sim.cases):
            E, B, _ = sim.fields[r]
            E.copy_(E0[r].reshape(-1))
            B.copy_(B0[r].reshape(-1))
            for s, sp in enumerate(c.species):
                cell, off = self._pos[r][s]
                u = u0[r][s].to(device=sim.device, dtype=torch.float32).reshape(-1).contiguous()
                ids = torch.arange(sp.n, dtype=torch.int32, device=sim.device)
                sim.load(r, s, cell, off, u, ids)

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

    def _ring(self):
        """every + 1 particle buffer sets per (run, species), allocated once:
        the recomputed steps of a segment each write their own set, so the
        reverse step reads a step's particles where its push read them."""
        if getattr(self, "_ring_bufs", None) is None:
            sim, torch = self.sim, self.sim.torch
            i32, f32 = torch.int32, torch.float32
            self._ring_bufs = [[[dict(cell=torch.empty(max(sp.n, 1), dtype=i32, device=sim.device),
                                      off=torch.empty(c.dim * max(sp.n, 1), dtype=f32, device=sim.device),
                                      u=torch.empty(3 * max(sp.n, 1), dtype=f32, device=sim.device),
                                      id=torch.empty(max(sp.n, 1), dtype=i32, device=sim.device)
                                      if sim.with_ids else None)
                                 for _ in range(self.every + 1)] for sp in c.species] for c in sim.cases]
        return self._ring_bufs

    def _sort_ring(self):
        """every + 1 (permutation, cell offsets) pairs per (run, species),
        allocated once: the sort of recomputed step j writes pair j + 1, which
        step j + 1 reads and the reverse step uses, with no copies."""
        if getattr(self, "_sort_bufs", None) is None:
            sim, torch = self.sim, self.sim.torch
            i32 = torch.int32
            self._sort_bufs = [[[dict(perm=torch.empty(max(sp.n, 1), dtype=i32, device=sim.device),
                                      cs=torch.empty(c.ncell + 1, dtype=i32, device=sim.device))
                                 for _ in range(self.every + 1)] for sp in c.species] for c in sim.cases]
        return self._sort_bufs

    def backward_device(self):
        """Reverse pass; per run (dW/dE0 (3, ncell), dW/dB0 (3, ncell),
        [dW/du0 (3, n) per species in case order]) as device tensors."""
        sim, torch = self.sim, self.sim.torch
        ring, sring = self._ring(), self._sort_ring()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        lam = self.lam
        sim.adjoint_seed(lam)
        for k0, snap in reversed(self.ckpts):
            k1 = min(k0 + self.every, self.nsteps)
            # the segment starts from its snapshot, loaded (sorted) into ring
            # set 0, with the workspace's permutation and offsets
            for r, c in enumerate(sim.cases):
                for s in range(len(c.species)):
                    sim.set_sort_outputs(r, s, None, None)
                    sim.set_particle_buffers(r, s, 0, ring[r][s][0])
            sim.restore(snap)
            states = []
            for j in range(k1 - k0):
                front, _ = sim.front()
                st = []
                for r, c in enumerate(sim.cases):
                    nc3 = 3 * c.ncell
                    EB = sim.field_blocks[r][:2 * nc3].clone()   # E and B of the step, one copy
                    parts = []
                    for s, sp in enumerate(c.species):
                        q = ring[r][s][j]
                        parts.append(dict(key=q["cell"], off=q["off"], u=q["u"], stride=sp.n,
                                          read_perm=sring[r][s][j]["perm"] if j else None,
                                          cell_start=sring[r][s][j]["cs"] if j else sim.cell_offsets(r, s)))
                        sim.set_particle_buffers(r, s, 1 - front, ring[r][s][j + 1])
                        sim.set_sort_outputs(r, s, sring[r][s][j + 1]["perm"], sring[r][s][j + 1]["cs"])
                    st.append(dict(E=EB[:nc3], B=EB[nc3:], parts=parts,
                                   perm=[sring[r][s][j + 1]["perm"][:sp.n] for s, sp in enumerate(c.species)]))
                sim.step(1)
                states.append(st)
            for st in reversed(states):
                sim.adjoint_step(st, lam)
        b.record()
        torch.cuda.synchronize()
        self.adjoint_ms = a.elapsed_time(b)
        sim.check()
        # back on the context's own buffers, at the initial state
        for r, c in enumerate(sim.cases):
            for s in range(len(c.species)):
                sim.set_sort_outputs(r, s, None, None)
                sim.set_particle_buffers(r, s, 0, sim.parts[r][s][0])
                sim.set_particle_buffers(r, s, 1, sim.parts[r][s][1])
        sim.restore(self.ckpts[0][1])
        # particle adjoints from the initial sorted order to case order
        out = []
        snap0 = self.ckpts[0][1]
        for r, c in enumerate(sim.cases):
            gU = []
            for s, sp in enumerate(c.species):
                ids = snap0[r]["parts"][s]["id"].long()
                g = torch.empty((3, sp.n), dtype=torch.float32, device=sim.device)
                g[:, ids] = lam[r]["lu"][s][:3 * sp.n].view(3, sp.n)
                gU.append(g)
            out.append((lam[r]["lE"].view(3, -1).clone(), lam[r]["lB"].view(3, -1).clone(), gU))
        return out

    def backward(self):
        """backward_device with numpy arrays."""
        return [(gE.cpu().numpy(), gB.cpu().numpy(), [g.cpu().numpy() for g in gU])
                for gE, gB, gU in self.backward_device()]


def energy_gradient(case, nsteps: int, every: int = 10, chunk: int = 0):
    """(W, dW/dE0, dW/dB0, [dW/du0 per species], forward_ms, adjoint_ms) of one run."""
    eg = EnergyGradient(case, nsteps, every, chunk)
    W = eg.forward()
    (gE, gB, gU), = eg.backward()
    return float(W[0]), gE, gB, gU, eg.forward_ms, eg.adjoint_ms


# contexts of FieldEnergy, keyed by (id(case), nsteps, every); the case is
# kept with its context so that its id is not reused while cached
_CONTEXTS = {}
_MAX_CONTEXTS = 4


def _context(case, nsteps: int, every: int) -> EnergyGradient:
    key = (id(case), int(nsteps), int(every))
    hit = _CONTEXTS.get(key)
    if hit is not None and hit[0] is case:
        return hit[1]
    while len(_CONTEXTS) >= _MAX_CONTEXTS:
        _, (_, old) = _CONTEXTS.popitem()
        old.sim.close()
    eg = EnergyGradient(case, nsteps, every)
    _CONTEXTS[key] = (case, eg)
    return eg


def _torch_function():
    import torch

    class FieldEnergy(torch.autograd.Function):
        """W(E0, B0, u0 of each species) = final field energy after nsteps.

        Inputs are float32 tensors with the case's layouts: E0, B0 (3, ncell)
        and u0 (3, n) per species; positions come from ``case``.  W and the
        gradients are on E0's device."""

        @staticmethod
        def forward(ctx, case, nsteps, every, E0, B0, *u0):
            eg = _context(case, nsteps, every)
            dev = eg.sim.device
            eg.set_initial([E0.detach().to(dev, torch.float32)], [B0.detach().to(dev, torch.float32)],
                           [[u.detach() for u in u0]])
            W = eg.forward()
            ctx.eg = eg
            ctx.like = [(t.shape, t.device) for t in (E0, B0, *u0)]
            return torch.tensor(float(W[0]), dtype=torch.float64, device=E0.device)

        @staticmethod
        def backward(ctx, gW):
            (gE, gB, gU), = ctx.eg.backward_device()
            g = gW.to(gE.device, torch.float32)
            grads = [gE * g, gB * g] + [x * g for x in gU]
            return (None, None, None, *[t.reshape(shape).to(dev) for t, (shape, dev) in zip(grads, ctx.like)])

    return FieldEnergy


def field_energy(case, nsteps: int, every: int, E0, B0, *u0):
    """Differentiable final field energy (see FieldEnergy)."""
    return _torch_function().apply(case, nsteps, every, E0, B0, *u0)
