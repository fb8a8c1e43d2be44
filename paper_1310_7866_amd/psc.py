"""Thin Python binding of ``libpsc.so`` (the C ABI in include/psc.h).

Argument marshalling only: PyTorch allocates the device buffers and supplies
the stream; every step of the particle-in-cell hot path runs in the HIP
kernels of the library.  There is no fallback: if the library is missing or
no GPU is present, construction raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence, Union

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; PSC_LIBRARY may name another build of the same sources
LIB_PATH = os.environ.get("PSC_LIBRARY") or os.path.join(HERE, "libpsc.so")

MAX_SPECIES = 4
B_HALF, E_FULL = 0, 1
DIAG_STRIDE = 10
DEV_NONFINITE, DEV_MOVE, DEV_KEY, DEV_OVERFULL = 1, 2, 4, 8

STATUS = {0: "PSC_OK", 1: "PSC_ERR_INVALID", 2: "PSC_ERR_CFL", 3: "PSC_ERR_LDS", 4: "PSC_ERR_HIP",
          5: "PSC_ERR_NONFINITE", 6: "PSC_ERR_PARTICLE", 7: "PSC_ERR_UNSUPPORTED", 8: "PSC_ERR_STATE"}

# every symbol include/psc.h declares
EXPORTS = ["psc_init_patches", "psc_workspace_size", "psc_bind", "psc_bind_static", "psc_load_particles",
           "psc_load_sorted", "psc_push_fields", "psc_push_particles", "psc_deposit_current", "psc_sort",
           "psc_sort_radix", "psc_step", "psc_get_particles", "psc_keys_to_cells", "psc_particle_count",
           "psc_front", "psc_sort_view", "psc_diagnostics", "psc_get_perm", "psc_marder", "psc_adjoint_step",
           "psc_adjoint_seed", "psc_set_launch", "psc_set_run_chunk", "psc_balance", "psc_partition",
           "psc_set_unit_order", "psc_hilbert_order", "psc_get_cell_offsets", "psc_set_particle_buffers",
           "psc_set_sort_outputs",
           "psc_check", "psc_status_string", "psc_last_error", "psc_destroy"]
LAUNCH_GRID, LAUNCH_QUEUE, LAUNCH_PARTITION = 0, 1, 2
RUN_ADJOINT = 1
RUN_VB = 2
RUN_TILE_FOLD = 4
ORDER_ROWMAJOR, ORDER_HILBERT = 0, 1


class PscError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class RunDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("gdims", C.c_int * 3), ("patch", C.c_int * 3),
                ("dx", C.c_double * 3), ("dt", C.c_double), ("order", C.c_int),
                ("n_species", C.c_int), ("q", C.c_double * 4), ("m", C.c_double * 4),
                ("w", C.c_double * 4), ("capacity", C.c_int64 * 4), ("flags", C.c_int)]


class AdjFwd(C.Structure):
    _fields_ = [("E", C.c_void_p), ("B", C.c_void_p), ("cell", C.c_void_p * 4), ("off", C.c_void_p * 4),
                ("u", C.c_void_p * 4), ("perm", C.c_void_p * 4), ("read_perm", C.c_void_p * 4),
                ("cell_start", C.c_void_p * 4), ("stride", C.c_int64 * 4)]


class AdjState(C.Structure):
    _fields_ = [("lE", C.c_void_p), ("lB", C.c_void_p), ("loff", C.c_void_p * 4), ("lu", C.c_void_p * 4)]


class RunBufs(C.Structure):
    _fields_ = [("E", C.c_void_p), ("B", C.c_void_p), ("J", C.c_void_p),
                ("cell", (C.c_void_p * 2) * 4), ("off", (C.c_void_p * 2) * 4),
                ("u", (C.c_void_p * 2) * 4), ("id", (C.c_void_p * 2) * 4)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpsc.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build()")
    L = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int, C.c_int64
    L.psc_init_patches.argtypes = [C.POINTER(RunDesc), i32, i32, C.POINTER(vp)]
    L.psc_workspace_size.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.psc_bind.argtypes = [vp, C.POINTER(RunBufs), i32, vp, vp]
    L.psc_bind_static.argtypes = [vp, C.POINTER(RunBufs), i32, vp]
    L.psc_load_particles.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp, vp]
    L.psc_load_sorted.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp, vp]
    L.psc_push_fields.argtypes = [vp, i32, vp]
    L.psc_push_particles.argtypes = [vp, vp]
    L.psc_deposit_current.argtypes = [vp, vp]
    L.psc_sort.argtypes = [vp, vp]
    L.psc_sort_radix.argtypes = [vp, vp]
    L.psc_marder.argtypes = [vp, vp, C.c_double, C.c_int, vp]
    L.psc_step.argtypes = [vp, i32, i32, vp]
    L.psc_get_particles.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
    L.psc_keys_to_cells.argtypes = [vp, i32, i64, vp, vp, vp]
    L.psc_particle_count.argtypes = [vp, i32, i32, C.POINTER(i64)]
    L.psc_front.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
    L.psc_sort_view.argtypes = [vp, i32, i32, C.POINTER(vp), C.POINTER(vp)]
    L.psc_diagnostics.argtypes = [vp, vp, vp, vp]
    L.psc_get_perm.argtypes = [vp, i32, i32, vp, vp]
    L.psc_adjoint_step.argtypes = [vp, C.POINTER(AdjFwd), C.POINTER(AdjState), vp]
    L.psc_adjoint_seed.argtypes = [vp, C.POINTER(AdjState), vp]
    L.psc_get_cell_offsets.argtypes = [vp, i32, i32, vp, vp]
    L.psc_set_particle_buffers.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp]
    L.psc_set_sort_outputs.argtypes = [vp, i32, i32, vp, vp, vp]
    L.psc_set_launch.argtypes = [vp, i32, i32, i32, i32, i32, vp]
    L.psc_set_run_chunk.argtypes = [vp, i32, i32, vp]
    L.psc_balance.argtypes = [vp, C.c_double, vp]
    L.psc_partition.argtypes = [C.POINTER(C.c_double), i32, C.POINTER(C.c_double), i32, C.POINTER(C.c_int32)]
    L.psc_set_unit_order.argtypes = [vp, i32, vp]
    L.psc_hilbert_order.argtypes = [i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.psc_check.argtypes = [vp, vp, C.POINTER(C.c_uint32), i32]
    L.psc_status_string.argtypes = [i32]
    L.psc_status_string.restype = C.c_char_p
    L.psc_last_error.argtypes = [vp, C.c_char_p, C.c_size_t]
    L.psc_destroy.argtypes = [vp]
    for name in EXPORTS:
        if name not in ("psc_status_string",):
            getattr(L, name).restype = i32
    _lib = L
    return L


def partition(loads: Sequence[float], caps: Sequence[float]) -> np.ndarray:
    """App. A greedy partition (host function of the library): patches per rank."""
    L = load_library()
    lo = np.ascontiguousarray(loads, dtype=np.float64)
    ca = np.ascontiguousarray(caps, dtype=np.float64)
    out = np.zeros(ca.size, np.int32)
    st = L.psc_partition(lo.ctypes.data_as(C.POINTER(C.c_double)), lo.size,
                         ca.ctypes.data_as(C.POINTER(C.c_double)), ca.size,
                         out.ctypes.data_as(C.POINTER(C.c_int32)))
    if st != 0:
        raise PscError(st, "psc_partition")
    return out


def hilbert_order(dim: int, np_: Sequence[int]) -> np.ndarray:
    """Patches of an np_[0] x np_[1] x np_[2] grid (x fastest) along the
    library's Hilbert curve: row-major patch indices in curve order (host
    function of the library)."""
    L = load_library()
    n = np.ascontiguousarray(np_, dtype=np.int32)
    out = np.zeros(int(n[0]) * int(n[1]) * int(n[2]), np.int32)
    st = L.psc_hilbert_order(int(dim), n.ctypes.data_as(C.POINTER(C.c_int32)),
                             out.ctypes.data_as(C.POINTER(C.c_int32)))
    if st != 0:
        raise PscError(st, "psc_hilbert_order")
    return out


def run_desc(case, capacity: Optional[Sequence[int]] = None, flags: int = 0) -> RunDesc:
    d = RunDesc()
    d.flags = int(flags) | (RUN_VB if getattr(case, "deposit", "esirkepov") == "vb" else 0)
    d.dim = case.dim
    for k in range(3):
        d.gdims[k] = int(case.gdims[k])
        d.patch[k] = int(case.patch[k])
        d.dx[k] = float(case.dx[k])
    d.dt = float(case.dt)
    d.order = int(case.order)
    d.n_species = len(case.species)
    for s, sp in enumerate(case.species):
        d.q[s], d.m[s], d.w[s] = sp.q, sp.m, sp.w
        d.capacity[s] = int(capacity[s] if capacity is not None else sp.n)
    return d


class PscSim:
    """One or more independent runs advanced together by the HIP library.

    ``cases``: a ``cases.Case`` or a list of them (a batch: one launch per
    kernel covers every run).  Buffers are torch tensors on ``device``.
    ``static_workspace``: bind with psc_bind_static (the library-held
    workspace) instead of a torch-allocated one.  ``tile_fold``: every run
    keeps per-patch current tiles folded by psc_deposit_current
    (PSC_RUN_TILE_FOLD) instead of adding its current into J in the particle
    kernel.
    """

    def __init__(self, cases, device: str = "cuda", with_ids: bool = True, chunk: int = 0,
                 adjoint: bool = False, static_workspace: bool = False, tile_fold: bool = False):
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("PscSim needs a GPU; the HIP library has no CPU path")
        self.L = load_library()
        self.cases = list(cases) if isinstance(cases, (list, tuple)) else [cases]
        self.device = torch.device(device)
        n_runs = len(self.cases)
        flags = (RUN_ADJOINT if adjoint else 0) | (RUN_TILE_FOLD if tile_fold else 0)
        descs = (RunDesc * n_runs)(*[run_desc(c, flags=flags) for c in self.cases])
        ctx = C.c_void_p()
        self._call(self.L.psc_init_patches(descs, n_runs, int(chunk), C.byref(ctx)), None)
        self.ctx = ctx
        nbytes = C.c_size_t()
        self._call(self.L.psc_workspace_size(self.ctx, C.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        if static_workspace:
            self.workspace = None
        else:
            self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
            ws_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        f32, i32 = torch.float32, torch.int32
        self.fields = []
        self.parts = []   # per run: per species: [set0, set1] of dict(cell, off, u, id)
        bufs = (RunBufs * n_runs)()
        self.field_blocks = []   # per run: one tensor holding E, B, J in turn
        for r, c in enumerate(self.cases):
            nc3 = 3 * c.ncell
            EBJ = torch.zeros(3 * nc3, dtype=f32, device=self.device)
            E, B, J = EBJ[:nc3], EBJ[nc3:2 * nc3], EBJ[2 * nc3:]
            E.copy_(torch.from_numpy(np.ascontiguousarray(c.E.reshape(-1), dtype=np.float32)))
            B.copy_(torch.from_numpy(np.ascontiguousarray(c.B.reshape(-1), dtype=np.float32)))
            self.field_blocks.append(EBJ)
            self.fields.append((E, B, J))
            bufs[r].E, bufs[r].B, bufs[r].J = E.data_ptr(), B.data_ptr(), J.data_ptr()
            per_sp = []
            for s, sp in enumerate(c.species):
                D = c.dim
                sets = []
                for k in range(2):
                    t = dict(cell=torch.empty(max(sp.n, 1), dtype=i32, device=self.device),
                             off=torch.empty(D * max(sp.n, 1), dtype=f32, device=self.device),
                             u=torch.empty(3 * max(sp.n, 1), dtype=f32, device=self.device),
                             id=torch.empty(max(sp.n, 1), dtype=i32, device=self.device) if with_ids else None)
                    sets.append(t)
                    bufs[r].cell[s][k] = t["cell"].data_ptr()
                    bufs[r].off[s][k] = t["off"].data_ptr()
                    bufs[r].u[s][k] = t["u"].data_ptr()
                    bufs[r].id[s][k] = t["id"].data_ptr() if with_ids else None
                per_sp.append(sets)
            self.parts.append(per_sp)
        if static_workspace:
            self._call(self.L.psc_bind_static(self.ctx, bufs, n_runs, self._stream()))
        else:
            self._call(self.L.psc_bind(self.ctx, bufs, n_runs, C.c_void_p(ws_ptr), self._stream()))
        self.with_ids = with_ids
        for r, c in enumerate(self.cases):
            for s, sp in enumerate(c.species):
                cell = torch.from_numpy(np.ascontiguousarray(sp.cell, dtype=np.int32)).to(self.device)
                off = torch.from_numpy(np.ascontiguousarray(sp.off, dtype=np.float32).reshape(-1)).to(self.device)
                u = torch.from_numpy(np.ascontiguousarray(sp.u, dtype=np.float32).reshape(-1)).to(self.device)
                gid = torch.arange(sp.n, dtype=i32, device=self.device)
                self.load(r, s, cell, off, u, gid)
                del cell, off, u, gid
        self.check()

    def load(self, r: int, s: int, cell, off, u, ids=None):
        """Load particles given as device tensors in geometric form (cell index,
        offsets (D*n), momenta (3*n), ids); sorts them by key on the device."""
        self.torch.cuda.synchronize()
        n = int(cell.numel())
        self._call(self.L.psc_load_particles(self.ctx, r, s, n, cell.data_ptr(), off.data_ptr(), u.data_ptr(),
                                             ids.data_ptr() if ids is not None else None, self._stream()))

    def load_sorted(self, r: int, s: int, key, off, u, ids=None):
        """Load particles already in sorted key order, as device_particles
        returns them (keys, offsets (D*n), momenta (3*n), ids); no sort."""
        n = int(key.numel())
        self._call(self.L.psc_load_sorted(self.ctx, r, s, n, key.data_ptr(), off.data_ptr(), u.data_ptr(),
                                          ids.data_ptr() if ids is not None else None, self._stream()))

    # -- plumbing ------------------------------------------------------------
    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _call(self, status: int, ctx="self"):
        if status != 0:
            msg = ""
            if ctx == "self" and getattr(self, "ctx", None):
                buf = C.create_string_buffer(512)
                self.L.psc_last_error(self.ctx, buf, 512)
                msg = buf.value.decode()
            raise PscError(status, msg)

    def close(self):
        if getattr(self, "ctx", None):
            self.torch.cuda.synchronize()
            self.L.psc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C ABI, call by call ------------------------------------------------
    def push_fields(self, op: int):
        self._call(self.L.psc_push_fields(self.ctx, op, self._stream()))

    def push_particles(self):
        self._call(self.L.psc_push_particles(self.ctx, self._stream()))

    def deposit_current(self):
        self._call(self.L.psc_deposit_current(self.ctx, self._stream()))

    def sort(self):
        self._call(self.L.psc_sort(self.ctx, self._stream()))

    def marder(self, d: float, ref=None, iters: int = 1):
        """Marder cleaning: E += d dt grad(div E - rho - ref); ref a device
        float64 tensor laid out like the gauss output of diagnostics()."""
        self._call(self.L.psc_marder(self.ctx, None if ref is None else ref.data_ptr(), float(d), int(iters),
                                     self._stream()))

    def sort_radix(self):
        """The same order by a general multi-pass radix sort (timing ablation)."""
        self._call(self.L.psc_sort_radix(self.ctx, self._stream()))

    def step(self, nsteps: int = 1, use_graph: bool = False):
        self._call(self.L.psc_step(self.ctx, int(nsteps), int(use_graph), self._stream()))

    def set_launch(self, mode: int, chunk: int = 0, workers: int = 0, threads: int = 0, run: int = 0):
        self._call(self.L.psc_set_launch(self.ctx, int(mode), int(chunk), int(workers), int(threads), int(run),
                                         self._stream()))

    def set_run_chunk(self, r: int, chunk: int):
        self._call(self.L.psc_set_run_chunk(self.ctx, int(r), int(chunk), self._stream()))

    def set_unit_order(self, order: int):
        self._call(self.L.psc_set_unit_order(self.ctx, int(order), self._stream()))

    def balance(self, cell_cost: float = 1.0):
        self._call(self.L.psc_balance(self.ctx, float(cell_cost), self._stream()))

    def check(self, clear: bool = False) -> int:
        word = C.c_uint32()
        st = self.L.psc_check(self.ctx, self._stream(), C.byref(word), int(clear))
        if st != 0:
            self._call(st)
        return int(word.value)

    def error_word(self, clear: bool = False) -> int:
        word = C.c_uint32()
        self.L.psc_check(self.ctx, self._stream(), C.byref(word), int(clear))
        return int(word.value)

    def front(self):
        f, p = C.c_int(), C.c_int()
        self._call(self.L.psc_front(self.ctx, C.byref(f), C.byref(p)))
        return f.value, p.value

    # -- read-back helpers (tests, diagnostics) -------------------------------
    def keys_to_cells(self, r: int, keys):
        torch = self.torch
        out = torch.empty_like(keys)
        self._call(self.L.psc_keys_to_cells(self.ctx, r, keys.numel(), keys.data_ptr(), out.data_ptr(),
                                            self._stream()))
        return out

    def particles(self, r: int, s: int):
        """Sorted-order particles of (run, species): dict of numpy arrays with
        'key', 'cell' (geometric), 'off' (D, n), 'u' (3, n), 'id'."""
        torch = self.torch
        c = self.cases[r]
        n = C.c_int64()
        self._call(self.L.psc_particle_count(self.ctx, r, s, C.byref(n)))
        n = n.value
        cell = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        off = torch.empty(c.dim * max(n, 1), dtype=torch.float32, device=self.device)
        u = torch.empty(3 * max(n, 1), dtype=torch.float32, device=self.device)
        ids = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        self._call(self.L.psc_get_particles(self.ctx, r, s, cell.data_ptr(), off.data_ptr(), u.data_ptr(),
                                            ids.data_ptr(), self._stream()))
        geo = self.keys_to_cells(r, cell[:n])
        torch.cuda.synchronize()
        return dict(key=cell[:n].cpu().numpy(), cell=geo.cpu().numpy(),
                    off=off[:c.dim * n].view(c.dim, n).cpu().numpy() if n else np.zeros((c.dim, 0), np.float32),
                    u=u[:3 * n].view(3, n).cpu().numpy() if n else np.zeros((3, 0), np.float32),
                    id=ids[:n].cpu().numpy())

    def front_buffer(self, r: int, s: int):
        """The particle buffer set written by the last push, in buffer order."""
        f, _ = self.front()
        c = self.cases[r]
        n = c.species[s].n
        t = self.parts[r][s][f]
        self.torch.cuda.synchronize()
        return dict(key=t["cell"][:n].cpu().numpy(),
                    cell=self.keys_to_cells(r, t["cell"][:n]).cpu().numpy(),
                    off=t["off"][:c.dim * n].view(c.dim, n).cpu().numpy(),
                    u=t["u"][:3 * n].view(3, n).cpu().numpy(),
                    id=t["id"][:n].cpu().numpy() if t["id"] is not None else None)

    def sort_view(self, r: int, s: int):
        """(perm, cell_start) of (run, species) as numpy arrays."""
        torch = self.torch
        p, cs = C.c_void_p(), C.c_void_p()
        self._call(self.L.psc_sort_view(self.ctx, r, s, C.byref(p), C.byref(cs)))
        n = self.cases[r].species[s].n
        nc = self.cases[r].ncell
        torch.cuda.synchronize()
        perm = np.empty(n, np.int32)
        cst = np.empty(nc + 1, np.int32)
        hip = C.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        if n:
            hip.hipMemcpy(perm.ctypes.data, p, perm.nbytes, 2)
        hip.hipMemcpy(cst.ctypes.data, cs, cst.nbytes, 2)
        return perm, cst

    def get_perm(self, r: int, s: int):
        """Device copy of the last sort's permutation of (run, species)."""
        n = self.cases[r].species[s].n
        out = self.torch.empty(max(n, 1), dtype=self.torch.int32, device=self.device)
        self._call(self.L.psc_get_perm(self.ctx, r, s, out.data_ptr(), self._stream()))
        return out[:n]

    def device_particles(self, r: int, s: int, ids: bool = True):
        """Sorted-order particles of (run, species) as device tensors
        (key int32 (n), off float32 (D*n), u float32 (3*n), id int32 (n)
        unless ids is False)."""
        torch = self.torch
        c = self.cases[r]
        n = c.species[s].n
        t = dict(key=torch.empty(max(n, 1), dtype=torch.int32, device=self.device),
                 off=torch.empty(c.dim * max(n, 1), dtype=torch.float32, device=self.device),
                 u=torch.empty(3 * max(n, 1), dtype=torch.float32, device=self.device))
        if ids:
            t["id"] = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        self._call(self.L.psc_get_particles(self.ctx, r, s, t["key"].data_ptr(), t["off"].data_ptr(),
                                            t["u"].data_ptr(), t["id"].data_ptr() if ids else None,
                                            self._stream()))
        return {k: v[:(c.dim * n if k == "off" else 3 * n if k == "u" else n)] for k, v in t.items()}

    def snapshot(self):
        """Device copy of the whole state (fields, sorted particles)."""
        snap = []
        for r, c in enumerate(self.cases):
            E, B, _ = self.fields[r]
            snap.append(dict(E=E.clone(), B=B.clone(),
                             parts=[self.device_particles(r, s) for s in range(len(c.species))]))
        return snap

    def restore(self, snap):
        """Put a snapshot back (restarts the context)."""
        for r, c in enumerate(self.cases):
            E, B, _ = self.fields[r]
            E.copy_(snap[r]["E"])
            B.copy_(snap[r]["B"])
            for s, p in enumerate(snap[r]["parts"]):
                self.load_sorted(r, s, p["key"], p["off"], p["u"], p["id"])

    def adjoint_step(self, fwd, lam):
        """One reverse step.  fwd: per run dict(E, B, parts=[dict(key, off, u)
        and optionally read_perm, cell_start, stride)], perm=[tensor]); lam:
        per run dict(lE, lB, loff=[...], lu=[...]) updated in place."""
        n_runs = len(self.cases)
        F = (AdjFwd * n_runs)()
        S = (AdjState * n_runs)()
        for r in range(n_runs):
            F[r].E, F[r].B = fwd[r]["E"].data_ptr(), fwd[r]["B"].data_ptr()
            S[r].lE, S[r].lB = lam[r]["lE"].data_ptr(), lam[r]["lB"].data_ptr()
            for s, p in enumerate(fwd[r]["parts"]):
                F[r].cell[s], F[r].off[s], F[r].u[s] = p["key"].data_ptr(), p["off"].data_ptr(), p["u"].data_ptr()
                F[r].perm[s] = fwd[r]["perm"][s].data_ptr()
                if p.get("read_perm") is not None:
                    F[r].read_perm[s] = p["read_perm"].data_ptr()
                if p.get("cell_start") is not None:
                    F[r].cell_start[s] = p["cell_start"].data_ptr()
                F[r].stride[s] = int(p.get("stride", 0))
                S[r].loff[s], S[r].lu[s] = lam[r]["loff"][s].data_ptr(), lam[r]["lu"][s].data_ptr()
        self._call(self.L.psc_adjoint_step(self.ctx, F, S, self._stream()))

    def cell_offsets(self, r: int, s: int):
        """Device copy of the current cell offsets of (run, species) (ncell + 1)."""
        out = self.torch.empty(self.cases[r].ncell + 1, dtype=self.torch.int32, device=self.device)
        self._call(self.L.psc_get_cell_offsets(self.ctx, r, s, out.data_ptr(), self._stream()))
        return out

    def set_particle_buffers(self, r: int, s: int, bset: int, bufs):
        """Point buffer set `bset` of (run, species) at bufs = dict(cell, off, u,
        id) (device tensors of the species' capacity)."""
        idp = bufs["id"].data_ptr() if bufs.get("id") is not None else None
        self._call(self.L.psc_set_particle_buffers(self.ctx, r, s, int(bset), bufs["cell"].data_ptr(),
                                                   bufs["off"].data_ptr(), bufs["u"].data_ptr(), idp,
                                                   self._stream()))

    def set_sort_outputs(self, r: int, s: int, perm=None, cs=None):
        """Direct the next sort's permutation (int32, capacity) and new cell
        offsets (int32, ncell + 1) of (run, species) to device tensors; both
        None returns to the workspace's arrays."""
        self._call(self.L.psc_set_sort_outputs(self.ctx, r, s, perm.data_ptr() if perm is not None else None,
                                               cs.data_ptr() if cs is not None else None, self._stream()))

    def adjoint_seed(self, lam):
        """Seed lam (per run dict(lE, lB, loff=[...], lu=[...]) of device
        tensors) for W = the current field energy: lE = E dV, lB = B dV,
        particle adjoints zero."""
        n_runs = len(self.cases)
        S = (AdjState * n_runs)()
        for r in range(n_runs):
            S[r].lE, S[r].lB = lam[r]["lE"].data_ptr(), lam[r]["lB"].data_ptr()
            for s, _ in enumerate(self.cases[r].species):
                S[r].loff[s], S[r].lu[s] = lam[r]["loff"][s].data_ptr(), lam[r]["lu"][s].data_ptr()
        self._call(self.L.psc_adjoint_seed(self.ctx, S, self._stream()))

    def field_arrays(self, r: int):
        self.torch.cuda.synchronize()
        E, B, J = self.fields[r]
        return E.cpu().numpy().reshape(3, -1), B.cpu().numpy().reshape(3, -1), J.cpu().numpy().reshape(3, -1)

    def diagnostics(self, with_gauss: bool = False):
        torch = self.torch
        n_runs = len(self.cases)
        out = torch.zeros(n_runs * DIAG_STRIDE, dtype=torch.float64, device=self.device)
        g = torch.zeros(sum(c.ncell for c in self.cases), dtype=torch.float64, device=self.device) if with_gauss else None
        self._call(self.L.psc_diagnostics(self.ctx, out.data_ptr(), g.data_ptr() if g is not None else None,
                                          self._stream()))
        torch.cuda.synchronize()
        d = out.cpu().numpy().reshape(n_runs, DIAG_STRIDE)
        return (d, g.cpu().numpy()) if with_gauss else d
