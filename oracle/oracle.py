"""ctypes front end of the double-precision oracle (psc_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  It shares nothing with the HIP library.

``OracleSim`` holds one run in float64 with absolute particle positions in
cell units and advances it with the time step of fig. psc_new:
B half step, particle loop (gather, Boris, move, Esirkepov deposit),
B half step, E full step, stable sort by patch-major cell key.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "psc_oracle.c"), os.path.join(_HERE, "psc_oracle_adjoint.c")]
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle into oracle/liboracle.so (plain gcc, -O2, FP64)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    srcs = [s for s in _SRC if os.path.exists(s)]
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("d", C.c_double * 3),
                ("dt", C.c_double), ("order", C.c_int), ("vb", C.c_int)]


def build_host_tuned(out_dir: str, openmp: bool) -> str:
    """Compile a copy of the oracle for timing it on the host that runs
    this call: gcc -O3 -march=native (this host's instruction set), still
    float64 with -ffp-contract=off; with ``openmp`` its particle loop and
    field updates run on every thread (see psc_oracle.c).  Returns the path
    of the library and leaves the default build alone."""
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "liboracle_omp.so" if openmp else "liboracle_1t.so")
    srcs = [s for s in _SRC if os.path.exists(s)]
    cmd = ["gcc", *HOST_TUNED_FLAGS, *(["-fopenmp"] if openmp else []), "-o", out] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    return out


HOST_TUNED_FLAGS = ["-O3", "-march=native", "-std=c99", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off"]

_lib = None


def use_library(path: Optional[str]):
    """Route the following oracle calls to the library at ``path`` (a
    build_host_tuned copy), or back to the default build (None)."""
    global _lib
    _lib = None if path is None else _bind(C.CDLL(path))


def set_threads(n: int) -> int:
    """Threads of the loaded oracle's parallel loops (1 unless it was built
    with OpenMP); returns the count in effect."""
    return int(lib().orc_set_threads(int(n)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or any(
                os.path.getmtime(s) > os.path.getmtime(_LIB) for s in _SRC if os.path.exists(s)):
            build()
        _lib = _bind(C.CDLL(_LIB))
    return _lib


def _bind(L):
    dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    g = C.POINTER(_Grid)
    L.orc_bspline.argtypes = [C.c_int, C.c_double]
    L.orc_bspline.restype = C.c_double
    L.orc_interp.argtypes = [g, dp, dp, dp]
    L.orc_interp.restype = C.c_double
    L.orc_boris.argtypes = [dp, dp, dp, C.c_double]
    L.orc_deposit.argtypes = [g, dp, dp, dp, C.c_double, C.c_double]
    L.orc_deposit_vb.argtypes = [g, dp, dp, dp, C.c_double, C.c_double]
    L.orc_push_particles.argtypes = [g, C.c_long, dp, dp, dp, dp, dp, C.c_double, C.c_double, C.c_double]
    L.orc_push_b.argtypes = [g, dp, dp, C.c_double]
    L.orc_push_e.argtypes = [g, dp, dp, C.c_void_p, C.c_double]
    L.orc_div_e.argtypes = [g, dp, dp]
    L.orc_marder.argtypes = [g, dp, dp, C.c_double]
    L.orc_div_b.argtypes = [g, dp, dp]
    L.orc_deposit_rho.argtypes = [g, C.c_long, dp, C.c_double, dp]
    L.orc_patch_keys.argtypes = [g, ip, ip]
    L.orc_stable_sort.argtypes = [C.c_long, ip, C.c_int32, ip]
    L.orc_stable_sort.restype = C.c_int
    L.orc_cell_of.argtypes = [g, dp]
    L.orc_cell_of.restype = C.c_long
    L.orc_field_energy.argtypes = [g, dp]
    L.orc_field_energy.restype = C.c_double
    L.orc_kinetic_energy.argtypes = [g, C.c_long, dp, C.c_double, C.c_double]
    L.orc_kinetic_energy.restype = C.c_double
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_set_threads.restype = C.c_int
    if hasattr(L, "orc_adjoint_step"):
        _bind_adjoint(L, g, dp, ip)
    return L


def _bind_adjoint(L, g, dp, ip):
    L.orc_adjoint_step.argtypes = [g, C.c_int, C.POINTER(C.c_long), C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_void_p), dp, dp, dp, dp, C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), dp, dp, dp]


def grid(dim: int, n: Sequence[int], d: Sequence[float], dt: float, order: int, vb: bool = False) -> _Grid:
    g = _Grid()
    g.vb = int(bool(vb))
    g.dim = dim
    for i in range(3):
        g.n[i] = int(n[i])
        g.d[i] = float(d[i])
    g.dt = float(dt)
    g.order = int(order)
    return g


def bspline(order: int, s: float) -> float:
    return lib().orc_bspline(order, float(s))


STAG_E = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5]])
STAG_B = np.array([[0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])


class OracleSpecies:
    def __init__(self, name, q, m, w, xi, u, ids):
        self.name, self.q, self.m, self.w = name, float(q), float(m), float(w)
        self.xi = np.ascontiguousarray(xi, dtype=np.float64)   # (3, n) cell units
        self.u = np.ascontiguousarray(u, dtype=np.float64)     # (3, n)
        self.ids = np.ascontiguousarray(ids, dtype=np.int64)

    @property
    def n(self):
        return self.xi.shape[1]


class OracleSim:
    """One periodic run in float64, built from a ``cases.Case``."""

    def __init__(self, case, sort_initial: bool = True):
        self.case = case
        self.dim = case.dim
        self.g = grid(case.dim, case.gdims, case.dx, case.dt, case.order,
                      vb=getattr(case, "deposit", "esirkepov") == "vb")
        self.nc = case.ncell
        self.E = case.E.astype(np.float64).reshape(-1).copy()
        self.B = case.B.astype(np.float64).reshape(-1).copy()
        self.J = np.zeros(3 * self.nc)
        nx, ny, nz = case.gdims
        self.species: List[OracleSpecies] = []
        for s in case.species:
            c = s.cell.astype(np.int64)
            i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
            xi = np.zeros((3, s.n))
            if case.dim == 2:
                xi[1] = j + s.off[0].astype(np.float64)
                xi[2] = k + s.off[1].astype(np.float64)
            else:
                xi[0] = i + s.off[0].astype(np.float64)
                xi[1] = j + s.off[1].astype(np.float64)
                xi[2] = k + s.off[2].astype(np.float64)
            self.species.append(OracleSpecies(s.name, s.q, s.m, s.w, xi, s.u, np.arange(s.n)))
        self.key_of_cell = patch_keys(self.g, case.patch)
        if sort_initial:
            self.sort()

    # -- pieces of the step ------------------------------------------------
    def push_b_half(self):
        lib().orc_push_b(C.byref(self.g), self.E, self.B, 0.5 * self.g.dt)

    def push_e_full(self):
        lib().orc_push_e(C.byref(self.g), self.E, self.B, self.J.ctypes.data, self.g.dt)

    def push_particles(self):
        self.J[:] = 0.0
        for s in self.species:
            lib().orc_push_particles(C.byref(self.g), s.n, s.xi, s.u, self.E, self.B, self.J,
                                     s.q, s.m, s.w)

    def keys(self, s: OracleSpecies) -> np.ndarray:
        return self.key_of_cell[self.cells(s)]

    def cells(self, s: OracleSpecies) -> np.ndarray:
        nx, ny, nz = self.case.gdims
        idx = [np.floor(s.xi[d]).astype(np.int64) % self.case.gdims[d] if (self.dim == 3 or d > 0)
               else np.zeros(s.n, np.int64) for d in range(3)]
        return idx[0] + nx * (idx[1] + ny * idx[2])

    def sort(self):
        for s in self.species:
            perm = stable_sort(self.keys(s), self.nc)
            s.xi = np.ascontiguousarray(s.xi[:, perm])
            s.u = np.ascontiguousarray(s.u[:, perm])
            s.ids = s.ids[perm]

    def step(self, nsteps: int = 1, sort: bool = True):
        for _ in range(nsteps):
            self.push_b_half()
            self.push_particles()
            self.push_b_half()
            self.push_e_full()
            if sort:
                self.sort()

    # -- diagnostics --------------------------------------------------------
    def rho(self) -> np.ndarray:
        r = np.zeros(self.nc)
        for s in self.species:
            lib().orc_deposit_rho(C.byref(self.g), s.n, np.ascontiguousarray(s.xi), s.q * s.w, r)
        return r

    def div_e(self) -> np.ndarray:
        out = np.zeros(self.nc)
        lib().orc_div_e(C.byref(self.g), self.E, out)
        return out

    def div_b(self) -> np.ndarray:
        out = np.zeros(self.nc)
        lib().orc_div_b(C.byref(self.g), self.B, out)
        return out

    def gauss(self) -> np.ndarray:
        return self.div_e() - self.rho()

    def marder(self, d: float, ref: Optional[np.ndarray] = None, iters: int = 1):
        """Marder's cleaning: E += d dt grad(F), F = Gauss residual - ref."""
        for _ in range(iters):
            F = self.gauss()
            if ref is not None:
                F = F - ref
            lib().orc_marder(C.byref(self.g), self.E, np.ascontiguousarray(F), float(d))

    def field_energy(self):
        return (lib().orc_field_energy(C.byref(self.g), self.E),
                lib().orc_field_energy(C.byref(self.g), self.B))

    def kinetic_energy(self):
        return [lib().orc_kinetic_energy(C.byref(self.g), s.n, s.u, s.m, s.w) for s in self.species]

    def by_id(self, s_index: int):
        """(xi, u) of a species reordered by particle id."""
        s = self.species[s_index]
        order = np.argsort(s.ids)
        return s.xi[:, order], s.u[:, order]


def patch_keys(g: _Grid, patch: Sequence[int]) -> np.ndarray:
    n = g.n[0] * g.n[1] * g.n[2]
    out = np.empty(n, np.int32)
    lib().orc_patch_keys(C.byref(g), np.array(patch, np.int32), out)
    return out


def stable_sort(keys: np.ndarray, nkeys: int) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.int32)
    perm = np.empty(keys.size, np.int32)
    if lib().orc_stable_sort(keys.size, keys, int(nkeys), perm) != 0:
        raise ValueError("key out of range")
    return perm


def interp(g: _Grid, F: np.ndarray, xi: Sequence[float], stag: Sequence[float]) -> float:
    return lib().orc_interp(C.byref(g), np.ascontiguousarray(F, np.float64),
                            np.asarray(xi, np.float64), np.asarray(stag, np.float64))


def boris(u, E, B, qdt_2m) -> np.ndarray:
    uu = np.array(u, np.float64)
    lib().orc_boris(uu, np.asarray(E, np.float64), np.asarray(B, np.float64), float(qdt_2m))
    return uu


def deposit(g: _Grid, xi0, xi1, qw, vx=0.0) -> np.ndarray:
    n = g.n[0] * g.n[1] * g.n[2]
    J = np.zeros(3 * n)
    lib().orc_deposit(C.byref(g), J, np.asarray(xi0, np.float64), np.asarray(xi1, np.float64),
                      float(qw), float(vx))
    return J


def deposit_vb(g: _Grid, xi0, xi1, qw, vx=0.0) -> np.ndarray:
    """Villasenor-Buneman current of one 1st-order particle (path cut at faces)."""
    n = g.n[0] * g.n[1] * g.n[2]
    J = np.zeros(3 * n)
    lib().orc_deposit_vb(C.byref(g), J, np.asarray(xi0, np.float64), np.asarray(xi1, np.float64),
                         float(qw), float(vx))
    return J


def rho_of(g: _Grid, xi: np.ndarray, qw: float) -> np.ndarray:
    n = g.n[0] * g.n[1] * g.n[2]
    r = np.zeros(n)
    xi = np.ascontiguousarray(np.asarray(xi, np.float64).reshape(3, -1))
    lib().orc_deposit_rho(C.byref(g), xi.shape[1], xi, float(qw), r)
    return r


def push_b(g: _Grid, E: np.ndarray, B: np.ndarray, h: float) -> None:
    lib().orc_push_b(C.byref(g), E, B, float(h))


def push_e(g: _Grid, E: np.ndarray, B: np.ndarray, J: Optional[np.ndarray], h: float) -> None:
    lib().orc_push_e(C.byref(g), E, B, None if J is None else J.ctypes.data, float(h))


def div_e(g: _Grid, E: np.ndarray) -> np.ndarray:
    out = np.zeros(E.size // 3)
    lib().orc_div_e(C.byref(g), np.ascontiguousarray(E, np.float64), out)
    return out


def div_b(g: _Grid, B: np.ndarray) -> np.ndarray:
    out = np.zeros(B.size // 3)
    lib().orc_div_b(C.byref(g), np.ascontiguousarray(B, np.float64), out)
    return out
