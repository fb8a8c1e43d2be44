"""Shared test helpers: compare GPU particle/field state with the oracle."""
from __future__ import annotations

import numpy as np


def gpu_positions(case, parts) -> np.ndarray:
    """Absolute positions in cell units (3, n) of GPU particles (x = 0 in 2-d)."""
    nx, ny, nz = case.gdims
    c = parts["cell"].astype(np.int64)
    i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
    xi = np.zeros((3, c.size))
    off = parts["off"].astype(np.float64)
    if case.dim == 2:
        xi[1] = j + off[0]
        xi[2] = k + off[1]
    else:
        xi[0] = i + off[0]
        xi[1] = j + off[1]
        xi[2] = k + off[2]
    return xi


def by_id(arr: np.ndarray, ids: np.ndarray) -> np.ndarray:
    out = np.empty_like(arr)
    out[..., ids] = arr
    return out


def periodic_diff(a: np.ndarray, b: np.ndarray, n: float) -> np.ndarray:
    d = a - b
    return d - n * np.round(d / n)


def particle_errors(case, gpu_parts, sim_oracle, s_index: int, vth: float):
    """(max position error in cells, max relative momentum error) per id."""
    xi_g = by_id(gpu_positions(case, gpu_parts), gpu_parts["id"])
    u_g = by_id(gpu_parts["u"].astype(np.float64), gpu_parts["id"])
    xi_o, u_o = sim_oracle.by_id(s_index)
    dpos = 0.0
    for d in (range(3) if case.dim == 3 else (1, 2)):
        dpos = max(dpos, np.abs(periodic_diff(xi_g[d], xi_o[d], case.gdims[d])).max(initial=0.0))
    scale = np.maximum(np.linalg.norm(u_o, axis=0), vth)
    du = (np.linalg.norm(u_g - u_o, axis=0) / scale).max(initial=0.0)
    return dpos, du
