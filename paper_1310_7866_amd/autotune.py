"""Launch-shape autotuner for the particle kernel.

For a context it times candidate launch shapes (workgroup size, particles
per lane, one workgroup per work item / persistent workgroups with per-XCD
queues / persistent workgroups over the App. A partition) and chunk sizes on
the live state during warm-up, keeps the fastest, and caches the choice in a
JSON file keyed by the architecture and an occupancy class (dimension,
order, patch size, particles per cell rounded to a power of two, number of
runs).  In a batch whose runs fall into several occupancy classes (patch
cells x particles-per-cell bucket) the chunk is then tuned per class: the
launch shape is one per context, the chunk is a per-run setting.
Optionally also picks the patch size by timing trial contexts.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

MODES = (0, 1, 2)
CHUNKS = (1024, 2048, 4096, 8192, 16384)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "psc_autotune.json")


def occupancy_class(cases) -> str:
    cs = cases if isinstance(cases, (list, tuple)) else [cases]
    c0 = cs[0]
    ppc = sum(c.n_particles for c in cs) / max(1, sum(c.ncell for c in cs))
    bucket = 2 ** int(round(math.log2(max(ppc, 1.0))))
    return f"d{c0.dim}o{c0.order}p{c0.patch[1]}x{c0.patch[2]}x{c0.patch[0]}ppc{bucket}r{len(cs)}"


def run_classes(cases) -> Dict[str, List[int]]:
    """Runs of a context grouped by occupancy class: cells per patch and
    particles per cell rounded to a power of two."""
    cs = cases if isinstance(cases, (list, tuple)) else [cases]
    groups: Dict[str, List[int]] = {}
    for r, c in enumerate(cs):
        ppc = c.n_particles / max(1, c.ncell)
        bucket = 2 ** int(round(math.log2(max(ppc, 1.0))))
        cells = c.patch[0] * c.patch[1] * c.patch[2]
        groups.setdefault(f"p{cells}ppc{bucket}", []).append(r)
    return groups


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _load(path: str) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path: str, data: Dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_push(sim, steps: int = 3) -> float:
    """Mean milliseconds of the particle kernel over `steps` full steps."""
    import torch
    from .psc import B_HALF, E_FULL
    stream = torch.cuda.current_stream()
    total = 0.0
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        sim.push_fields(B_HALF)
        a.record(stream)
        sim.push_particles()
        b.record(stream)
        sim.push_fields(B_HALF)
        sim.deposit_current()
        sim.push_fields(E_FULL)
        sim.sort()
        torch.cuda.synchronize()
        total += a.elapsed_time(b)
    return total / steps


THREADS = (256, 384, 512)
RUNS = (1, 2)


def tune(sim, cache: Optional[str] = DEFAULT_CACHE, steps: int = 2,
         modes: Sequence[int] = MODES, chunks: Sequence[int] = CHUNKS,
         threads: Sequence[int] = THREADS, runs: Sequence[int] = RUNS, force: bool = False):
    """Pick and apply the fastest launch shape for `sim`: first the workgroup
    size and particles per lane (persistent queue launch, 4096-particle
    chunks), then the launch mode and chunk size with those.  Returns
    (launch dict with mode, chunk, threads, run; its ms; table of every
    candidate's ms).  The state advances by the timed steps (use during
    warm-up)."""
    from .psc import PscError
    key = f"{_arch()}/{occupancy_class(sim.cases)}"
    data = _load(cache) if cache else {}
    groups = run_classes(sim.cases)
    if not force and key in data:
        e = data[key]
        launch = {k: e[k] for k in ("mode", "chunk", "threads", "run")}
        sim.set_launch(**launch)
        apply_class_chunks(sim, e.get("class_chunks", {}))
        return launch, e["ms"], e.get("table", {}), e.get("class_chunks", {})
    table = {}
    best = None

    def trial(launch):
        nonlocal best
        try:
            sim.set_launch(**launch)
        except PscError:
            return                              # shape not possible (LDS)
        sim.step(1)                             # settle (first launch of a shape)
        ms = time_push(sim, steps)
        table["{mode}/{chunk}/{threads}/{run}".format(**launch)] = ms
        if best is None or ms < best[1]:
            best = (dict(launch), ms)

    base_mode = 1 if 1 in modes else modes[0]
    base_chunk = 4096 if 4096 in chunks else chunks[0]
    for nt in threads:
        for run in runs:
            trial(dict(mode=base_mode, chunk=base_chunk, threads=nt, run=run))
    nt, run = best[0]["threads"], best[0]["run"]
    for mode in modes:
        for chunk in chunks:
            if (mode, chunk) != (base_mode, base_chunk):
                trial(dict(mode=mode, chunk=chunk, threads=nt, run=run))
    launch, ms = best
    sim.set_launch(**launch)
    # several occupancy classes in one context: the chunk of each class's
    # runs in turn, the largest classes first, the others at the best so far
    class_chunks = {}
    if len(groups) > 1:
        order = sorted(groups, key=lambda k: -sum(sim.cases[r].n_particles for r in groups[k]))
        for cls in order:
            best_ch, best_ms = launch["chunk"], ms
            for ch in chunks:
                if ch == launch["chunk"]:
                    continue
                for r in groups[cls]:
                    sim.set_run_chunk(r, ch)
                sim.step(1)
                t = time_push(sim, steps)
                table[f"class/{cls}/{ch}"] = t
                if t < best_ms:
                    best_ch, best_ms = ch, t
            for r in groups[cls]:
                sim.set_run_chunk(r, best_ch)
            class_chunks[cls] = best_ch
            ms = best_ms
    sim.check()
    if cache:
        data[key] = dict(launch, ms=ms, table=table, class_chunks=class_chunks)
        _save(cache, data)
    return launch, ms, table, class_chunks


def apply_class_chunks(sim, class_chunks: Dict[str, int]) -> None:
    """Set the chunk of every run of `sim` whose occupancy class has one."""
    for cls, runs in run_classes(sim.cases).items():
        if cls in class_chunks:
            for r in runs:
                sim.set_run_chunk(r, class_chunks[cls])


def tune_patch(make_cases, patches: Iterable[int], steps: int = 2, **kw):
    """Time trial contexts built by make_cases(patch) for each patch size;
    returns (best patch, {patch: ms})."""
    from .psc import PscSim
    import torch
    res = {}
    for p in patches:
        sim = PscSim(make_cases(p), with_ids=False, **kw)
        sim.step(1)
        res[p] = time_push(sim, steps)
        sim.close()
        del sim
        torch.cuda.empty_cache()
    best = min(res, key=res.get)
    return best, res
