"""Benchmark of the particle-in-cell hot path on one MI355X.

Workload (default): the 3-d periodic counter-streaming electron Weibel
setup, 256^3 cells, 32 electrons per cell in two beams at +-0.3c along z
with v_th = 0.05c, immobile ions, 1st-order shape, float32 cell-index +
offset particles, 8^3 patches -- 536,870,912 particles.  A step is one full
pass of the hot path in the order of the paper's optimized time step: B
half step, fused particle kernel (gather, Boris, move, Esirkepov deposit),
B half step, current fold, E full step, sort.  Inputs are synthetic and
seeded, resident in HBM before the timed region.

Prints one JSON line: whole-step particle throughput (particle pushes per
second over complete steps), the roofline of the dominant kernel (the fused
particle kernel) from HIP events recorded on its stream inside the timed
region, and the double-precision oracle timed on a bounded sample on the
host (one thread and every thread).  Extra keys: the same measurement on the
2-d Harris sheet, the adjoint, the batched runs and the sort ablation.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# launch shapes chosen by the autotuner on MI355X, per occupancy class
TUNED = os.path.join(ROOT, "paper_1310_7866_amd", "tuned_gfx950.json")
# non-packed FP32 vector issue: 256 CUs x 64 lanes x 2.4 GHz (FMA = 2 flop)
VALU_PEAK_TFLOPS = 256 * 64 * 2.4e9 * 2 / 1e12
# wave64 VALU instructions per second: each CU issues one per clock over its
# four 16-lane SIMDs (one wave instruction takes four cycles on a SIMD)
VALU_ISSUE_PEAK = 256 * 2.4e9


def algorithmic_bytes(case) -> float:
    """Minimum HBM bytes of one particle-kernel launch: every particle's state
    read and written once (int32 cell + D float32 offsets + 3 float32 momenta),
    plus each patch's E and B read and its 3-component current tile written."""
    D = case.dim
    per_particle = 2 * (4 + 4 * D + 12)
    return case.n_particles * per_particle + case.ncell * (6 + 3) * 4


# every n-th particle of a workload for the oracle's baseline and error legs
CPU_THIN = {"weibel3d": 32, "harris2d": 1, "thermal2d": 1, "harris2d_small": 1, "thermal2d_1024x512": 4}


def make_case(name: str):
    from paper_1310_7866_amd import cases
    if name == "harris2d":
        return cases.harris2d()
    if name == "thermal2d":
        return cases.thermal2d()
    if name == "weibel3d":
        return cases.weibel3d()
    if name == "harris2d_small":
        return cases.harris2d(ny=256, nz=256, ppc=64, seed=5050, steps=50)
    if name == "thermal2d_1024x512":   # the 2-d order-1 kernel at full size (16.8 M particles)
        import dataclasses
        return dataclasses.replace(cases.thermal2d(ny=1024, nz=512, ppc=16, order=1, patch=32), name=name)
    raise SystemExit(f"unknown workload {name}")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, thin: int, batch_error: bool = False, tune_cache=None):
    """The oracle as it stands on every `thin`-th particle of the workload
    (full grid) for one complete step, timed on this host with one thread
    and with every thread the process may use.  Both legs use a copy of the
    oracle compiled here for this host (gcc -O3 -march=native, float64
    with -ffp-contract=off, no fast-math: the same arithmetic as the tests'
    build); the threaded leg is built with OpenMP, whose particle loop gives
    each thread its own current array and whose field updates split the
    grid.  The sort stays single-threaded in both.  The first leg's state
    after the step gives the GPU path's error."""
    import tempfile
    from oracle import oracle as O
    from paper_1310_7866_amd import cases
    sample = cases.thin(case, thin)
    tmp = os.path.join(os.environ.get("TMPDIR", tempfile.gettempdir()), f"psc_oracle_{os.getpid()}")
    libs = {1: O.build_host_tuned(tmp, openmp=False), 0: O.build_host_tuned(tmp, openmp=True)}
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    legs, first = {}, None
    for want in (1, threads):
        O.use_library(libs[1 if want == 1 else 0])
        used = O.set_threads(want)
        sim = O.OracleSim(sample)
        t0 = time.perf_counter()
        sim.push_b_half()
        t1 = time.perf_counter()
        sim.push_particles()
        t2 = time.perf_counter()
        sim.push_b_half()
        sim.push_e_full()
        t3 = time.perf_counter()
        sim.sort()
        t4 = time.perf_counter()
        legs[used] = dict(value=sample.n_particles / (t4 - t0), seconds=t4 - t0, particle_loop_s=t2 - t1,
                          fields_s=(t1 - t0) + (t3 - t2), sort_s=t4 - t3)
        print(f"[bench] oracle on {used} thread(s): {t4 - t0:.2f} s per step", file=sys.stderr, flush=True)
        if first is None:
            first = sim
        else:
            del sim
    O.use_library(None)
    err = oracle_error(sample, first)
    extra = {}
    if batch_error:
        extra["error_of_batched_path"] = batched_oracle_error(tune_cache=tune_cache)
    top = max(legs)
    return dict(**extra, value=legs[top]["value"], unit="particle pushes/s", cores=top, kind="oracle",
                sample=f"1 full step of every {thin}th particle ({sample.n_particles} particles) "
                       f"of the {case.name} workload on the full "
                       f"{'x'.join(str(g) for g in case.gdims if g > 1)} grid, float64",
                cpu_model=cpu_model(), compiler="gcc " + " ".join(O.HOST_TUNED_FLAGS) + " [-fopenmp]",
                threads={str(k): v for k, v in sorted(legs.items())},
                error_of_gpu_path=err)


def oracle_error(sample, osim, g=None, run=0):
    """The float32 GPU path against the float64 oracle after the same full
    step on the same sample: largest position difference (cells), largest
    momentum difference relative to the species' largest |u|, and largest
    field differences relative to the largest oracle value.  g: a context
    already stepped that holds the sample as run `run` (a batch), else one
    is made for the sample alone."""
    import numpy as np
    from paper_1310_7866_amd.psc import PscSim
    own = g is None
    if own:
        g = PscSim(sample, with_ids=True)
        g.step(1)
        g.check()
    nx, ny, nz = sample.gdims
    dpos, du = 0.0, 0.0
    for s in range(len(sample.species)):
        p = g.particles(run, s)
        ids = p["id"].astype(np.int64)
        c = p["cell"].astype(np.int64)
        idx = (c % nx, (c // nx) % ny, c // (nx * ny))
        dims = (1, 2) if sample.dim == 2 else (0, 1, 2)
        order = np.argsort(osim.species[s].ids)
        xo, uo = osim.species[s].xi[:, order], osim.species[s].u[:, order]
        for k, d in enumerate(dims):
            xg = np.empty(ids.size)
            xg[ids] = idx[d] + p["off"][k].astype(np.float64)
            diff = xg - xo[d]
            diff -= sample.gdims[d] * np.round(diff / sample.gdims[d])
            dpos = max(dpos, float(np.abs(diff).max(initial=0.0)))
        ug = np.empty((3, ids.size))
        ug[:, ids] = p["u"].astype(np.float64)
        du = max(du, float(np.abs(ug - uo).max(initial=0.0) / max(np.abs(uo).max(initial=0.0), 1e-30)))
    E, B, J = g.field_arrays(run)
    rel = lambda a, b: float(np.abs(a.astype(np.float64).ravel() - b).max() / max(np.abs(b).max(), 1e-30))
    out = dict(steps=1, max_position_cells=dpos, max_momentum_rel=du,
               E_rel=rel(E, osim.E), B_rel=rel(B, osim.B), J_rel=rel(J, osim.J))
    if own:
        g.close()
    return out


def batched_oracle_error(n_runs: int = 64, thin: int = 4, tune_cache=None):
    """The batched path against the oracle: three runs of the batch
    workload (its first, middle and last, every `thin`-th particle) in one
    context with the batch's launch shape, one full step replayed from a HIP
    graph, each run against the oracle stepping it alone; the largest errors
    over the runs (as in oracle_error)."""
    from oracle import oracle as O
    from paper_1310_7866_amd import autotune as AT
    from paper_1310_7866_amd import cases
    from paper_1310_7866_amd.psc import PscSim
    cs = cases.twostream_batch(n_runs=n_runs, seed=4064)
    # the batch's launch shape from the tuning cache (the library's default without an entry)
    entry = AT._load(tune_cache or AT.DEFAULT_CACHE).get(f"{AT._arch()}/{AT.occupancy_class(cs)}")
    sub = [cases.thin(cs[i], thin) for i in (0, n_runs // 2, n_runs - 1)]
    osims = []
    for c in sub:
        o = O.OracleSim(c)
        o.step(1)
        osims.append(o)
    g = PscSim(sub, with_ids=True)
    if entry:
        g.set_launch(**{k: entry[k] for k in ("mode", "chunk", "threads", "run")})
    g.step(1, use_graph=True)
    g.check()
    errs = [oracle_error(c, o, g, r) for r, (c, o) in enumerate(zip(sub, osims))]
    g.close()
    out = {k: max(e[k] for e in errs) for k in errs[0] if k != "steps"}
    out.update(steps=1, runs=f"runs 0, {n_runs // 2}, {n_runs - 1} of the batch, every {thin}th particle, "
                              f"{sum(c.n_particles for c in sub)} particles, in one context with the batch's launch shape")
    return out


def sort_ablation_leg(sim, stream, steps: int):
    """The per-step sort by a general multi-pass radix sort of the keys
    (psc_sort_radix) in place of the single-pass move-code counting sort,
    timed on the same state after the timed region."""
    import torch
    from paper_1310_7866_amd.psc import B_HALF, E_FULL
    ev = lambda: torch.cuda.Event(enable_timing=True)
    pairs = [(ev(), ev()) for _ in range(steps)]
    for k in range(steps):
        sim.push_fields(B_HALF)
        sim.push_particles()
        sim.push_fields(B_HALF)
        sim.deposit_current()
        sim.push_fields(E_FULL)
        pairs[k][0].record(stream)
        sim.sort_radix()
        pairs[k][1].record(stream)
    torch.cuda.synchronize()
    sim.check()
    return dict(radix_sort_ms=sum(a.elapsed_time(b) for a, b in pairs) / steps, steps=steps)


def supercell_leg(sizes=(4, 8, 12, 16, 24, 32, 48), steps: int = 10):
    """Patch (super-cell) size sweep of the Harris workload: every patch
    stages its fields and accumulates its current in LDS, so small patches
    amortise the tile loads over few particles and large ones hold fewer
    workgroups per compute unit.  Default launch shape, one context each."""
    import torch
    from paper_1310_7866_amd import cases
    from paper_1310_7866_amd.psc import B_HALF, E_FULL, PscError, PscSim
    case = cases.harris2d()
    out = {}
    for P in sizes:
        case.patch = (1, P, P)
        try:
            sim = PscSim(case, with_ids=False)
        except PscError as e:
            out[f"{P}x{P}"] = dict(error=str(e))
            continue
        stream = torch.cuda.current_stream()
        sim.step(2)
        ev = lambda: torch.cuda.Event(enable_timing=True)
        pe = [(ev(), ev()) for _ in range(steps)]
        t0, t1 = ev(), ev()
        torch.cuda.synchronize()
        t0.record(stream)
        for k in range(steps):
            sim.push_fields(B_HALF)
            pe[k][0].record(stream)
            sim.push_particles()
            pe[k][1].record(stream)
            sim.push_fields(B_HALF)
            sim.deposit_current()
            sim.push_fields(E_FULL)
            sim.sort()
        t1.record(stream)
        torch.cuda.synchronize()
        sim.check()
        push_ms = sum(a.elapsed_time(b) for a, b in pe) / steps
        step_ms = t0.elapsed_time(t1) / steps
        out[f"{P}x{P}"] = dict(push_ms=round(push_ms, 4), step_ms=round(step_ms, 4),
                               push_pushes_per_s=case.n_particles / (push_ms / 1e3))
        print(f"[bench] patch {P}x{P}: push {push_ms:.3f} ms, step {step_ms:.3f} ms", file=sys.stderr, flush=True)
        sim.close()
        del sim
        torch.cuda.empty_cache()
    case.patch = (1, 32, 32)
    return dict(workload=f"harris2d 1024x512, order 2, {case.n_particles} particles", steps=steps, patches=out)


def marder_leg(steps: int = 2000, every: int = 50, frac: float = 0.5):
    """Gauss-law drift of a long float32 run (Harris 256x256, order 2) with
    and without Marder cleaning every `every` steps (coefficient `frac` of
    the stability bound, reference = the residual at the start), and the
    cost of the cleaning.  Drift: max over nodes of |G^n - G^0|, G the Gauss
    residual div E - rho in units of the reference density."""
    import numpy as np
    import torch
    from paper_1310_7866_amd import cases
    from paper_1310_7866_amd.psc import PscSim
    c = cases.harris2d(ny=256, nz=256, ppc=64, order=2, patch=32, seed=5050, steps=steps)
    d = frac * 2.0 / (c.dt * (4.0 / c.dx[1] ** 2 + 4.0 / c.dx[2] ** 2))
    out = dict(workload=f"harris2d 256x256, order 2, {c.n_particles} particles, {steps} steps",
               every=every, d=d, d_over_bound=frac)
    for clean in (False, True):
        sim = PscSim(c, with_ids=False)
        _, g0 = sim.diagnostics(with_gauss=True)
        ref = torch.from_numpy(g0).cuda()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for k in range(0, steps, every):
            sim.step(min(every, steps - k), use_graph=True)
            if clean:
                sim.marder(d, ref=ref)
        b.record()
        torch.cuda.synchronize()
        sim.check()
        _, g = sim.diagnostics(with_gauss=True)
        tag = "with_marder" if clean else "without"
        out[tag] = dict(max_drift=float(np.abs(g - g0).max()), rms_drift=float(np.sqrt(np.mean((g - g0) ** 2))),
                        ms=a.elapsed_time(b))
        print(f"[bench] marder {tag}: drift {out[tag]['max_drift']:.3e}, {out[tag]['ms']:.1f} ms", file=sys.stderr,
              flush=True)
        sim.close()
        del sim
        torch.cuda.empty_cache()
    out["overhead"] = out["with_marder"]["ms"] / out["without"]["ms"] - 1.0
    return out


def deposit_leg(steps: int = 10):
    """1st-order particle kernel with the Esirkepov and the Villasenor-Buneman
    deposit on the same thermal 2-d workload (1024x512 cells, 16 electron-ion
    pairs per cell, v_th 0.1 / 0.02) and the 3-d Weibel setup at 128^3."""
    import torch
    from paper_1310_7866_amd import cases
    from paper_1310_7866_amd.psc import B_HALF, E_FULL, PscSim
    out = {}
    for case in (cases.thermal2d(ny=1024, nz=512, ppc=16, order=1, patch=32),
                 cases.weibel3d(ppc=32, order=1, patch=8, nxyz=(128, 128, 128))):
        row = {}
        for dep in ("esirkepov", "vb"):
            case.deposit = dep
            sim = PscSim(case, with_ids=False)
            stream = torch.cuda.current_stream()
            sim.step(3)
            ev = lambda: torch.cuda.Event(enable_timing=True)
            pe = [(ev(), ev()) for _ in range(steps)]
            torch.cuda.synchronize()
            for k in range(steps):
                sim.push_fields(B_HALF)
                pe[k][0].record(stream)
                sim.push_particles()
                pe[k][1].record(stream)
                sim.push_fields(B_HALF)
                sim.deposit_current()
                sim.push_fields(E_FULL)
                sim.sort()
            torch.cuda.synchronize()
            sim.check()
            ms = sum(a.elapsed_time(b) for a, b in pe) / steps
            row[dep] = dict(push_ms=round(ms, 4), pushes_per_s=case.n_particles / (ms / 1e3))
            print(f"[bench] {case.name} {dep}: push {ms:.3f} ms", file=sys.stderr, flush=True)
            sim.close()
            del sim
            torch.cuda.empty_cache()
        case.deposit = "esirkepov"
        out[f"{case.name} {'x'.join(str(g) for g in case.gdims if g > 1)}, {case.n_particles} particles"] = row
    return out


def deposit_ablation_leg(steps: int = 10):
    """The 1st-order Villasenor-Buneman particle kernel on the thermal 2-d
    workload (1024x512 cells, 16 electron-ion pairs per cell) with 4x4, 8x8
    and 16x16 super-cells, one particle per lane.  The library it runs is
    whichever PSC_LIBRARY names: built with -DPSC_FRAMES=0 (per-lane LDS
    atomics), -DPSC_JCOPIES=16 (redundant tiles) and -DPSC_MIX=1 (lanes
    spread over the item's cells) it measures the shared-memory deposit
    variants against the frames of the default build.  A super-cell size
    whose tiles do not fit in LDS is reported as null."""
    import torch
    from paper_1310_7866_amd import cases
    from paper_1310_7866_amd.psc import B_HALF, E_FULL, PscError, PscSim
    out = {}
    for P in (4, 8, 16):
        case = cases.thermal2d(ny=1024, nz=512, ppc=16, order=1, patch=P)
        case.deposit = "vb"
        sim = None
        try:
            sim = PscSim(case, with_ids=False)
            sim.set_launch(mode=1, chunk=4096, threads=256, run=1)
        except PscError as e:
            print(f"[bench] ablation {P}x{P}: {e}", file=sys.stderr, flush=True)
            out[f"{P}x{P}"] = None
            if sim is not None:
                sim.close()
            continue
        stream = torch.cuda.current_stream()
        sim.step(3)
        ev = lambda: torch.cuda.Event(enable_timing=True)
        pe = [(ev(), ev()) for _ in range(steps)]
        torch.cuda.synchronize()
        for k in range(steps):
            sim.push_fields(B_HALF)
            pe[k][0].record(stream)
            sim.push_particles()
            pe[k][1].record(stream)
            sim.push_fields(B_HALF)
            sim.deposit_current()
            sim.push_fields(E_FULL)
            sim.sort()
        torch.cuda.synchronize()
        sim.check()
        ms = sum(a.elapsed_time(b) for a, b in pe) / steps
        out[f"{P}x{P}"] = dict(push_ms=round(ms, 4), pushes_per_s=case.n_particles / (ms / 1e3))
        print(f"[bench] ablation {P}x{P}: push {ms:.3f} ms", file=sys.stderr, flush=True)
        sim.close()
        del sim
        torch.cuda.empty_cache()
    return dict(workload=f"thermal2d 1024x512, order 1, VB deposit, {case.n_particles} particles, run 1",
                library=os.environ.get("PSC_LIBRARY", "in-tree"), supercells=out)


def adjoint_leg(every: int = 10, nsteps: int = 50):
    """Gradient of the final field energy on the 256 x 256 double Harris sheet
    (64 particles per cell at n = 1, 2nd order, 32 x 32 patches): forward with
    checkpoints every `every` steps, then the hand-written reverse."""
    from paper_1310_7866_amd import cases
    from paper_1310_7866_amd.adjoint import EnergyGradient
    c = cases.harris2d(ny=256, nz=256, ppc=64, order=2, patch=32, seed=5050, steps=nsteps)
    eg = EnergyGradient(c, nsteps, every)
    eg.forward()           # warm-up (kernel loading, graph-free)
    eg.backward()
    W = eg.forward()
    eg.backward()
    return dict(workload=f"harris2d 256x256, order 2, {c.n_particles} particles, {nsteps} steps, "
                         f"checkpoints every {every}",
                forward_ms=eg.forward_ms, adjoint_ms=eg.adjoint_ms,
                adjoint_over_forward=eg.adjoint_ms / eg.forward_ms, W=float(W[0]))


def batch_leg(steps: int = 10, n_runs: int = 64, tune_cache=None, retune=False):
    """64 independent two-stream runs (uneven grids, ragged patches) advanced
    in one context (autotuned launch shape, HIP-graph replay) vs the same runs
    advanced one after another in their own contexts."""
    import numpy as np
    import torch
    from paper_1310_7866_amd import cases
    from paper_1310_7866_amd.autotune import apply_class_chunks, tune
    from paper_1310_7866_amd.psc import PscSim
    cs = cases.twostream_batch(n_runs=n_runs, seed=4064)
    n = sum(c.n_particles for c in cs)
    batch = PscSim(cs, with_ids=False)
    launch, _, table, class_chunks = tune(batch, cache=tune_cache, steps=2, force=retune)
    batch.step(2, use_graph=True)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    batch.step(steps, use_graph=True)
    b.record()
    torch.cuda.synchronize()
    batch.check()
    batch_ms = a.elapsed_time(b)
    del batch
    torch.cuda.empty_cache()
    # the same runs, one context each, one after another
    plain_ms = 0.0
    for c in cs:
        sim = PscSim(c, with_ids=False)
        sim.step(2)
        torch.cuda.synchronize()
        a.record()
        sim.step(steps)
        b.record()
        torch.cuda.synchronize()
        plain_ms += a.elapsed_time(b)
        sim.close()
        del sim
    torch.cuda.empty_cache()
    # agreement of batched vs alone after the same steps on a few runs
    dev = 0.0
    pick = [0, n_runs // 2, n_runs - 1]
    sub = [cs[i] for i in pick]
    bt = PscSim(sub)
    bt.set_launch(**launch)
    apply_class_chunks(bt, class_chunks)
    bt.step(steps, use_graph=True)
    for r, c in enumerate(sub):
        al = PscSim(c)
        al.step(steps)
        pa, pb = al.particles(0, 0), bt.particles(r, 0)
        oa, ob = np.argsort(pa["id"]), np.argsort(pb["id"])
        dev = max(dev, float(np.abs(pa["u"][:, oa] - pb["u"][:, ob]).max()))
        al.close()
    bt.close()
    return dict(workload=f"{n_runs} two-stream runs, {n} particles, "
                         f"{sum(c.ncell for c in cs)} cells, order 1",
                launch=launch, class_chunks=class_chunks, steps=steps,
                batched_pushes_per_s=n * steps / (batch_ms / 1e3),
                plain_pushes_per_s=n * steps / (plain_ms / 1e3),
                batched_over_plain=plain_ms / batch_ms,
                max_abs_du_vs_alone=dev)


def measure(case, args, sort_ablation: bool):
    """Warm-up and timed steps of one workload in its own context: whole-step
    throughput, the particle kernel's and the sort's mean duration from HIP
    events on the stream they run on, and the particle kernel's roofline."""
    import torch
    from paper_1310_7866_amd.psc import PscSim, B_HALF, E_FULL
    print(f"[bench] workload {case.name}: gdims={case.gdims} order={case.order} patch={case.patch} "
          f"particles={case.n_particles}", file=sys.stderr, flush=True)
    sim = PscSim(case, with_ids=False, chunk=args.chunk)
    if args.unit_order:
        from paper_1310_7866_amd.psc import ORDER_HILBERT, ORDER_ROWMAJOR
        sim.set_unit_order(ORDER_HILBERT if args.unit_order == "hilbert" else ORDER_ROWMAJOR)
    stream = torch.cuda.current_stream()
    launch = None
    if args.launch:
        mode, chunk, threads, run = (int(x) for x in args.launch.split(","))
        launch = dict(mode=mode, chunk=chunk, threads=threads, run=run)
        sim.set_launch(**launch)
    elif not args.no_tune:
        from paper_1310_7866_amd.autotune import tune
        launch, ms, _, _ = tune(sim, cache=args.tune_cache, steps=2, force=args.retune)
        print(f"[bench] autotuned launch {launch} ({ms:.3f} ms)", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        sim.step(1)
    sim.check()

    ev = lambda: torch.cuda.Event(enable_timing=True)
    push_ev = [(ev(), ev()) for _ in range(args.steps)]
    sort_ev = [(ev(), ev()) for _ in range(args.steps)]
    t_start, t_end = ev(), ev()
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for k in range(args.steps):
        sim.push_fields(B_HALF)
        push_ev[k][0].record(stream)
        sim.push_particles()
        push_ev[k][1].record(stream)
        sim.push_fields(B_HALF)
        sim.deposit_current()
        sim.push_fields(E_FULL)
        sort_ev[k][0].record(stream)
        sim.sort()
        sort_ev[k][1].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    sim.check()

    total_ms = t_start.elapsed_time(t_end)
    push_ms = sum(a.elapsed_time(b) for a, b in push_ev) / args.steps
    sort_ms = sum(a.elapsed_time(b) for a, b in sort_ev) / args.steps
    ablation = sort_ablation_leg(sim, stream, min(args.steps, 10)) if sort_ablation else None
    n = case.n_particles
    abytes = algorithmic_bytes(case)
    achieved_gbs = abytes / (push_ms / 1e3) / 1e9
    roof = dict(bound="hbm", achieved=round(achieved_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved_gbs / HBM_PEAK_GBS, 4), traffic=None,
                algorithmic_bytes=abytes, kernel_ms=push_ms)
    # hardware counters of this kernel source at this launch shape, if recorded
    roofs = None
    counters = _recorded_counters(case, launch)
    if counters is not None:
        tb = counters["bytes_per_launch"]
        roof.update(traffic=tb, traffic_gbs=round(tb / (push_ms / 1e3) / 1e9, 1),
                    traffic_frac=round(tb / (push_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                    traffic_over_algorithmic=round(tb / abytes, 3))
        valu_rate = counters["valu_per_launch"] / (push_ms / 1e3)
        roofs = {"hbm_frac": roof["frac"],
                 "valu_issue": {"achieved_instr_per_s": valu_rate, "peak_instr_per_s": VALU_ISSUE_PEAK,
                                "frac": round(valu_rate / VALU_ISSUE_PEAK, 4)},
                 "counters": counters["source"]}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return dict(value=n * args.steps / (total_ms / 1e3), ms_per_step=total_ms / args.steps, launch=launch,
                push_kernel_ms=push_ms, push_kernel_pushes_per_s=n / (push_ms / 1e3), sort_ms=sort_ms,
                wall_s_timed=wall, roofline=roof, roofs=roofs,
                sort_ablation=(dict(ablation, counting_sort_ms=sort_ms,
                                    radix_over_counting=ablation["radix_sort_ms"] / sort_ms) if ablation else None))


def workload_label(case) -> str:
    return (f"{case.name} {'x'.join(str(g) for g in case.gdims if g > 1)} cells, order {case.order}, "
            f"patches {'x'.join(str(p) for p, g in zip(case.patch, case.gdims) if g > 1)}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="weibel3d", choices=("weibel3d", "harris2d", "thermal2d", "harris2d_small",
                                                                      "thermal2d_1024x512"))
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--cpu-thin", type=int, default=0,
                    help="oracle baseline on every n-th particle (0: 32 for weibel3d, 1 for the 2-d workloads)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the Harris, adjoint, batch and sort-ablation legs")
    ap.add_argument("--only", choices=("adjoint", "batch", "supercells", "marder", "deposit", "ablation"),
                    default=None,
                    help="run only the adjoint or the batch leg and print its JSON")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--launch", default="", help="fixed launch shape mode,chunk,threads,run (skips tuning)")
    ap.add_argument("--tune-cache", default=TUNED, help="autotuner cache (JSON) to read and extend")
    ap.add_argument("--retune", action="store_true", help="time every launch shape again")
    ap.add_argument("--unit-order", choices=("hilbert", "rowmajor"), default=None,
                    help="order in which patches are handed out to the particle kernel's workgroups "
                         "(default: the library's, row-major)")
    ap.add_argument("--calibrate", action="store_true",
                    help="first run a 1 GiB fill and a 1 GiB device copy (reference kernels of known "
                         "traffic for hardware-counter runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the particle path has no multi-GPU code "
              "(its sharding is a design, not an implementation); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.only == "adjoint":
        print(json.dumps({"adjoint": adjoint_leg()}))
        return
    if args.only == "batch":
        print(json.dumps({"batched": batch_leg(tune_cache=args.tune_cache, retune=args.retune)}))
        return
    if args.only == "supercells":
        print(json.dumps({"supercells": supercell_leg()}))
        return
    if args.only == "marder":
        print(json.dumps({"marder": marder_leg()}))
        return
    if args.only == "deposit":
        print(json.dumps({"deposit": deposit_leg()}))
        return
    if args.only == "ablation":
        print(json.dumps({"deposit_ablation": deposit_ablation_leg()}))
        return

    if args.calibrate:
        n = 256 * 1024 * 1024                      # float32 -> 1 GiB
        src = torch.ones(n, dtype=torch.float32, device="cuda")   # fill: writes 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)                                             # copy: reads and writes 1 GiB
        torch.cuda.synchronize()
        print(f"[bench] calibration fill + copy of {4 * n} bytes", file=sys.stderr, flush=True)
        del src, dst
        torch.cuda.empty_cache()

    case = make_case(args.workload)
    res = measure(case, args, sort_ablation=not args.no_extras)
    out = {
        "metric": "particle pushes/sec (gather+push+deposit) and % HBM roofline; adjoint/forward time",
        "value": res["value"],
        "unit": "particle pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload_label(case), "particles": case.n_particles, "cells": case.ncell,
                   "order": case.order, "patch": list(case.patch), "parallelism": "single GPU",
                   "launch": res["launch"], "unit_order": args.unit_order or "rowmajor"},
        "push_kernel_ms": res["push_kernel_ms"],
        "push_kernel_pushes_per_s": res["push_kernel_pushes_per_s"],
        "sort_ms": res["sort_ms"],
        "wall_s_timed": res["wall_s_timed"],
        "roofline": res["roofline"],
    }
    if res["roofs"] is not None:
        out["roofs"] = res["roofs"]
    if res["sort_ablation"] is not None:
        out["sort_ablation"] = res["sort_ablation"]
    if not args.no_extras:
        if args.workload != "harris2d":
            print("[bench] harris2d leg", file=sys.stderr, flush=True)
            hc = make_case("harris2d")
            hr = measure(hc, args, sort_ablation=False)
            out["harris2d"] = dict(workload=workload_label(hc), particles=hc.n_particles,
                                   pushes_per_s=hr["value"], ms_per_step=hr["ms_per_step"],
                                   push_kernel_ms=hr["push_kernel_ms"], sort_ms=hr["sort_ms"],
                                   launch=hr["launch"], roofline=hr["roofline"], roofs=hr["roofs"])
            del hc
        print("[bench] adjoint leg", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_leg()
        print("[bench] batch leg", file=sys.stderr, flush=True)
        out["batched"] = batch_leg(tune_cache=args.tune_cache, retune=args.retune)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_thin or CPU_THIN.get(case.name, 1),
                                           batch_error=not args.no_extras, tune_cache=args.tune_cache)
    print(json.dumps(out))


def push_source_hash() -> str:
    """Hash of the code the particle kernel is compiled from: its own file,
    the device helpers, and the data structures of the internal header (the
    launcher declarations after them do not change the kernel), with
    comments and white space removed so that editing a comment keeps it."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_1310_7866_amd", "csrc")
    texts = []
    for name in ("psc_push.hip", "psc_device.h"):
        with open(os.path.join(csrc, name)) as f:
            texts.append(f.read())
    with open(os.path.join(csrc, "psc_internal.h")) as f:
        texts.append(f.read().split("// launchers (defined in the .hip files)")[0])
    h = hashlib.sha256()
    for text in texts:
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def _recorded_counters(case, launch):
    """HBM bytes and VALU instructions per particle-kernel launch from the
    hardware-counter record of this workload, if it was taken on the current
    kernel source with the same launch shape."""
    path = os.path.join(ROOT, "profiles", f"counters_{case.name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != push_source_hash() or rec.get("launch") != launch:
        return None
    return rec


if __name__ == "__main__":
    main()
