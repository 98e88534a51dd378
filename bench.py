"""Benchmark of the NeuralFVM time step on one MI355X.

One benchmark step is one full time step of the hot path (destruction half
step, explicit update, Poisson right-hand side, multigrid-preconditioned
pressure solve to the residual target, projection, destruction half step) over
the whole grid, with all fields resident in device memory.

Default workload: the ventilated room at its largest size, 10 x 4 x 3 m on
1024 x 512 x 256 cells (134M), 8-24 seeded solid blocks, supply vent under
the ceiling and exhaust at the floor, 9 multigrid levels, mixed precision
(FP32 scalars and level-0 sweeps, BF16 coarse levels, FP64 velocity,
pressure, residual and projection), pressure solved to a relative residual
of 1e-6 every step.

Prints one JSON line (rank 0).  Only one GPU is used: --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, vendor figure

WORKLOADS = {
    "channel3d": "3D heated channel 256x64x64, 7 levels",
    "channel2d": "2D turbulent channel 256x64, 6 levels",
    "room": "3D ventilated room 10x4x3 m on 512x256x128 cells with seeded blocks, 8 levels",
    "bigroom": "3D ventilated room 10x4x3 m on 1024x512x256 cells (134M) with seeded blocks, "
               "9 levels",
    "open_channel_128": "open channel at 5 mm, 128x128x128 (L = 0.64 m), 8 levels",
    "open_channel_512": "open channel at 5 mm, 512x128x128 (L = 2.56 m), 8 levels",
    "open_channel_2048": "open channel at 5 mm, 2048x128x128 (L = 10.24 m), 8 levels",
}

# The paper's GPU wall times for 100 steps of its open channel at 5 mm with
# slice-based stencils (Sec. 3.3, Table 1; RTX PRO 5000 Blackwell, precision
# and multigrid iteration count not stated), by streamwise cell count.
PAPER_TABLE1_GPU_S = {128: 5.5, 512: 22.8, 2048: 140.7}


# kernel sources whose hash identifies the build the committed counter
# summaries were taken with
KERNEL_SOURCES = ("k_mg.hip", "k_physics.hip", "nfvm_device.hpp", "nfvm_internal.hpp")
PROFILE_FILES = {
    ("channel3d", "mixed"): "kernels_channel3d_256x64x64_mixed.md",
    ("room", "mixed"): "kernels_room_512x256x128_mixed.md",
    ("bigroom", "mixed"): "kernels_bigroom_1024x512x256_mixed.md",
}

# Unfused per-operator byte model of the rest of a step, per cell (each
# operand read once and each result written once at its storage precision):
# the explicit update, the two destruction half steps, the right-hand side
# and the projection.  The cycle's model is model_cycle_bytes below.
MODEL_STEP_B = {"fp64": 344.0, "fp32": 172.0, "mixed": 190.0}
# kernels of the pressure solve (the rest of a step is the physics kernels)
SOLVE_KERNELS = ("smooth0", "smooth0_zero", "restrict0", "prolong0", "fcg_apply", "fcg_update",
                 "smooth_coarse", "restrict_coarse", "prolong_coarse", "bottom", "fcg_start",
                 "finalize", "smooth0_pair")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2603_21869_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, precision: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload; None when there is none or when the kernel
    sources changed since the counters were taken."""
    name = PROFILE_FILES.get((workload, precision))
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return None, None
    traffic, sha = {}, None
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 3 and parts[0] == "traffic":
                traffic[parts[1]] = float(parts[2])
            elif len(parts) == 2 and parts[0] == "source_sha256":
                sha = parts[1]
    if sha != kernel_source_hash():
        return None, name + " (stale: kernel sources changed)"
    return traffic.get(kernel), name


# V-cycle shape of the room workloads: three pre- and post-sweeps on the
# finest level and six on every coarser one (the solid blocks make the
# rediscretised coarse operators the weak part of the cycle; measured on the
# 1024x512x256 room in mixed precision: V(2,2) 13.8 iterations and 81 ms per
# step, V(3,3) with 4 coarse sweeps 10.1 / 76.5 ms, with 6 9.1 / 74.2 ms,
# V(4,4) with 6 8.5 / 77.6 ms)
ROOM_CYCLE = dict(nu1=3, nu2=3, nu_coarse=6)


def smoothing_of(case) -> str:
    """The V-cycle shape of a case in words."""
    s = f"V({case.nu1},{case.nu2}) damped Jacobi"
    if case.nu_coarse:
        s += f", {case.nu_coarse}+{case.nu_coarse} sweeps on the coarse levels"
    return s


def coarse_storage_of(case) -> str:
    from paper_2603_21869_amd import cases as C
    if case.precision != C.PREC_MIXED:
        return "as level 0"
    lim = case.coarse_fp32_cells or 131072
    if lim >= 2**31 - 1:
        return "BF16 on every coarse level"
    return f"FP32 on coarse levels of >= {lim} cells, BF16 below (LDS bottom levels in FP32)"


def model_cycle_bytes(case) -> float:
    """Unfused per-operator byte model of one preconditioned iteration of a
    case, in bytes per fine cell: on a level with nu sweeps per side each
    sweep moves 3 values per cell (x, b read, x written), the residual 3, the
    restriction 1 1/8 and the prolongation and correction 2 1/8 (values per
    cell of that level, at its storage size: the level-0 type on level 0 and
    on coarse levels of at least coarse_fp32_cells cells in mixed precision,
    the coarse type below); the coarsest solve is left out; the outer
    iteration moves 5 values per fine cell (z read, p, x and r updated) in
    the outer type."""
    from paper_2603_21869_amd import cases as C
    s0, sc, so = {C.PREC_FP64: (8, 8, 8), C.PREC_FP32: (4, 4, 4),
                  C.PREC_MIXED: (4, 2, 8)}[case.precision]
    lim = case.coarse_fp32_cells or 131072
    n = list(case.n)
    total = 0.0
    N0 = float(case.ncells)
    for l in range(case.n_levels - 1):
        cells = float(n[0] * n[1] * n[2])
        nu = case.nu1 + case.nu2 if l == 0 or not case.nu_coarse else 2 * case.nu_coarse
        size = s0 if l == 0 or (case.precision == C.PREC_MIXED and cells >= lim) else sc
        total += (3 * nu + 6.25) * size * cells / N0
        n = [max(1, k // 2) if a < case.dim else k for a, k in enumerate(n)]
    return total + 5 * so


def make_case(name: str, precision: int, tol: float):
    from paper_2603_21869_amd import cases as C
    if name == "channel3d":
        return C.channel3d(precision=precision, tol=tol)
    if name == "channel2d":
        return C.channel2d(precision=precision, tol=tol)
    if name == "room":
        return C.room3d(precision=precision, tol=tol).copy(**ROOM_CYCLE)
    if name == "bigroom":
        return C.room3d(1024, 512, 256, n_levels=9, precision=precision, tol=tol,
                        n_steps=100).copy(**ROOM_CYCLE)
    if name.startswith("open_channel_"):
        return C.open_channel(int(name.rsplit("_", 1)[1]), precision=precision, tol=tol)
    raise SystemExit(f"unknown workload {name}")


def timed_steps(g, steps: int):
    """steps time steps of grid g between two device synchronisations."""
    import torch
    from paper_2603_21869_amd import nfvm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s, stats = g.step(steps, allow=(nfvm.NFVM_OK, nfvm.NFVM_E_NOTCONV, nfvm.NFVM_E_DIVERGED))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, stats, s


def profile_steps(g, steps: int):
    """The same steps with HIP events around every kernel launch (stream
    launches: the events would split the graphs).  Returns the summed event
    time and, per kernel, launches, seconds and mean algorithmic bytes."""
    from paper_2603_21869_amd import nfvm
    nfvm.nfvm_profile(g.h, (1 << len(nfvm.KERNELS)) - 1)
    sec, _, _ = timed_steps(g, steps)
    prof = {name: nfvm.nfvm_profile_read(g.h, kid) for kid, name in enumerate(nfvm.KERNELS)}
    nfvm.nfvm_profile(g.h, 0)
    return sec, prof


def run_gpu(case, steps: int, warmup: int, stream: int, warm_start: bool = False):
    """Throughput of `steps` steps on a fresh grid after `warmup` steps."""
    from paper_2603_21869_amd import nfvm
    g = nfvm.Grid(case, stream=stream)
    nfvm.nfvm_set_option(g.h, nfvm.NFVM_OPT_WARM_START, 1.0 if warm_start else 0.0)
    if warmup:
        g.step(warmup, allow=(nfvm.NFVM_OK, nfvm.NFVM_E_NOTCONV, nfvm.NFVM_E_DIVERGED))
    sec, stats, s = timed_steps(g, steps)
    g.close()
    return sec, stats, s


# Algorithmic bytes per cell of the reverse-mode calls (FP64 throughout;
# each operand read once and each result written once): the state packed
# into the padded layout (read + written), for the explicit stage nu_t
# formed once (type byte, k, omega in; nu_t out), the weights pass (type
# byte, the state it reads, output adjoints in; per-cell weights out) and
# the gather pass (type byte, state, output adjoints and weights in; input
# adjoints out).
#   explicit stage: 6 x 16 + 25 + (1 + 48 + 48 + 112) + (1 + 56 + 48 + 112 + 56)
#                   (u v w T k omega packed; weights read u v w k omega nu_t,
#                   the gather also T)
#   destruction:    5 x 16 + (1 + 40 + 16 + 120) + (1 + 40 + 16 + 120 + 40)
REVERSE_BYTES_PER_CELL = {"explicit_adjoint": 603, "destroy_adjoint": 474}


def run_reverse(g, case, tol: float, repeats: int = 3):
    """The reverse modes at the grid's current state, adjoints of the
    outputs seeded N(0, 1): the explicit stage's and the destruction step's
    (wall time per call, each call waits for its stream; algorithmic bytes
    per second against the HBM peak) and one whole step's (forward step
    with its solve, then the stages' reverse modes and the adjoint solve,
    both solves to `tol`)."""
    import numpy as np
    import torch
    from paper_2603_21869_amd import nfvm
    names = ("u", "v", "w", "p", "T", "k", "omega")
    f = g.fields()
    st = {n: torch.from_numpy(np.ascontiguousarray(f[n], dtype=np.float64)).cuda() for n in names}
    del f
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    bars = {n: torch.randn(st[n].shape, dtype=torch.float64, device="cuda", generator=gen)
            for n in names}
    outs = {n: torch.empty_like(st[n]) for n in names}
    ptr = lambda d: {n: t.data_ptr() for n, t in d.items()}

    def timed(fn):
        fn()  # allocates the call's scratch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(repeats):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / repeats

    out = {}
    t_ex = timed(lambda: nfvm.nfvm_explicit_adjoint_device(g.h, ptr(st), ptr(bars), ptr(outs)))
    half = 0.5 * case.dt
    five = {n: outs[n].data_ptr() for n in ("u", "v", "w", "k", "omega")}
    t_des = timed(lambda: nfvm.nfvm_destroy_adjoint_device(
        g.h, ptr(st), half, bars["k"].data_ptr(), bars["omega"].data_ptr(), five))
    for name, t in (("explicit_adjoint", t_ex), ("destroy_adjoint", t_des)):
        b = REVERSE_BYTES_PER_CELL[name] * case.ncells
        out[name] = dict(ms=round(t * 1e3, 3), bytes_per_cell=REVERSE_BYTES_PER_CELL[name],
                         GBs=round(b / t / 1e9, 1), frac=round(b / t / 1e9 / PEAK_HBM_GBS, 4))
    stats = []

    def step_adj():
        s, _ = nfvm.nfvm_step_adjoint_device(g.h, ptr(st), ptr(bars), ptr(outs), tol=tol,
                                             max_cycles=200)
        stats.append(s)

    t_step = timed(step_adj)
    out["step_adjoint"] = dict(ms=round(t_step * 1e3, 2),
                               mcell_steps_s=round(case.ncells / t_step / 1e6, 2), tol=tol,
                               forward_cycles=stats[-1][0]["cycles"],
                               adjoint_cycles=stats[-1][1]["cycles"])
    del st, bars, outs
    torch.cuda.empty_cache()
    return out


def run_probes(g, case, points: int = 256, repeats: int = 5):
    """Line probes (Sec. 3.1) along three lines through the middle of the
    box, one per axis, `points` each: host wall time per call (points up,
    the device interpolation, results back)."""
    from paper_2603_21869_amd import nfvm
    import numpy as np
    L = [case.n[d] * case.h[d] for d in range(3)]
    mid = [0.5 * x for x in L]
    lines = []
    for d in range(case.dim):
        a, b = list(mid), list(mid)
        a[d], b[d] = 0.0, L[d]
        lines.append(nfvm.line(a, b, points))
    pts = np.concatenate(lines)
    g.probe(pts)
    t0 = time.perf_counter()
    for _ in range(repeats):
        v = g.probe(pts)
    t = (time.perf_counter() - t0) / repeats
    return dict(probe_ms_host=round(t * 1e3, 3), probe_points=int(len(pts)),
                probe_nan_points=int(np.isnan(v).any(axis=1).sum()))


def run_pcie(g, case, steps: int):
    """Throughput with the fields handed over in host memory: upload, the
    steps, download (on a grid whose tile choices exist already)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.set_fields(case.fields)
    g.step(steps, allow=(0, -5))
    g.fields()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    return case.ncells * steps / sec / 1e6


def run_serve(n_req: int, slots: int, seed: int = 0):
    """Replay the first n_req requests of the seeded serving trace (Poisson
    arrivals, 20/s; edges from {64, 96, 128, 192, 256}; channel or room; 50
    mixed-precision steps each) against the server in real time, after tuning
    the tile shapes of three cubic channels (64^3, 128^3, 256^3) before the
    server starts (served grids take the choices of the nearest tuned size)."""
    from paper_2603_21869_amd import cases as C, nfvm
    trace = C.serve_trace(seed=seed, n_requests=n_req)
    cases = [C.serve_case(r) for r in trace]
    descs = [nfvm.Desc(c) for c in cases]
    t_tune = time.perf_counter()
    for e in (64, 128, 256):
        nfvm.nfvm_tune(nfvm.Desc(C.serve_case(dict(n=(e, e, e), geometry="channel", seed=1,
                                                   n_steps=1))))
    t_tune = time.perf_counter() - t_tune
    srv = nfvm.nfvm_server_create(0.0, slots)
    t0 = time.perf_counter()
    tickets = []
    for r, c, d in zip(trace, cases, descs):
        wait = t0 + r["arrival"] - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        tickets.append(nfvm.nfvm_submit(srv, d, c.fields, r["n_steps"]))
    nfvm.nfvm_server_drain(srv)
    times = [nfvm.nfvm_request_times(srv, t) for t in tickets]
    status = [nfvm.nfvm_poll(srv, t, None, allow=(0, -4, -5))[0] for t in tickets]
    nfvm.nfvm_server_destroy(srv)
    lat = sorted(t[3] - t[0] for t in times)
    first = sorted(t[2] - t[0] for t in times if t[2] >= 0)
    span = max(t[3] for t in times) - min(t[0] for t in times)
    work = sum(c.ncells * r["n_steps"] for c, r in zip(cases, trace))
    pct = lambda a, q: a[min(len(a) - 1, int(math.ceil(q * len(a))) - 1)]
    return {"requests": n_req, "slots": slots, "arrival_rate_per_s": 20.0,
            "ok": sum(1 for s in status if s == 0),
            "throughput_mcell_steps_s": round(work / span / 1e6, 2),
            "makespan_s": round(span, 3),
            "latency_p50_s": round(pct(lat, 0.5), 3), "latency_p99_s": round(pct(lat, 0.99), 3),
            "first_converged_step_p50_s": round(pct(first, 0.5), 3),
            "first_converged_step_p99_s": round(pct(first, 0.99), 3),
            "mean_cells": int(sum(c.ncells for c in cases) / n_req),
            "pretune_s": round(t_tune, 2), "pretuned_edges": [64, 128, 256]}


def run_batch(n_grids: int = 8, edge: int = 64, steps: int = 10):
    """Batched stepping (one launch per multigrid kernel and level over all
    grids) against the same grids stepped one after the other: n_grids
    mixed-precision channels of edge^3 cells from the serving recipe."""
    from paper_2603_21869_amd import cases as C, nfvm
    import torch
    cases = [C.serve_case(dict(n=(edge, edge, edge), geometry="channel", seed=900 + i,
                               n_steps=steps)) for i in range(n_grids)]
    cells = sum(c.ncells for c in cases)
    out = {"grids": n_grids, "cells_per_grid": cases[0].ncells, "steps": steps}
    for mode in ("sequential", "batched"):
        gs = [nfvm.Grid(c) for c in cases]
        if mode == "batched":
            nfvm.nfvm_step_batch([g.h for g in gs], 2)
            t0 = time.perf_counter()
            nfvm.nfvm_step_batch([g.h for g in gs], steps)
        else:
            for g in gs:
                g.step(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for g in gs:
                g.step(steps)
        torch.cuda.synchronize()
        out[mode + "_mcell_steps_s"] = round(cells * steps / (time.perf_counter() - t0) / 1e6, 2)
        for g in gs:
            g.close()
    return out


def copy_bandwidth(mib: int = 1024, reps: int = 5) -> float:
    """Achievable HBM bandwidth on this device: a plain device-to-device copy
    of `mib` MiB (bytes read + written / time, best of `reps`)."""
    import torch
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * mib * (1 << 20) / best / 1e9


def run_paper_table(stream: int, precision: int, tol: float, steps: int = 100):
    """The paper's time-profiling workload (Sec. 3.3, Table 1): 100 steps of
    the open channel at 5 mm for each of its three streamwise lengths, timed
    the same way as the headline (fields resident, after two warm-up steps)."""
    from paper_2603_21869_amd import cases as C
    rows = []
    for nx, paper_s in PAPER_TABLE1_GPU_S.items():
        case = C.open_channel(nx, precision=precision, tol=tol, n_steps=steps)
        sec, stats, _ = run_gpu(case, steps, 2, stream)
        rows.append({"cells": case.ncells, "n": list(case.n), "levels": case.n_levels,
                     "steps": steps, "seconds": round(sec, 3),
                     "mcell_steps_s": round(case.ncells * steps / sec / 1e6, 2),
                     "mean_cycles": sum(x["cycles"] for x in stats) / len(stats),
                     "paper_gpu_seconds": paper_s,
                     "paper_mcell_steps_s": round(case.ncells * steps / paper_s / 1e6, 2)})
    return rows


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_sample(workload: str, tol: float):
    """The bounded sample of a workload that the oracle is timed on: the
    large room as the same room (same blocks in metres, vents, physics,
    tolerance and cycle shape) on a 256 x 128 x 64 grid, the other workloads
    as themselves."""
    from paper_2603_21869_amd import cases as C
    if workload == "bigroom":
        case = C.room3d(256, 128, 64, n_levels=7, precision=C.PREC_FP64, tol=tol,
                        n_steps=1).copy(**ROOM_CYCLE)
        what = ("one time step of the same room (same blocks, vents, physics, tol, cycle "
                "shape) on a 256x128x64 grid (1/64 of the cells), 7 levels")
    else:
        case = make_case(workload, C.PREC_FP64, tol)
        what = "time steps of the same workload from its initial state"
    return case, what


def _pin(core):
    try:
        old = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {core})
        return old
    except (AttributeError, OSError):
        return None


def oracle_worker(workload: str, tol: float, core: int) -> None:
    """One copy of the all-core leg: build the sample, say so, wait for the
    common start, time one oracle step on its own core, print the seconds."""
    from oracle import oracle as O
    _pin(core)
    case, _ = _cpu_sample(workload, tol)
    O.lib()
    print("ready", flush=True)
    sys.stdin.readline()
    t0 = time.perf_counter()
    O.step(case, 1)
    print(json.dumps({"seconds": time.perf_counter() - t0}), flush=True)


def cpu_all_cores(workload: str, tol: float, ncells: int, max_procs: int = 16):
    """The unchanged serial oracle on every host core at once: one process
    per core (at most 16), each stepping its own copy of the sample, started
    together; throughput = copies x cells / the slowest copy's step time."""
    import subprocess
    try:
        cores = sorted(os.sched_getaffinity(0))
    except AttributeError:
        cores = list(range(os.cpu_count() or 1))
    cores = cores[:max_procs]
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker",
                               str(c), "--workload", workload, "--tol", repr(tol)],
                              stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)
             for c in cores]
    try:
        for pr in procs:
            if pr.stdout.readline().strip() != "ready":
                raise RuntimeError("oracle worker failed to start")
        for pr in procs:
            pr.stdin.write("go\n")
            pr.stdin.flush()
        secs = []
        for pr in procs:
            secs.append(json.loads(pr.stdout.readline())["seconds"])
            print(f"[bench] oracle copy {len(secs)}/{len(procs)}: {secs[-1]:.2f} s",
                  file=sys.stderr, flush=True)
    finally:
        for pr in procs:
            try:
                pr.stdin.close()
                pr.wait(timeout=600)
            except (OSError, subprocess.TimeoutExpired):
                pr.kill()
    slowest = max(secs)
    return dict(value=round(len(cores) * ncells / slowest / 1e6, 4), unit="Mcell-steps/s",
                cores=len(cores), kind="oracle",
                sample=f"{len(cores)} copies of the serial FP64 oracle, one per host core, "
                       f"each stepping the same sample once, started together; slowest "
                       f"{slowest:.2f} s, fastest {min(secs):.2f} s")


def cpu_baseline(workload: str, tol: float, budget_s: float = 20.0, all_cores: bool = True):
    """The serial FP64 oracle, pinned to one host core, on a bounded sample of
    the workload (one step of the large room's sample; up to four steps of
    the other workloads), and beside it the same oracle on every host core
    at once (one copy per core)."""
    from oracle import oracle as O
    O.build()
    case, what = _cpu_sample(workload, tol)
    old_aff = None
    try:
        old_aff = os.sched_getaffinity(0)
        _pin(min(old_aff))
    except (AttributeError, OSError):
        old_aff = None
    try:
        t0 = time.perf_counter()
        f, st, status = O.step(case, 1)
        per = time.perf_counter() - t0
        n = 1
        if workload != "bigroom":
            extra = int(max(0, min(3, budget_s / per - 1)))
            if extra:
                t2 = time.perf_counter()
                O.step(case, extra, fields=f)
                per = (per + time.perf_counter() - t2) / (1 + extra)
                n += extra
    finally:
        if old_aff is not None:
            os.sched_setaffinity(0, old_aff)
    out = dict(value=round(case.ncells / per / 1e6, 4), unit="Mcell-steps/s", cores=1,
               kind="oracle",
               sample=f"{n} {what}; serial FP64 oracle pinned to one core ({cpu_model()}), "
                      f"{per:.2f} s/step, {st[0]['cycles']} V-cycles in its first step")
    if all_cores:
        # an optional leg: a failure is reported, not raised
        try:
            out["all_cores"] = cpu_all_cores(workload, tol, case.ncells)
        except Exception as e:  # noqa: BLE001
            out["all_cores"] = {"error": f"{type(e).__name__}: {e}"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bigroom", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="mixed", choices=["fp64", "fp32", "mixed"])
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-all-cores", action="store_true",
                    help="time the oracle on one core only (not also on every core)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the other precisions and tolerances of the same workload")
    ap.add_argument("--all-variants", action="store_true",
                    help="also Algorithm 1's cycle, nearest upsampling, Heun stage, FP32")
    ap.add_argument("--serve", type=int, default=256,
                    help="requests of the serving trace to replay (0: skip)")
    ap.add_argument("--serve-slots", type=int, default=9)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--lambda2", type=int, default=1,
                    help="lambda2 post-processing calls timed after the run (0: skip)")
    ap.add_argument("--no-paper-table", action="store_true",
                    help="skip the paper's open-channel timing workload (three lengths)")
    ap.add_argument("--only-steps", action="store_true",
                    help="only the timed steps of the workload (for profiler runs)")
    ap.add_argument("--no-reverse", action="store_true",
                    help="skip the reverse-mode timings")
    ap.add_argument("--only-reverse", action="store_true",
                    help="only the reverse-mode calls after the warm-up (for profiler runs)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB five times (for "
                         "scaling hardware byte counters) and exit")
    ap.add_argument("--oracle-worker", type=int, default=-1, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_worker >= 0:
        oracle_worker(args.workload, args.tol, args.oracle_worker)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration_mb:
        import torch
        n = args.copy_calibration_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "repeats": 5}))
        return

    import torch
    from paper_2603_21869_amd import cases as C, nfvm
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    prec = {"fp64": C.PREC_FP64, "fp32": C.PREC_FP32, "mixed": C.PREC_MIXED}[args.precision]
    case = make_case(args.workload, prec, args.tol)
    print(f"[bench] {args.workload} {case.n} {args.precision} tol={args.tol}", file=sys.stderr,
          flush=True)

    # timed run: graphs on, no per-kernel events (they would split the graphs)
    g = nfvm.Grid(case, stream=stream)
    if args.warmup:
        g.step(args.warmup, allow=(nfvm.NFVM_OK, nfvm.NFVM_E_NOTCONV))
    if args.only_reverse:
        rev = run_reverse(g, case, args.tol)
        g.close()
        print(json.dumps({"workload": args.workload, "reverse_mode": rev}))
        return
    sec, stats, status = timed_steps(g, args.steps)
    ms_per_step = sec / args.steps * 1e3
    value = case.ncells * args.steps / sec / 1e6
    cycles = [s["cycles"] for s in stats]
    mean_cycles = sum(cycles) / len(cycles)
    rel = [s["rel_residual"] for s in stats]
    if args.only_steps:
        g.close()
        print(json.dumps({"workload": args.workload, "value": round(value, 3),
                          "ms_per_step": round(ms_per_step, 4), "mean_cycles": mean_cycles}))
        return
    print(f"[bench] {value:.1f} Mcell-steps/s, {mean_cycles:.2f} cycles", file=sys.stderr,
          flush=True)

    # the same steps again with HIP events around every kernel launch
    psec, prof = profile_steps(g, args.steps)
    kernel_table = {}
    for k, v in prof.items():
        if not v["launches"]:
            continue
        avg = v["seconds"] / v["launches"]
        kernel_table[k] = dict(launches=v["launches"], avg_us=round(avg * 1e6, 3),
                               bytes_per_launch=round(v["bytes_per_launch"]),
                               GBs=round(v["bytes_per_launch"] / avg / 1e9, 1) if avg > 0 else 0.0,
                               share=round(v["seconds"] / psec, 4))
    # dominant kernel: the largest summed device time over every kernel
    dom = max(prof, key=lambda k: prof[k]["seconds"])
    d = prof[dom]
    avg = d["seconds"] / max(1, d["launches"])
    achieved = d["bytes_per_launch"] / avg / 1e9 if avg > 0 else 0.0
    # the pressure solve as a whole: its kernels' summed device time per step,
    # their algorithmic bytes, and the unfused byte model of a V(2,2) cycle
    t_solve = sum(prof[k]["seconds"] for k in SOLVE_KERNELS) / args.steps
    b_solve = sum(prof[k]["bytes_per_launch"] * prof[k]["launches"] for k in SOLVE_KERNELS) \
        / args.steps
    t_phys = sum(v["seconds"] for k, v in prof.items() if k not in SOLVE_KERNELS) / args.steps
    model_cycle = model_cycle_bytes(case)
    model_solve = model_cycle * case.ncells * mean_cycles
    model_step = model_solve + MODEL_STEP_B[args.precision] * case.ncells
    solve = {
        "kernel_ms_per_step": round(t_solve * 1e3, 4),
        "physics_kernel_ms_per_step": round(t_phys * 1e3, 4),
        "algorithmic_GBs": round(b_solve / t_solve / 1e9, 1),
        "model_bytes_per_cell_cycle": round(model_cycle, 1),
        "model_GBs": round(model_solve / t_solve / 1e9, 1),
        "model_frac": round(model_solve / t_solve / 1e9 / PEAK_HBM_GBS, 4),
        "step_model_GBs": round(model_step / (ms_per_step * 1e-3) / 1e9, 1),
        "step_model_frac": round(model_step / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
    }
    pcie = run_pcie(g, case, max(2, args.steps // 2))
    post = None
    if args.lambda2 > 0:
        # the lambda2 vortex criterion of the stepped velocity, handed back
        # in host memory (device kernel plus the FP64 copy over PCIe)
        g.lambda2()
        t0 = time.perf_counter()
        for _ in range(args.lambda2):
            l2 = g.lambda2()
        lsec = (time.perf_counter() - t0) / args.lambda2
        post = dict(lambda2_ms_host=round(lsec * 1e3, 3), calls=args.lambda2,
                    vortex_cells=int((l2 < 0).sum()))
        del l2
        post.update(run_probes(g, case))
    reverse = None
    if not args.no_reverse:
        print("[bench] reverse mode", file=sys.stderr, flush=True)
        try:  # reported beside the forward step: a failure does not end the run
            reverse = run_reverse(g, case, args.tol)
        except Exception as e:  # noqa: BLE001
            reverse = {"error": f"{type(e).__name__}: {e}"}
    g.close()
    copy_GBs = round(copy_bandwidth(), 1)

    variants = {}
    if not args.no_variants:
        k2 = max(3, args.steps // 2)
        runs = [("fp64", C.PREC_FP64, args.tol, {}, False)]
        if args.tol > 1e-9:
            # the tolerances at which every field meets 1e-6 of the converged
            # FP64 solution on the small rooms (mixed: 1e-9, FP64: 1e-8)
            runs += [("mixed_tol_1e-9", C.PREC_MIXED, 1e-9, {}, False),
                     ("fp64_tol_1e-8", C.PREC_FP64, 1e-8, {}, False)]
        runs += [(args.precision + "_warm_start", prec, args.tol, {}, True),
                 # Algorithm 1 as printed (undamped scalar-diagonal Jacobi,
                 # V(0,1), nearest upsampling, plain iteration): its
                 # convergence or divergence on this workload
                 (args.precision + "_alg1_literal", prec, args.tol, dict(literal=1), False),
                 # the plain V(2,2) cycle of the channel workloads
                 (args.precision + "_v22", prec, args.tol, dict(nu1=2, nu2=2, nu_coarse=0),
                  False)]
        if args.precision == "mixed":
            # every coarse level in BF16
            runs += [("mixed_all_coarse_bf16", prec, args.tol,
                      dict(coarse_fp32_cells=2**31 - 1), False)]
        if args.all_variants:
            runs += [("fp32", C.PREC_FP32, args.tol, {}, False),
                     (args.precision + "_nearest_prolongation", prec, args.tol,
                      dict(prolong=C.PROL_NEAREST), False),
                     (args.precision + "_alg1_v01_nearest", prec, args.tol,
                      dict(prolong=C.PROL_NEAREST, nu1=0, nu2=1), False),
                     (args.precision + "_heun_rk2", prec, args.tol, dict(rk_order=2), False)]
        for vname, pv, tv, kw, warm in runs:
            if vname.split("_")[0] == args.precision and tv == args.tol and not kw and not warm:
                continue
            c2 = make_case(args.workload, pv, tv).copy(**kw)
            print(f"[bench] variant {vname}", file=sys.stderr, flush=True)
            s2, st2, _ = run_gpu(c2, k2, 1, stream, warm_start=warm)
            bad = [i for i, x in enumerate(st2) if x["status"] != 0]
            if bad:
                # a failed solve ends the run: no throughput, where and how
                x = st2[bad[0]]
                variants[vname] = dict(value=None, tol=tv, failed_at_step=bad[0] + 1,
                                       status=x["status"], cycles=x["cycles"],
                                       rel_residual=x["rel_residual"])
            else:
                variants[vname] = dict(value=round(c2.ncells * k2 / s2 / 1e6, 2),
                                       ms_per_step=round(s2 / k2 * 1e3, 3), tol=tv,
                                       mean_cycles=sum(x["cycles"] for x in st2) / len(st2),
                                       last_rel_residual=st2[-1]["rel_residual"])
            del c2
    traffic, traffic_src = measured_traffic(args.workload, args.precision, dom)
    out = {
        "metric": "Mcell-steps/s at 1e-6 residual, % HBM peak; p50/p99 latency, batched solves",
        "value": round(value, 3),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "mixed": "f32+bf16 with f64 refinement"}[args.precision],
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "cells": case.ncells,
                   "precision": args.precision, "tol": args.tol, "dt": case.dt,
                   "levels": case.n_levels, "smoothing": smoothing_of(case),
                   "coarse_storage": coarse_storage_of(case),
                   "parallelism": "single GPU"},
        "solver": {"mean_cycles": mean_cycles, "max_rel_residual": max(rel),
                   "statuses": sorted({x["status"] for x in stats})},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic, "traffic_source": traffic_src,
                     "avg_launch_us": round(avg * 1e6, 2),
                     "algorithmic_bytes_per_launch": d["bytes_per_launch"],
                     "copy_GBs": copy_GBs, "solve": solve},
        "kernels": kernel_table,
        "variants": variants,
        "event_timed_ms_per_step": round(psec / args.steps * 1e3, 4),
        "pcie_inclusive_mcell_steps_s": round(pcie, 2),
        "postprocess": post,
        "reverse_mode": reverse,
        "tuning_entries": len(nfvm.nfvm_tuning_table()),
        "paper_context": "paper: 19-46x GPU over 32-core CPU (RTX PRO 5000 Blackwell vs "
                         "Threadripper 9970X); 23.8-38.1 Mcell-steps/s on its open channel",
    }
    if not args.no_batch:
        print("[bench] batching", file=sys.stderr, flush=True)
        out["batching"] = run_batch()
    if args.serve:
        print("[bench] serving", file=sys.stderr, flush=True)
        out["serving"] = run_serve(args.serve, args.serve_slots)
    if not args.no_paper_table:
        print("[bench] paper table", file=sys.stderr, flush=True)
        out["paper_table"] = run_paper_table(stream, prec, args.tol)
    if not args.no_cpu:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload, args.tol,
                                           all_cores=not args.no_all_cores)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
