"""Benchmark of the NeuralFVM time step on one MI355X.

One benchmark step is one full time step of the hot path (destruction half
step, explicit update, Poisson right-hand side, multigrid-preconditioned
pressure solve to the residual target, projection, destruction half step) over
the whole grid, with all fields resident in device memory.

Default workload: the 3D heated channel, 256 x 64 x 64 cells (2.56 x 0.64 x
0.64 m, inlet 0.1 m/s, bottom wall 310 K, Boussinesq buoyancy, seeded 1 %
velocity noise), 7 multigrid levels, mixed precision (FP32 scalars, FP32 /
BF16 V-cycle, FP64 velocity, pressure, residual and projection), pressure
solved to a relative residual of 1e-6 every step.

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
    "room": "3D ventilated room 512x256x128 with seeded blocks, 8 levels",
    "bigroom": "3D ventilated room 1024x512x256 with seeded blocks, 9 levels",
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
}


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


def make_case(name: str, precision: int, tol: float):
    from paper_2603_21869_amd import cases as C
    if name == "channel3d":
        return C.channel3d(precision=precision, tol=tol)
    if name == "channel2d":
        return C.channel2d(precision=precision, tol=tol)
    if name == "room":
        return C.room3d(precision=precision, tol=tol)
    if name == "bigroom":
        return C.room3d(1024, 512, 256, n_levels=9, precision=precision, tol=tol, n_steps=100)
    if name.startswith("open_channel_"):
        return C.open_channel(int(name.rsplit("_", 1)[1]), precision=precision, tol=tol)
    raise SystemExit(f"unknown workload {name}")


def run_gpu(case, steps: int, warmup: int, profile: bool, stream: int, graphs: bool = True,
            warm_start: bool = False):
    import torch
    from paper_2603_21869_amd import nfvm
    g = nfvm.Grid(case, stream=stream)
    nfvm.nfvm_set_option(g.h, nfvm.NFVM_OPT_GRAPHS, 1.0 if graphs else 0.0)
    nfvm.nfvm_set_option(g.h, nfvm.NFVM_OPT_WARM_START, 1.0 if warm_start else 0.0)
    if warmup:
        g.step(warmup, allow=(nfvm.NFVM_OK, nfvm.NFVM_E_NOTCONV))
    torch.cuda.synchronize()
    if profile:
        nfvm.nfvm_profile(g.h, (1 << len(nfvm.KERNELS)) - 1)
    t0 = time.perf_counter()
    s, stats = g.step(steps, allow=(nfvm.NFVM_OK, nfvm.NFVM_E_NOTCONV))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {}
    if profile:
        for kid, name in enumerate(nfvm.KERNELS):
            prof[name] = nfvm.nfvm_profile_read(g.h, kid)
    g.close()
    return t1 - t0, stats, prof, s


def run_pcie(case, steps: int, stream: int):
    """Throughput with the fields handed over in host memory: upload, the
    steps, download (the grid and its tile choices exist already)."""
    import torch
    from paper_2603_21869_amd import nfvm
    g = nfvm.Grid(case, stream=stream)
    g.step(1, allow=(nfvm.NFVM_OK, nfvm.NFVM_E_NOTCONV))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.set_fields(case.fields)
    g.step(steps, allow=(nfvm.NFVM_OK, nfvm.NFVM_E_NOTCONV))
    g.fields()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    g.close()
    return case.ncells * steps / sec / 1e6


def run_serve(n_req: int, slots: int, seed: int = 0):
    """Replay the first n_req requests of the seeded serving trace (Poisson
    arrivals, 20/s; edges from {64, 96, 128, 192, 256}; channel or room; 50
    mixed-precision steps each) against the server in real time."""
    from paper_2603_21869_amd import cases as C, nfvm
    trace = C.serve_trace(seed=seed, n_requests=n_req)
    cases = [C.serve_case(r) for r in trace]
    descs = [nfvm.Desc(c) for c in cases]
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
            "mean_cells": int(sum(c.ncells for c in cases) / n_req)}


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
        sec, stats, _, _ = run_gpu(case, steps, 2, False, stream)
        rows.append({"cells": case.ncells, "n": list(case.n), "levels": case.n_levels,
                     "steps": steps, "seconds": round(sec, 3),
                     "mcell_steps_s": round(case.ncells * steps / sec / 1e6, 2),
                     "mean_cycles": sum(x["cycles"] for x in stats) / len(stats),
                     "paper_gpu_seconds": paper_s,
                     "paper_mcell_steps_s": round(case.ncells * steps / paper_s / 1e6, 2)})
    return rows


def cpu_baseline(case, budget_s: float = 20.0):
    """The serial FP64 oracle on a bounded number of steps of the same workload."""
    from oracle import oracle as O
    O.build()
    t0 = time.perf_counter()
    f, st, status = O.step(case, 1)
    t1 = time.perf_counter()
    n = 1
    per = t1 - t0
    extra = int(max(0, min(3, budget_s / per - 1)))
    if extra:
        t2 = time.perf_counter()
        O.step(case, extra, fields=f)
        t3 = time.perf_counter()
        per = (t1 - t0 + t3 - t2) / (1 + extra)
        n += extra
    return dict(value=case.ncells / per / 1e6, unit="Mcell-steps/s", cores=1, kind="oracle",
                sample=f"{n} step(s) of the same workload from its initial state, serial FP64 "
                       f"oracle, {per:.2f} s/step")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="channel3d", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="mixed", choices=["fp64", "fp32", "mixed"])
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--serve", type=int, default=24,
                    help="requests of the serving trace to replay (0: skip)")
    ap.add_argument("--serve-slots", type=int, default=9)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--lambda2", type=int, default=3,
                    help="lambda2 post-processing calls timed after the run (0: skip)")
    ap.add_argument("--no-paper-table", action="store_true",
                    help="skip the paper's open-channel timing workload (three lengths)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB five times (for "
                         "scaling hardware byte counters) and exit")
    args = ap.parse_args()
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
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2603_21869_amd import cases as C, nfvm
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    prec = {"fp64": C.PREC_FP64, "fp32": C.PREC_FP32, "mixed": C.PREC_MIXED}[args.precision]
    case = make_case(args.workload, prec, args.tol)

    # timed run: graphs on, no per-kernel events (they would split the graphs)
    sec, stats, _, status = run_gpu(case, args.steps, args.warmup, False, stream, graphs=True)
    ms_per_step = sec / args.steps * 1e3
    value = case.ncells * args.steps / sec / 1e6
    cycles = [s["cycles"] for s in stats]
    rel = [s["rel_residual"] for s in stats]
    # kernel timing: the same workload and step count with HIP events around
    # every hot kernel launch (stream launches)
    psec, _, prof, _ = run_gpu(case, args.steps, args.warmup, True, stream, graphs=False)

    # dominant kernel: largest summed device time in the timed region
    dom = max(prof, key=lambda k: prof[k]["seconds"])
    d = prof[dom]
    avg = d["seconds"] / max(1, d["launches"])
    achieved = d["bytes_per_launch"] / avg / 1e9 if avg > 0 else 0.0
    kernel_table = {k: dict(launches=v["launches"], avg_us=(v["seconds"] / v["launches"] * 1e6)
                            if v["launches"] else 0.0,
                            GBs=(v["bytes_per_launch"] / (v["seconds"] / v["launches"]) / 1e9)
                            if v["launches"] and v["seconds"] > 0 else 0.0,
                            share=v["seconds"] / psec)
                    for k, v in prof.items() if v["launches"]}

    variants = {}
    if not args.no_variants:
        # the same workload with each solve started from the previous step's
        # increment (NFVM_OPT_WARM_START; the default starts from zero)
        sw, stw, _, _ = run_gpu(case, args.steps, args.warmup, False, stream, warm_start=True)
        variants[args.precision + "_warm_start"] = dict(
            value=case.ncells * args.steps / sw / 1e6, ms_per_step=sw / args.steps * 1e3,
            mean_cycles=sum(x["cycles"] for x in stw) / len(stw))
        # Algorithm 1's upsampling read as nearest (piecewise constant), in
        # the V(2,2) cycle and in Algorithm 1's own V(0,1) shape
        # and the explicit stage as Heun's second-order Runge-Kutta method
        for vname, kw in (("nearest_prolongation", dict(prolong=C.PROL_NEAREST)),
                          ("alg1_v01_nearest", dict(prolong=C.PROL_NEAREST, nu1=0, nu2=1)),
                          ("heun_rk2", dict(rk_order=2))):
            c2 = make_case(args.workload, prec, args.tol).copy(**kw)
            k2 = max(5, args.steps // 2)
            s2, st2, _, _ = run_gpu(c2, k2, args.warmup, False, stream)
            variants[args.precision + "_" + vname] = dict(
                value=c2.ncells * k2 / s2 / 1e6, ms_per_step=s2 / k2 * 1e3,
                mean_cycles=sum(x["cycles"] for x in st2) / len(st2),
                statuses=sorted({x["status"] for x in st2}))
        for pname, pv in (("fp64", C.PREC_FP64), ("fp32", C.PREC_FP32), ("mixed", C.PREC_MIXED)):
            if pv == prec:
                continue
            c2 = make_case(args.workload, pv, args.tol)
            k2 = max(5, args.steps // 2)
            s2, st2, _, _ = run_gpu(c2, k2, args.warmup, False, stream)
            variants[pname] = dict(value=c2.ncells * k2 / s2 / 1e6,
                                   ms_per_step=s2 / k2 * 1e3,
                                   mean_cycles=sum(x["cycles"] for x in st2) / len(st2))

    pcie = run_pcie(case, args.steps, stream)
    post = None
    if args.lambda2 > 0:
        # the lambda2 vortex criterion of the stepped velocity, handed back
        # in host memory (device kernel plus the FP64 copy over PCIe)
        from paper_2603_21869_amd import nfvm
        g = nfvm.Grid(case, stream=stream)
        g.step(1, allow=(nfvm.NFVM_OK, nfvm.NFVM_E_NOTCONV))
        g.lambda2()
        t0 = time.perf_counter()
        for _ in range(args.lambda2):
            l2 = g.lambda2()
        sec = (time.perf_counter() - t0) / args.lambda2
        g.close()
        post = dict(lambda2_ms_host=round(sec * 1e3, 3), calls=args.lambda2,
                    vortex_cells=int((l2 < 0).sum()))
    traffic, traffic_src = measured_traffic(args.workload, args.precision, dom)
    out = {
        "metric": "Mcell-steps/s at 1e-6 residual",
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
                   "levels": case.n_levels, "smoothing": "V(2,2) damped Jacobi",
                   "parallelism": "single GPU"},
        "solver": {"mean_cycles": sum(cycles) / len(cycles), "max_rel_residual": max(rel)},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic, "traffic_source": traffic_src,
                     "avg_launch_us": round(avg * 1e6, 2),
                     "algorithmic_bytes_per_launch": d["bytes_per_launch"],
                     "copy_GBs": round(copy_bandwidth(), 1)},
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kernel_table.items()},
        "variants": variants,
        "stream_launch_ms_per_step": round(psec / args.steps * 1e3, 4),
        "pcie_inclusive_mcell_steps_s": round(pcie, 2),
        "postprocess": post,
        "tuning": [list(t) for t in nfvm.nfvm_tuning_table()],
        "paper_context": "paper: 19-46x GPU over 32-core CPU (RTX PRO 5000 Blackwell vs "
                         "Threadripper 9970X); 23.8-38.1 Mcell-steps/s on its open channel",
    }
    if not args.no_batch:
        out["batching"] = run_batch()
    if args.serve:
        out["serving"] = run_serve(args.serve, args.serve_slots)
    if not args.no_paper_table:
        out["paper_table"] = run_paper_table(stream, prec, args.tol)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(make_case(args.workload, C.PREC_FP64, args.tol))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
