#!/usr/bin/env python3
"""Throughput of the VLBM refinement hot path on one MI355X.

One step = one coarse step of the whole hot path: the recursive sub-cycle of
every level (fused ghost-fill / reflux-capture / stream / collide launches),
and for a dynamic workload a tag-and-regrid every 5 coarse steps (inside the
timed region). Default workload: the Kelvin-Helmholtz shear layer, 4096 x 4096
coarse, periodic, three refinement levels at r = 2 that track the two layers
by tagging, clustering, merge and split; FP64, seed 0, inputs resident in HBM
before the timed region.

metric: fine-equivalent cell updates per second = (nx0 r^L)(ny0 r^L) r^L per
coarse step (the updates a uniform finest-level grid would need), over the
timed steps. The JSON line also carries the roofline of the dominant kernel
(the level and launch form with the most kernel time; algorithmic bytes: 16
populations in + 16 out per cell update, two updates per cell for a fused
two-sub-step launch, over the launch's own duration from per-kernel events),
the conservation defect per coarse step, and the oracle timed on the host
cores on a bounded sample (for the 4096^2 problem: its largest down-scale
whose dense oracle arrays fit in 8 GB).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic per launch of the dominant kernel of the default workload
# (kh4096, FP64, 512-cell tiles, flags 17: the level-0 step launch, 16,646,144
# cells; flag 2048 leaves that level's 32,512 tiles as they are, so the value
# holds with flags 17 | 2048), from rocprofv3 FETCH_SIZE x 2.000 and WRITE_SIZE x 1.000 (the scales
# a plain 2 GiB device copy reads on the same counters: 1,048,588 KiB fetched
# and 2,097,152 KiB written per 2 GiB); valid only for the kernel source it
# was measured on.
MEASURED_TRAFFIC = {"kernel_sha256_16": "f9a98e712236bc2e", "workload": "kh4096",
                    "precision": "fp64", "tile_cells": 512, "flags": (17, 17 | 2048), "kernel": "step_kernel",
                    "level": 0, "bytes_per_launch": (2 * 1067192.9 + 2082632.1) * 1024}


# dynamic-refinement workloads: re-tag and regrid every few coarse steps
# (the density-gradient indicator is per cell, so it halves with each level
# on a smeared layer: the shear layer needs a lower threshold to keep level 3)
# shock_bubble: the fused finest level (the autotuner's pick from timing steps
# alone) makes every regrid build fused tile lists too, which costs more host
# time per regrid than the fused launches save over five coarse steps: plain
# 256-cell tiles measure fastest over the timed region, regrids included
DYNAMIC = {"shock_bubble": {"max_box": 64, "threshold": 0.05, "tuning": (256, 0)},
           "kh_strip": {"max_box": 128, "threshold": 0.01},
           "kh4096": {"max_box": 128, "threshold": 0.01, "tuning": (512, 17 | 2048)}}


def kernel_hash():
    import hashlib
    path = os.path.join(ROOT, "paper_2609_35529_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def build_case(name, steps):
    from paper_2609_35529_amd import workloads as wl
    if name == "quadrant512":
        return wl.quadrant(n0=512, seed=0, steps=steps)
    if name == "sod":
        return wl.sod_2d(steps=steps)
    if name == "shock_bubble":
        return wl.shock_bubble(steps=steps)
    if name == "patches":
        return wl.patch_set(seed=0, steps=steps)
    if name == "kh_strip":
        return wl.kelvin_helmholtz_strip(steps=steps)
    if name == "kh4096":
        return wl.kelvin_helmholtz(n0=4096, seed=0, nlev=4, steps=steps, dynamic=True)
    if name == "uniform4096":
        import numpy as np
        n = 4096
        U = wl.random_smooth_U(n, n, seed=0)
        return wl.Case("uniform4096", n, n, 1.0 / n, 2, 1, 1.4, 4.0, 0.8, (0,) * 4, [], [U], steps)
    raise SystemExit(f"unknown workload {name}")


WORKLOADS_3D = ("blast3d",)


def bench_3d(args):
    """The three-dimensional (D3Q6) path: 3-D blast in a reflecting box, 256^3
    coarse cells with one r = 2 patch of 256^3 fine cells (FP64 unless
    --precision says otherwise)."""
    import torch
    from paper_2609_35529_amd import vlbm3
    from paper_2609_35529_amd import workloads as wl
    case = wl.blast3d(n0=args.n0_3d, steps=args.warmup + args.steps)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream()
    prec = {"fp64": vlbm3.FP64, "fp32": vlbm3.FP32, "fp32s": vlbm3.FP32_STORAGE}[args.precision]
    solver = vlbm3.Solver3.from_case(case, stream=stream, precision=prec)
    # the library's default (non-temporal stores; 512-cell tiles in FP64, 1024
    # in the FP32 forms) unless given
    tuning = {"tile_cells": args.tile_cells or (512 if prec == vlbm3.FP64 else 1024),
              "flags": args.flags if args.tile_cells else 1}
    solver.set_tuning(tuning["tile_cells"], tuning["flags"])
    T0, L0 = solver.totals()
    # dynamic refinement: tag and regrid every `regrid_every` coarse steps,
    # inside the timed region
    regrid_every = 5
    amr = {"regrids": 0, "regrid_s": 0.0, "updates": 0, "boxes": []}

    def run(n):
        done = 0
        while done < n:
            k = n - done
            if args.amr_threshold is not None:
                k = min(k, regrid_every)
            solver.advance(k)
            if args.amr_threshold is not None:
                act = [solver.active_cells(l) for l in range(case.nlev)]
                amr["updates"] += k * sum(a * case.r ** l for l, a in enumerate(act))
                solver.sync()  # regrid_s: the regrid's own time, not the steps queued before it
                t = time.perf_counter()
                solver.tag_and_regrid(args.amr_threshold, buffer=args.amr_buffer,
                                      min_box=args.amr_min_box, max_box=args.amr_max_box or 64)
                amr["regrid_s"] += time.perf_counter() - t
                amr["regrids"] += 1
                amr["boxes"].append(len(solver.boxes()))
            done += k

    print(f"[bench] {case.name} warmup {args.warmup}", file=sys.stderr, flush=True)
    run(args.warmup)
    torch.cuda.synchronize()
    amr.update(regrids=0, regrid_s=0.0, updates=0, boxes=[])
    t0 = time.perf_counter()
    run(args.steps)
    solver.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    amr_timed = dict(amr)
    prof_steps = min(args.steps, 20)
    solver.set_profiling(True)
    solver.advance(prof_steps)
    kt = solver.kernel_times()
    solver.set_profiling(False)
    T1, L1 = solver.totals()
    fe_step = case.fine_equivalent_per_coarse_step()
    upd = (case.actual_updates_per_coarse_step() if args.amr_threshold is None
           else amr_timed["updates"] / args.steps)
    dom = max(kt, key=lambda k: kt[k][0])
    dom_ms, dom_calls, dom_cells = kt[dom]
    avg_s = dom_ms / 1e3 / dom_calls
    bytes_per_launch = dom_cells / dom_calls * 2 * 30 * (8 if prec == vlbm3.FP64 else 4)
    achieved = bytes_per_launch / avg_s / 1e9
    scale = max(abs(x) for x in T0)
    out = {
        "metric": "fine-equiv cell updates/s",
        "value": fe_step * args.steps / wall,
        "unit": "cell updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32s": "f64 math, f32 storage"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{case.name}: {case.nx0}^3 coarse, levels {case.nlev}, "
                               + (f"initial boxes {case.boxes}, tag and regrid every {regrid_every} coarse steps, "
                                  if args.amr_threshold is not None else f"boxes {case.boxes}, ")
                               + f"r={case.r}, beta={case.beta}, c={case.c:.4f}, reflecting walls, D3Q6",
                   "fine_equiv_per_step": fe_step, "actual_updates_per_step": upd,
                   "launches_per_step": sum(v[1] for v in kt.values()) / prof_steps,
                   "tuning": tuning, "precision": args.precision},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "step3_kernel",
                     "level": dom, "bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": avg_s * 1e6, "launches": dom_calls,
                     "timing": f"per-kernel events over {prof_steps} further coarse steps"},
        "actual_updates_per_s": upd * args.steps / wall,
        "amr": ({"regrid_every": regrid_every, "regrids": amr_timed["regrids"],
                 "regrid_s": amr_timed["regrid_s"], "threshold": args.amr_threshold,
                 "buffer": args.amr_buffer, "min_box": args.amr_min_box,
                 "max_box": args.amr_max_box or 64,
                 "boxes_min": min(amr_timed["boxes"]), "boxes_max": max(amr_timed["boxes"])}
                if args.amr_threshold is not None and amr_timed["boxes"] else None),
        "conservation_drift_rel": [float(abs((T1[k] - T0[k]) - (L1[k] - L0[k])) / scale) for k in range(5)],
        "cpu_baseline": None,
    }
    solver.close()
    del solver
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if args.no_cpu_baseline:
        out["cpu_baseline"] = {"value": None, "unit": "fine-equiv cell updates/s", "cores": 1, "kind": "oracle",
                               "sample": "not run (--no-cpu-baseline)"}
    else:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_blast3d_downscale(args, prec, stream)
    print(json.dumps(out))


def cpu_baseline_blast3d_downscale(args, prec, stream, mem_cap=8e9):
    """The 3-D oracle, single-threaded, on the blast down-scaled to the
    largest n0^3 (a multiple of 32) whose dense oracle arrays fit in mem_cap:
    every level over the whole domain at its own resolution, 4 x 30 doubles
    and 2 bytes per cell (96^3 coarse and its 192^3 fine level: 7.7 GB). The
    hierarchy is the line's initial one (the central half refined), held
    fixed; the oracle's steps are timed for about args.cpu_budget seconds. The
    GPU advances the same down-scale as many steps, and the line reports their
    largest relative population difference."""
    import numpy as np
    from oracle import oracle3 as O3
    from paper_2609_35529_amd import vlbm3, workloads as wl
    per_cell = 4 * 30 * 8 + 2
    n0 = 32
    while per_cell * ((n0 + 32) ** 3) * sum(8 ** l for l in range(2)) <= mem_cap:
        n0 += 32
    case = wl.blast3d(n0=n0, steps=0)
    o = O3.Oracle3(case.nx0, case.ny0, case.nz0, case.dx0, r=case.r, nlev=case.nlev, gamma=case.gamma,
                   c=case.c, beta=case.beta, bc=case.bc)
    o.set_boxes(case.boxes)
    for l in range(case.nlev):
        o.set_state(l, case.full_state(l) if case.origins else case.states[l])
    el, n = 0.0, 0
    while el < args.cpu_budget or n < 2:
        t0 = time.perf_counter()
        o.advance(1)
        el += time.perf_counter() - t0
        n += 1
    g = vlbm3.Solver3.from_case(case, stream=stream, precision=prec)
    g.advance(n)
    worst = 0.0
    for l in range(case.nlev):
        Fo, Fg = o.get_pop(l), g.get_populations(l)
        m = ~np.isnan(Fo)
        if m.any():
            worst = max(worst, float(np.max(np.abs(Fg[m] - Fo[m]) / np.maximum(np.abs(Fo[m]), 1e-3))))
    g.close()
    upd = case.actual_updates_per_coarse_step()
    return {"value": case.fine_equivalent_per_coarse_step() * n / el, "unit": "fine-equiv cell updates/s",
            "cores": 1, "kind": "oracle",
            "sample": f"blast3d down-scaled to {n0}^3 coarse with its central-half patch ({2 * n0}^3 fine "
                      f"cells), the largest multiple of 32 whose dense oracle arrays fit in {mem_cap / 1e9:.0f} GB: "
                      f"{n} coarse steps ({el:.1f} s), static hierarchy, FP64, one thread; the value is the "
                      "down-scale's fine-equivalent rate",
            "actual_updates_per_s": upd * n / el, "host": host_cpu(),
            "gpu_vs_oracle_max_rel": worst, "gpu_vs_oracle_bitwise": bool(worst == 0.0 and prec == vlbm3.FP64)}


def actual_updates_per_step(case):
    return case.actual_updates_per_coarse_step()


def host_cpu():
    """The host the oracle runs on: CPU model and the logical CPUs it offers."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "available_to_process": avail}


def cpu_baseline(case, budget_s=15.0, boxes=None, mem_cap=8e9, sensor=None, adaptive_dt=None):
    """The oracle, single-threaded, on a bounded prefix of the same workload.
    A dynamic workload is sampled on the hierarchy the GPU run starts its timed
    region with (`boxes`), held fixed. The oracle keeps three dense arrays of
    16 doubles per cell of every level; above mem_cap bytes it is not run."""
    from tests import exact
    if boxes is not None:
        import dataclasses
        case = dataclasses.replace(case, boxes=list(boxes))
    need = sum(3 * 16 * 8 * (case.nx0 * case.r ** l) * (case.ny0 * case.r ** l)
               for l in range(case.nlev))
    if need > mem_cap:
        return {"value": None, "unit": "fine-equiv cell updates/s", "cores": 1, "kind": "oracle",
                "sample": f"not run: the oracle's dense level arrays need {need / 1e9:.0f} GB",
                "host": host_cpu()}
    o = exact.run_oracle(case, steps=0)
    if sensor:
        o.set_sensor(True, *sensor)
    if adaptive_dt is not None:
        o.set_time_stepping(True, adaptive_dt)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < budget_s and n < case.steps:
        o.advance(1)
        n += 1
    el = time.perf_counter() - t0
    fe = case.fine_equivalent_per_coarse_step() * n / el
    held = f", hierarchy of the GPU run's timed region ({len(boxes)} boxes) held fixed" if boxes else ""
    if sensor:
        held += f", adaptive beta (C, beta_min, beta_max) = {tuple(sensor)}"
    if adaptive_dt is not None:
        held += f", adaptive time step (kappa = {adaptive_dt})"
    return {"value": fe, "unit": "fine-equiv cell updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{case.name} full size, first {n} coarse steps ({el:.1f} s){held}, FP64, "
                      f"one thread", "host": host_cpu()}


def cpu_baseline_kh_downscale(args, prec, stream, n0=256, strip=False):
    """The oracle, single-threaded, on the Kelvin-Helmholtz problem down-scaled
    to n0^2 coarse cells with the same three dynamic levels: the largest
    down-scale whose dense oracle arrays (every level over the whole domain,
    the finest one 2048^2 here) fit in 8 GB. With strip, the 4096 x 512 strip
    down-scaled to n0 x n0 / 8 coarse cells (n0 = 1024: the finest level
    8192 x 1024, 7.2 GB of dense arrays). The hierarchy comes from the GPU
    solver's tag-and-regrid on the same down-scale (regrid every
    args.regrid_every coarse steps), which the oracle follows box for box; the
    oracle's own steps are timed. The same run gives the GPU's difference to
    the oracle at the bench's precision (FP64: largest relative population
    difference; FP32 forms: the smooth-cell error of the FP32 tolerance)."""
    import numpy as np
    from paper_2609_35529_amd import vlbm, workloads as wl
    from tests import exact
    from tests.parity import fp32_error
    key = "kh_strip" if strip else "kh4096"
    if strip:
        case = wl.kelvin_helmholtz_strip(n0=n0, ny0=n0 // 8, seed=0, nlev=4, steps=0)
    else:
        case = wl.kelvin_helmholtz(n0=n0, seed=0, nlev=4, steps=0, dynamic=True)
    thr, buf = DYNAMIC[key]["threshold"], args.amr_buffer
    mn, mx = args.amr_min_box, args.amr_max_box or DYNAMIC[key]["max_box"]
    g = vlbm.Solver.from_case(case, precision=prec, stream=stream)
    g.set_tuning(*DYNAMIC["kh4096"]["tuning"])
    for _ in range(case.nlev - 1):
        g.tag_and_regrid(thr, buffer=buf, min_box=mn, max_box=mx)
    o = exact.run_oracle(case, steps=0)
    o.regrid(g.boxes())
    el, n = 0.0, 0
    while el < args.cpu_budget or n < 2 * args.regrid_every:
        k = args.regrid_every
        g.advance(k)
        t0 = time.perf_counter()
        o.advance(k)
        el += time.perf_counter() - t0
        n += k
        g.tag_and_regrid(thr, buffer=buf, min_box=mn, max_box=mx)
        o.regrid(g.boxes())
    upd = sum(o.active_mask(l).sum() * case.r ** l for l in range(case.nlev))
    err = {}
    if prec == vlbm.FP64:
        worst = 0.0
        for l in range(case.nlev):
            Fo, Fg = o.get_pop(l), g.get_populations(l)
            m = ~np.isnan(Fo)
            if m.any():
                worst = max(worst, float(np.max(np.abs(Fg[m] - Fo[m]) / np.maximum(np.abs(Fo[m]), 1e-3))))
        err = {"gpu_vs_oracle_max_rel": worst, "gpu_vs_oracle_bitwise": bool(worst == 0.0)}
    else:
        from tests.parity import smooth_mask
        e = fp32_error(o, g, case)
        cells = [int(smooth_mask(o.get_state(l)).sum()) for l in range(case.nlev)]
        err = {"gpu_vs_oracle_smooth_rel_err": float(e.max()), "per_component": e.max(axis=0).tolist(),
               "per_level": e.max(axis=1).tolist(), "smooth_cells_per_level": cells}
    g.close()
    what = (f"kelvin_helmholtz strip down-scaled to {n0}x{n0 // 8} coarse, 3 dynamic levels (finest "
            f"{n0 * 8}x{n0}), whose dense oracle arrays fit in 8 GB" if strip else
            f"kelvin_helmholtz down-scaled to {n0}^2 coarse, 3 dynamic levels (finest {n0 * 8}^2), "
            "the largest down-scale whose dense oracle arrays fit in 8 GB")
    return {"value": case.fine_equivalent_per_coarse_step() * n / el, "unit": "fine-equiv cell updates/s",
            "cores": 1, "kind": "oracle",
            "sample": f"{what}: {n} coarse steps ({el:.1f} s) with a regrid every {args.regrid_every} on the GPU "
                      "run's boxes, FP64, one thread; the value is the down-scale's fine-equivalent rate",
            "actual_updates_per_s": float(upd) * n / el, "host": host_cpu(), **err}


def copy_probe(gib=2.0, reps=20):
    """Bandwidth of a plain device-to-device copy of known size (the practical
    HBM ceiling, and the reference for scaling hardware byte counters)."""
    import torch
    n = int(gib * 2 ** 30 / 8)
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    return {"copy_bytes_per_launch": 2 * n * 8, "copy_us": s * 1e6, "copy_GBs": 2 * n * 8 / s / 1e9}


def serve_benchmark(n_requests=48, rate=64.0, seed=0, budget_gib=64.0, quantum=25,
                    check_accuracy=True, precision="fp32s", policy="share", tuning=None, seq_tuning=None):
    """Served stream: continuous batching (FP32 bulk, FP64 interfaces) against
    sequential plain FP64, same requests, same arrival times. tuning /
    seq_tuning: (tile_cells, flags) of the served and the sequential solves."""
    import numpy as np
    import torch
    from paper_2609_35529_amd import serve, vlbm, workloads as wl
    from tests.parity import smooth_mask
    stream = torch.cuda.Stream()
    reqs = wl.request_stream(n_requests, rate, seed=seed)
    prec = {"fp32": vlbm.FP32, "fp32s": vlbm.FP32_STORAGE, "fp64": vlbm.FP64}[precision]
    srv = serve.Server(int(budget_gib * 2 ** 30), precision=prec, quantum=quantum,
                       stream=stream, keep_states=check_accuracy, policy=policy, tuning=tuning)
    print(f"[bench] served stream (batched {precision})", file=sys.stderr, flush=True)
    served, wall_s = srv.run(reqs)
    print("[bench] sequential FP64", file=sys.stderr, flush=True)
    seq, wall_q = serve.run_sequential(reqs, precision=vlbm.FP64, stream=stream,
                                       keep_states=check_accuracy, tuning=seq_tuning)
    out = {"requests": n_requests, "rate_per_s": rate, "seed": seed,
           "served_precision": precision, "policy": policy, "tuning": tuning, "seq_tuning": seq_tuning,
           "batched": serve.summarize(served, wall_s),
           "sequential_fp64": serve.summarize(seq, wall_q)}
    if check_accuracy:
        ref = {r.rid: r.state for r in seq}
        worst, nan_mismatch, compared = 0.0, 0, 0
        for r in served:
            Uo = ref[r.rid]
            nan_mismatch += int(np.count_nonzero(np.isnan(Uo) != np.isnan(r.state)))
            m = smooth_mask(Uo) & np.isfinite(r.state).all(axis=0)
            if not m.any():
                continue
            compared += 1
            for k in range(4):
                scale = np.nanmax(np.abs(Uo[k]))
                worst = max(worst, float(np.max(np.abs(r.state[k][m] - Uo[k][m])) / scale))
        out["served_vs_fp64_smooth_rel_err"] = worst
        out["served_vs_fp64_compared_solves"] = compared
        out["served_vs_fp64_nan_mismatch_cells"] = nan_mismatch
    return out


def _tuning_arg(s):
    return tuple(int(x) for x in s.split(",")) if s else None


def serve_sweep(args):
    """The served benchmark at every arrival rate of --rates (else --rate); a
    single rate gives one record, several a list under "rates"."""
    rates = [float(x) for x in args.rates.split(",")] if args.rates else [args.rate]
    recs = [serve_benchmark(args.requests, r, precision=args.serve_precision, policy=args.serve_policy,
                            tuning=_tuning_arg(args.serve_tuning), seq_tuning=_tuning_arg(args.seq_tuning))
            for r in rates]
    return recs[0] if len(recs) == 1 else {"rates": recs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="kh4096")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "fp32s"],
                    help="fp32s: FP32 storage, relaxation evaluated in FP64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--amr-threshold", type=float, default=None,
                    help="density-gradient tag threshold (default: the workload's)")
    ap.add_argument("--amr-buffer", type=int, default=4)
    ap.add_argument("--regrid-every", type=int, default=5, help="coarse steps between tag-and-regrids")
    ap.add_argument("--amr-min-box", type=int, default=16)
    ap.add_argument("--amr-max-box", type=int, default=0,
                    help="largest box side in fine cells (0: the workload's default)")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch autotuner")
    ap.add_argument("--tile-cells", type=int, default=0, help="fixed launch tuning (skips the autotuner)")
    ap.add_argument("--flags", type=int, default=0, help="launch flags with --tile-cells")
    ap.add_argument("--tune-steps", type=int, default=5,
                    help="coarse steps timed per autotuner candidate (real steps of the run)")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the served-stream benchmark (batched FP32 storage vs sequential FP64)")
    ap.add_argument("--serve-only", action="store_true", help="only the served-stream benchmark")
    ap.add_argument("--requests", type=int, default=48)
    ap.add_argument("--rate", type=float, default=64.0)
    ap.add_argument("--serve-precision", default="fp32s", choices=["fp32", "fp32s", "fp64"])
    ap.add_argument("--serve-policy", default="share", choices=["share", "srpt", "fixed"])
    ap.add_argument("--serve-tuning", default=None, metavar="TILE,FLAGS",
                    help="launch tuning of the served solves (vlbm_set_tuning)")
    ap.add_argument("--seq-tuning", default=None, metavar="TILE,FLAGS",
                    help="launch tuning of the sequential FP64 solves")
    ap.add_argument("--rates", default=None, metavar="R1,R2,...",
                    help="arrival rates (requests/s) of the served stream; default: --rate")
    ap.add_argument("--n0-3d", type=int, default=256, help="coarse cells per axis of the 3-D workload")
    ap.add_argument("--adaptive-dt", type=float, default=None, metavar="KAPPA",
                    help="adaptive time step: c = 2 kappa max(|u| + c_s) every coarse step")
    ap.add_argument("--sensor", default=None, metavar="C,BMIN,BMAX",
                    help="space/time-adaptive beta (eq. sensor-B) with these constants")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only measure a plain 2 GiB device copy and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus}: the solver runs on a single GPU; sharding across GPUs "
              "is designed but not implemented, so only --gpus 1 is measured.", file=sys.stderr)
        sys.exit(2)
    if args.workload in WORKLOADS_3D:
        bench_3d(args)
        return
    if args.copy_probe:
        print(json.dumps(copy_probe()))
        return
    if args.serve_only:
        print(json.dumps(serve_sweep(args)))
        return
    import torch
    from paper_2609_35529_amd import vlbm

    case = build_case(args.workload, args.warmup + args.steps)
    prec = {"fp64": vlbm.FP64, "fp32": vlbm.FP32, "fp32s": vlbm.FP32_STORAGE}[args.precision]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream()  # a dedicated stream (default priority): graphs need one
    solver = vlbm.Solver.from_case(case, precision=prec, stream=stream)
    sensor = None
    if args.sensor:
        sensor = [float(x) for x in args.sensor.split(",")]
        solver.set_sensor(True, *sensor)
    if args.adaptive_dt is not None:  # c chosen every coarse step from the state
        solver.set_time_stepping(True, args.adaptive_dt)
    T0, L0 = solver.totals()

    tuning = None
    if not args.tile_cells and args.workload in DYNAMIC and "tuning" in DYNAMIC[args.workload]:
        args.tile_cells, args.flags = DYNAMIC[args.workload]["tuning"]
    dynamic = args.workload in DYNAMIC
    if dynamic and args.amr_max_box == 0:
        args.amr_max_box = DYNAMIC[args.workload]["max_box"]
    if dynamic and args.amr_threshold is None:
        args.amr_threshold = DYNAMIC[args.workload]["threshold"]
    regrid_every = args.regrid_every
    amr = {"regrids": 0, "boxes": [], "regrid_s": 0.0, "updates": 0}

    def run(n):
        """n coarse steps; the dynamic-AMR workload re-tags and regrids every
        regrid_every coarse steps (inside the timed region)."""
        if not dynamic:
            solver.advance(n)
            return
        done = 0
        while done < n:
            if solver.steps() % regrid_every == 0:
                solver.sync()  # regrid_s: the regrid's own time, not the steps queued before it
                t = time.perf_counter()
                solver.tag_and_regrid(args.amr_threshold, buffer=args.amr_buffer,
                                      min_box=args.amr_min_box, max_box=args.amr_max_box)
                amr["regrid_s"] += time.perf_counter() - t
                amr["regrids"] += 1
                amr["boxes"].append(len(solver.boxes()))
            k = min(n - done, regrid_every - solver.steps() % regrid_every)
            solver.advance(k)
            act = [solver.active_cells(l) for l in range(case.nlev)]
            amr["updates"] += k * sum(a * case.r ** l for l, a in enumerate(act))
            done += k

    if dynamic:  # build the hierarchy before tuning and timing
        for _ in range(case.nlev - 1):
            solver.tag_and_regrid(args.amr_threshold, buffer=args.amr_buffer,
                                  min_box=args.amr_min_box, max_box=args.amr_max_box)
    if args.tile_cells:
        solver.set_tuning(args.tile_cells, args.flags)
        tuning = {"tile_cells": args.tile_cells, "flags": args.flags}
    elif not args.no_tune:
        # on the hierarchy the timed region starts from (a dynamic workload
        # keeps the choice through its regrids); the trial steps are untimed
        print(f"[bench] {case.name} autotune", file=sys.stderr, flush=True)
        tile, flags = solver.autotune(steps_per_trial=args.tune_steps)
        tuning = {"tile_cells": tile, "flags": flags}
    print(f"[bench] {case.name} warmup {args.warmup}", file=sys.stderr, flush=True)
    run(args.warmup)
    torch.cuda.synchronize()
    amr.update(regrids=0, boxes=[], regrid_s=0.0, updates=0)
    timed_boxes = solver.boxes() if dynamic else None
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    run(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    upd_timed = amr["updates"]
    amr_timed = {k: (list(v) if isinstance(v, list) else v) for k, v in amr.items()}
    # Per-kernel durations come from a second region of the same run: every
    # step launch records its own start and end (launch-extension events on
    # the solver's stream). Those events lengthen the gaps between launches,
    # so they stay out of the throughput region above.
    prof_steps = min(args.steps, 100)
    solver.set_profiling(True)
    tp = time.perf_counter()
    run(prof_steps)
    ktimes = solver.kernel_times()
    prof_wall = time.perf_counter() - tp
    solver.set_profiling(False)
    T1, L1 = solver.totals()
    healthy = solver.check_health()
    # conservation defect coarse step by coarse step (regrids included):
    # ((T - T0) - (L - L0)) / max|T0| per component
    drift_steps = 10
    Tp, Lp = solver.totals()
    drift_series = []
    for _ in range(drift_steps):
        run(1)
        Tn, Ln = solver.totals()
        sc = max(abs(x) for x in Tp)
        drift_series.append([float(((Tn[k] - Tp[k]) - (Ln[k] - Lp[k])) / sc) for k in range(4)])
        Tp, Lp = Tn, Ln

    fe_step = case.fine_equivalent_per_coarse_step()
    value = fe_step * args.steps / wall
    upd = actual_updates_per_step(case) if not dynamic else upd_timed / args.steps
    esz = 8 if prec == vlbm.FP64 else 4
    bytes_per_update = 2 * 16 * esz
    nl = sum(v[1] for v in ktimes.values()) / prof_steps
    if args.adaptive_dt is not None:  # the one-thread update of the link speed, every coarse step
        nl += 1
    if sensor:
        # a separate next-Qmax clear per coarse step only where the finest
        # level takes one step per coarse step; the SEN step also reads W
        # (32 B), writes W (32 B) and beta (8 B) and reads the mask (1 B)
        nl = nl + (1 if case.nlev == 1 or case.r == 1 else 0)
        bytes_per_update += 73
    # dominant kernel: the (level, launch form) with the largest kernel time.
    # Algorithmic bytes of one launch: 16 populations read and 16 written per
    # cell update, and a fused launch makes two updates per cell (both
    # sub-steps). What a fused launch must move is half of that (the
    # intermediate time level stays on chip): reported as blocked_bytes.
    dom = max(ktimes, key=lambda k: ktimes[k][0])
    dom_ms, dom_calls, dom_cells = ktimes[dom]
    avg_launch_s = dom_ms / 1e3 / dom_calls
    updates_per_launch = dom_cells / dom_calls * (2 if dom[1] else 1)
    bytes_per_launch = updates_per_launch * bytes_per_update
    blocked_bytes = dom_cells / dom_calls * bytes_per_update
    achieved = bytes_per_launch / avg_launch_s / 1e9
    kernel_name = "fused_kernel" if dom[1] else "step_kernel"
    traffic = None
    m = MEASURED_TRAFFIC
    if (kernel_hash() == m["kernel_sha256_16"] and args.workload == m["workload"]
            and args.precision == m["precision"] and tuning and m["kernel"] == kernel_name
            and m["level"] == dom[0] and m["tile_cells"] in (None, tuning["tile_cells"])
            and tuning["flags"] in m["flags"]):
        traffic = m["bytes_per_launch"]
    scale = max(abs(x) for x in T0)
    drift = [float(abs((T1[k] - T0[k]) - (L1[k] - L0[k])) / scale) for k in range(4)]
    # the whole path: algorithmic bytes of every step launch of a coarse step
    # over the timed wall time per coarse step (launches of different levels
    # may overlap on the chip, so this is not a sum of per-launch rates)
    path_bytes = sum(v[2] * (2 if k[1] else 1) for k, v in ktimes.items()) / prof_steps * bytes_per_update
    path_gbs = path_bytes / (wall / args.steps) / 1e9

    out = {
        "metric": "fine-equiv cell updates/s",
        "value": value,
        "unit": "cell updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32s": "f64 math, f32 storage"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{case.name}: {case.nx0}x{case.ny0} coarse, levels {case.nlev}, "
                               f"boxes {case.boxes}, r={case.r}, beta={case.beta}, "
                               f"c={case.c:.4f}, seed 0",
                   "fine_equiv_per_step": fe_step, "actual_updates_per_step": upd,
                   "launches_per_step": nl, "tuning": tuning,
                   "precision": args.precision,
                   "adaptive_dt_kappa": args.adaptive_dt,
                   "adaptive_beta": (dict(zip(("C", "beta_min", "beta_max"), sensor))
                                     if sensor else None)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel_name, "level": dom[0], "bytes_per_launch": bytes_per_launch,
                     "updates_per_launch": updates_per_launch, "bytes_per_update": bytes_per_update,
                     "blocked_bytes_per_launch": blocked_bytes,
                     "avg_launch_us": avg_launch_s * 1e6, "launches": dom_calls,
                     "kernel_share": dom_ms / sum(v[0] for v in ktimes.values()),
                     "timing": f"per-kernel events over {prof_steps} further coarse steps "
                               f"({prof_wall * 1e3 / prof_steps:.4f} ms/step with events)",
                     "path": {"bytes_per_step": path_bytes, "achieved": path_gbs,
                              "frac": path_gbs / HBM_PEAK_GBS}},
        "kernels": [{"level": k[0], "fused": bool(k[1]), "launches_per_step": v[1] / prof_steps,
                     "avg_launch_us": v[0] * 1e3 / v[1],
                     "frac": v[2] / v[1] * (2 if k[1] else 1) * bytes_per_update / (v[0] / 1e3 / v[1]) / 1e9
                     / HBM_PEAK_GBS}
                    for k, v in sorted(ktimes.items()) if v[1]],
        "actual_updates_per_s": upd * args.steps / wall,
        "amr": ({"regrid_every": regrid_every, "regrids": amr_timed["regrids"],
                 "boxes_min": min(amr_timed["boxes"]), "boxes_max": max(amr_timed["boxes"]),
                 "regrid_s": amr_timed["regrid_s"], "max_box": args.amr_max_box,
                 "threshold": args.amr_threshold,
                 "levels": [solver.active_cells(l) for l in range(case.nlev)]}
                if dynamic and amr_timed["boxes"] else None),
        "gpu_event_ms": gpu_ms,
        "conservation_drift_rel": drift,
        "drift_per_step": {"steps": drift_steps, "max_abs": max(abs(x) for d in drift_series for x in d),
                           "series": drift_series},
        "healthy": healthy,
    }
    # the timed solve is done: its device memory goes back before the served
    # stream and the baseline legs run
    solver.close()
    del solver, case
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_serve:
        out["served"] = serve_sweep(args)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        if args.workload == "kh4096":
            out["cpu_baseline"] = cpu_baseline_kh_downscale(args, prec, stream)
        elif args.workload == "kh_strip":
            out["cpu_baseline"] = cpu_baseline_kh_downscale(args, prec, stream, n0=1024, strip=True)
        else:
            out["cpu_baseline"] = cpu_baseline(build_case(args.workload, 10 ** 6), args.cpu_budget,
                                               boxes=timed_boxes if dynamic else None, sensor=sensor,
                                               adaptive_dt=args.adaptive_dt)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
