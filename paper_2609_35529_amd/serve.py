"""Continuous-batching server for independent Riemann-problem solves.

Requests arrive over time (Poisson arrivals from ``workloads.request_stream``).
The loop admits every arrived request whose device footprint
(``vlbm_footprint_bytes``) fits into the free budget. Admitted solves keep their
populations resident in HBM. Each iteration advances all resident solves by one
quantum of coarse steps with ``vlbm_batch_advance``: one launch per phase
serves every solve at once. Solves that finish are read back (their level-0
state) and freed; their slots and bytes go to the next arrivals. Latency is
completion time minus arrival time.

At admission, every `health_every` iterations and when a solve finishes,
each resident solve is scanned (``vlbm_check_health``: rho <= 0, p <= 0 or
NaN on any active cell). An unhealthy solve fails alone: it is reported with ``failed`` set and
freed, and the others continue untouched (their states never share memory).

``run_sequential`` is the reference path: one solve at a time in arrival order,
plain FP64, no batching.

This module schedules and marshals only; every step of the method runs in the
library's kernels.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np

from . import vlbm
from . import workloads as wl


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    done: float
    steps: int
    fine_equiv: float
    state: Optional[np.ndarray] = None
    failed: bool = False

    @property
    def latency(self):
        return self.done - self.arrival


def _percentile(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else float("nan")


def summarize(results: List[Result], wall: float) -> Dict:
    ok = [r for r in results if not r.failed]
    lat = [r.latency for r in ok]
    fe = sum(r.fine_equiv for r in ok)
    return {"solves": len(ok), "failed": len(results) - len(ok), "wall_s": wall,
            "solves_per_s": len(ok) / wall,
            "fine_equiv_per_s": fe / wall, "p50_latency_s": _percentile(lat, 50),
            "p99_latency_s": _percentile(lat, 99), "mean_latency_s": float(np.mean(lat))}


def _fine_equiv(case, steps):
    return case.fine_equivalent_per_coarse_step() * steps


class Server:
    """Admission by footprint + continuous batching of resident solves."""

    # cost model of one coarse step: bytes moved at a sustained bandwidth plus a
    # fixed cost per launch (phase); used only to share GPU time fairly
    BANDWIDTH = 4.5e12
    LAUNCH_S = 6e-6

    def __init__(self, budget_bytes: int, precision=vlbm.FP32_STORAGE, quantum=25,
                 max_resident=64, stream=None, keep_states=False, slice_s=0.02,
                 policy="share", health_every=8, tuning=None):
        """Per iteration, resident solves advance together in shared launches.
        policy "fixed": every solve takes `quantum` coarse steps.
        policy "share": every solve gets an equal share of a slice_s-second
        iteration, converted to steps with the cost model (processor sharing).
        policy "srpt": the slice is filled in order of least remaining work
        (whole remainders first), every solve still taking at least one step, so
        short solves finish early and long ones never stall."""
        self.budget = int(budget_bytes)
        self.precision = precision
        self.quantum = int(quantum)
        self.max_resident = int(max_resident)
        self.stream = stream
        self.keep_states = keep_states
        self.slice_s = slice_s
        self.policy = policy
        self.health_every = int(health_every)
        self.tuning = tuning  # (tile_cells, flags) of every solve (vlbm_set_tuning), or None

    def step_cost(self, case):
        esz = 4 if self.precision == vlbm.FP32 else 8
        return (case.actual_updates_per_coarse_step() * 32 * esz / self.BANDWIDTH
                + case.launches_per_coarse_step() * self.LAUNCH_S)

    def plan(self, resident):
        """Coarse steps each resident solve takes this iteration."""
        if self.policy == "fixed":
            return [min(self.quantum, e["left"]) for e in resident]
        if self.policy == "share":
            share = self.slice_s / max(1, len(resident))
            return [int(max(1, min(e["left"], share // e["cost"]))) for e in resident]
        budget = self.slice_s
        n = [1] * len(resident)
        budget -= sum(e["cost"] for e in resident)
        for i in sorted(range(len(resident)), key=lambda i: resident[i]["left"] * resident[i]["cost"]):
            e = resident[i]
            extra = int(min(e["left"] - 1, max(0.0, budget) // e["cost"]))
            n[i] += extra
            budget -= extra * e["cost"]
        return n

    def run(self, requests: List[dict], time_scale: float = 1.0) -> (List[Result], float):
        """Serve requests (arrival times in seconds, scaled by time_scale)."""
        import torch
        pending = sorted(requests, key=lambda r: r["arrival"])
        queue: List[dict] = []
        resident: List[dict] = []
        results: List[Result] = []
        used = 0
        t0 = time.perf_counter()
        i = 0
        it = 0
        while i < len(pending) or queue or resident:
            now = time.perf_counter() - t0
            while i < len(pending) and pending[i]["arrival"] * time_scale <= now:
                queue.append(pending[i])
                i += 1
            # admission in arrival order while the footprint fits
            while queue and len(resident) < self.max_resident:
                req = queue[0]
                case = wl.request_case(req)
                need = vlbm.footprint_bytes(case, self.precision, max_levels=case.nlev)
                if need > self.budget:
                    raise RuntimeError(f"request {req['id']} needs {need} bytes > budget")
                if used + need > self.budget:
                    break
                queue.pop(0)
                s = vlbm.Solver.from_case(case, precision=self.precision, stream=self.stream)
                if self.tuning:
                    s.set_tuning(*self.tuning)
                if self.health_every > 0 and not s.check_health():  # a bad initial state
                    now = time.perf_counter() - t0
                    results.append(Result(req["id"], req["arrival"] * time_scale, now, now, 0, 0.0,
                                          None, failed=True))
                    s.close()
                    continue
                used += need
                resident.append(dict(req=req, case=case, solver=s, need=need,
                                     left=req["steps"], cost=self.step_cost(case),
                                     admitted=time.perf_counter() - t0))
            if not resident:
                if i < len(pending):  # idle until the next arrival
                    wait = pending[i]["arrival"] * time_scale - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                continue
            n = self.plan(resident)
            vlbm.batch_advance([e["solver"] for e in resident], n)
            it += 1
            scan = self.health_every > 0 and it % self.health_every == 0
            for e, k in zip(resident, n):
                e["left"] -= k
            still = []
            for e in resident:
                if (scan or e["left"] <= 0) and not e["solver"].check_health():
                    r = e["req"]
                    results.append(Result(r["id"], r["arrival"] * time_scale, e["admitted"],
                                          time.perf_counter() - t0, r["steps"] - e["left"], 0.0,
                                          None, failed=True))
                    e["solver"].close()
                    used -= e["need"]
                    continue
                if e["left"] > 0:
                    still.append(e)
                    continue
                state = e["solver"].get_state(0) if self.keep_states else None
                if not self.keep_states:
                    e["solver"].sync()
                done = time.perf_counter() - t0
                r = e["req"]
                results.append(Result(r["id"], r["arrival"] * time_scale, e["admitted"], done,
                                      r["steps"], _fine_equiv(e["case"], r["steps"]), state))
                e["solver"].close()
                used -= e["need"]
            resident = still
        wall = time.perf_counter() - t0
        return results, wall


def run_sequential(requests: List[dict], precision=vlbm.FP64, stream=None, time_scale=1.0,
                   keep_states=False, tuning=None):
    """One solve at a time in arrival order, no batching (tuning: the
    single-solve launch settings, vlbm_set_tuning)."""
    results: List[Result] = []
    t0 = time.perf_counter()
    for req in sorted(requests, key=lambda r: r["arrival"]):
        wait = req["arrival"] * time_scale - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        case = wl.request_case(req)
        adm = time.perf_counter() - t0
        s = vlbm.Solver.from_case(case, precision=precision, stream=stream)
        if tuning:
            s.set_tuning(*tuning)
        s.advance(req["steps"])
        state = s.get_state(0) if keep_states else None
        s.sync()
        done = time.perf_counter() - t0
        results.append(Result(req["id"], req["arrival"] * time_scale, adm, done, req["steps"],
                              _fine_equiv(case, req["steps"]), state))
        s.close()
    return results, time.perf_counter() - t0
