"""Per-step metrics of a running solve as JSON lines.

Every `every` coarse steps one line: the coarse step count, the conserved
totals T_k and the boundary ledger L_k (Sec. 4.1.2: what entered through
non-periodic sides), the conservation defect ((T - T0) - (L - L0)) / max|T0|
per component, whether every active cell is healthy (rho > 0, p > 0, no
NaN), and the step kernels' time per level since the previous line. Only
library calls: the totals and the health scan are device reductions.
"""
from __future__ import annotations

import json
from typing import IO, List

import numpy as np


def run_logged(solver, n_steps: int, every: int, out: IO[str]) -> List[dict]:
    """Advance `solver` by n_steps coarse steps, writing one line to `out`
    every `every` steps (and after the last); returns the records."""
    if every < 1:
        raise ValueError("every must be >= 1")
    T0, L0 = solver.totals()
    scale = float(np.max(np.abs(T0))) or 1.0
    records = []
    done = 0
    solver.set_profiling(True)
    try:
        while done < n_steps:
            k = min(every, n_steps - done)
            solver.advance(k)
            done += k
            T, L = solver.totals()
            kt = solver.kernel_times()
            solver.set_profiling(True)  # restarts the per-kernel accumulators
            rec = {
                "coarse_steps": solver.steps(),
                "totals": [float(x) for x in T],
                "ledger": [float(x) for x in L],
                "defect_rel": [float(((T[i] - T0[i]) - (L[i] - L0[i])) / scale) for i in range(len(T))],
                "healthy": bool(solver.check_health()),
                "kernel_ms": {f"{lvl}{'f' if fused else ''}": round(v[0], 6) for (lvl, fused), v in kt.items()},
            }
            out.write(json.dumps(rec) + "\n")
            records.append(rec)
    finally:
        solver.set_profiling(False)
    return records
