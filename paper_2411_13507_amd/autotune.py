"""Pick the fastest forward-pass options for a batch signature.

The FP64 polish makes every option set below reach the same optimum (or the
same verified certificate), so the options only move time: between the FP32
ADMM warm start and the polish (iterations, penalty), and between launch
configurations (schedule: one launch per degree group or one for the whole
batch; launch shape: instances per workgroup and the waves per SIMD the
register budget is sized for).  ``tune`` times the (iterations, penalty)
candidates in the default launch configuration, then the launch
configurations with the winner, each on a sample of the batch with HIP
events on the current stream, and caches the result per (GPU architecture,
size signature) in a JSON file.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional, Tuple

import numpy as np
import torch

from . import _lib
from .api import SegmentBatchGPU

CACHE = os.environ.get("RBP_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "rbp_autotune.json"))
CANDIDATES: Tuple[Tuple[int, float], ...] = ((0, 0.1), (5, 0.1), (10, 0.1), (20, 0.1), (10, 0.03), (10, 0.3), (10, 1.0))
# (schedule, launch shape): grouped with one wavefront per workgroup and
# registers for two per SIMD (the default), the same with registers for one
# per SIMD, grouped with two instances per workgroup, one launch for the batch
LAUNCHES: Tuple[Tuple[int, int], ...] = ((0, 0), (0, 1), (0, 2), (1, 0))


def signature(problem) -> str:
    deg = np.asarray(problem.degree)
    nf = np.diff(np.asarray(problem.poly_off))[np.asarray(problem.poly_idx)]
    r = np.diff(np.asarray(problem.reach_off))
    arch = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "cpu"
    return f"{arch}|p{deg.min()}-{deg.max()}|nf{int(np.median(nf))}|r{int(np.median(r))}"


def _load() -> Dict[str, dict]:
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(db: Dict[str, dict]) -> None:
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(db, fh, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def opts_for(admm_iters: int, rho: float, schedule: int = 0, launch_shape: int = 0) -> _lib.SolveOpts:
    o = _lib.default_opts()
    o.admm_iters = int(admm_iters)
    o.rho = float(rho)
    o.schedule = int(schedule)
    o.launch_shape = int(launch_shape)
    return o


def _from_record(rec: dict) -> _lib.SolveOpts:
    return opts_for(rec["admm_iters"], rec["rho"], rec.get("schedule", 0), rec.get("launch_shape", 0))


def tune(problem, sample: int = 4096, reps: int = 5, candidates: Iterable[Tuple[int, float]] = CANDIDATES,
         launches: Iterable[Tuple[int, int]] = LAUNCHES, use_cache: bool = True) -> _lib.SolveOpts:
    """Return the fastest options for ``problem`` (a batch with the C
    description's arrays), measured on its first ``sample`` instances."""
    key = signature(problem)
    db = _load() if use_cache else {}
    if key in db:
        return _from_record(db[key])
    n = min(sample, len(problem.degree))
    sub = problem.subset(range(n)) if hasattr(problem, "subset") else problem
    gb = SegmentBatchGPU(sub)
    x0 = torch.as_tensor(sub.x0, device=gb.device)
    goal = torch.as_tensor(sub.goal, device=gb.device)
    out = gb.alloc_outputs()
    stream = torch.cuda.current_stream(gb.device)

    def time_opts(o):
        o.store_for_backward = 0
        gb.solve(x0, goal, opts=o, out=out)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in evs:
            e0.record(stream)
            gb.solve(x0, goal, opts=o, out=out)
            e1.record(stream)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in evs]))

    timings = {(k, rho): time_opts(opts_for(k, rho)) for k, rho in candidates}
    best = min(timings, key=timings.get)
    shapes = {(sc, sh): time_opts(opts_for(best[0], best[1], sc, sh)) for sc, sh in launches}
    best_l = min(shapes, key=shapes.get)
    gb.close()
    db[key] = {"admm_iters": best[0], "rho": best[1], "schedule": best_l[0], "launch_shape": best_l[1],
               "ms": {f"{k}/{r}": t for (k, r), t in timings.items()},
               "ms_launch": {f"schedule{sc}/shape{sh}": t for (sc, sh), t in shapes.items()}, "sample": n}
    tune.last = db[key]
    if use_cache:
        _store(db)
    return opts_for(best[0], best[1], best_l[0], best_l[1])


tune.last = None


def cached(problem) -> Optional[_lib.SolveOpts]:
    rec = _load().get(signature(problem))
    return None if rec is None else _from_record(rec)
