"""Autotuner of the batched step's schedule (one launch per phase with one workgroup or one
wavefront per touched block in the TSDF and label phases, and its grid size; or each map's
own kernels over several streams, and their number).

Each candidate runs the same frames on freshly created maps (the maps are mutated by a
step, so candidates never share them); the step times after the first (which also sizes
the scratch buffers and captures the graph) are compared, by their median or their mean,
and the fastest candidate is cached in a JSON file keyed by the GPU architecture and a
workload signature.  The mean over every step of a workload is the figure to compare when
its steps differ (maps that run out of frames leave later steps smaller): the schedules
that tie on full steps need not tie on the rest.
"""
from __future__ import annotations

import json
import os
import time

# (schedule, grid): schedules 0..3 run one launch per phase (bit 0 = TSDF, bit 1 = labels,
# each 0 workgroup / 1 wavefront per touched block) on a grid of that many workgroups;
# schedule 4 runs each map's own kernels with the maps spread over `grid` streams
CANDIDATES = [(s, g) for s in (0, 1, 2, 3) for g in (1024, 2048, 4096)] + [(4, k) for k in (2, 4, 8, 16)]


def cache_path():
    return os.environ.get("MAPCORE_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mapcore", "batch_tune.json"))


def _arch():
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name)


def tune(signature, build, run_step, n_steps=3, candidates=CANDIDATES, use_cache=True, score="median"):
    """build() -> Batch on fresh maps; run_step(batch, k) runs step k (synchronous); steps
    1..n_steps are timed.  score: "median" or "mean" of those step times.
    Returns (schedule, grid, timings {cand: seconds per step by that score})."""
    import torch
    if score not in ("median", "mean"):
        raise ValueError(f"score must be 'median' or 'mean', not {score!r}")
    key = f"{_arch()}|{signature}|{score}"
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            c = cache[key]
            return c["schedule"], c["grid"], {tuple(map(int, k.split(","))): v for k, v in c["timings"].items()}
    timings = {}
    for sched, grid in candidates:
        batch = build()
        batch.configure(sched, grid, True)
        run_step(batch, 0)
        ts = []
        for k in range(1, n_steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run_step(batch, k)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        timings[(sched, grid)] = ts[len(ts) // 2] if score == "median" else sum(ts) / len(ts)
        for m in batch.maps:
            m.close()
        batch.close()
    best = min(timings, key=timings.get)
    cache[key] = {"schedule": best[0], "grid": best[1],
                  "timings": {f"{k[0]},{k[1]}": v for k, v in timings.items()}}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as fh:
            json.dump(cache, fh, indent=1)
    except OSError:
        pass
    return best[0], best[1], timings
