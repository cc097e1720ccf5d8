"""Autotuner for the launch knobs of fdc_run_histories.

Only knobs that cannot change a result bit are searched: waves per workgroup,
persistent grid size, the LDS sub-tally's kind and size, units per wave per round
and the processing order of the histories
(integer tallies make every setting bitwise identical; the GPU tests check
it).  Each candidate is timed on the caller's real plans; the plans are then
rewound (tallies cleared, history counters back to 0), so tuning leaves no
trace in the results.  The choice is cached in a JSON file keyed by device and
workload signature.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

from . import fdc as F

CANDIDATES = (
    [dict(waves_per_block=w) for w in (4, 8, 16)]
    + [dict(waves_per_block=4, blocks_per_cu=4)]
    + [dict(waves_per_block=16, blocks_per_cu=1, tally_slots=4096, units_per_wave=u) for u in (1, 2, 4)]
    + [dict(waves_per_block=8, blocks_per_cu=2, tally_slots=2048, units_per_wave=u) for u in (1, 2, 4)]
    + [dict(waves_per_block=4, blocks_per_cu=4, tally_slots=1024, units_per_wave=u) for u in (2, 4)]
    + [dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=u, tally_mode=1) for u in (1, 2, 4, 8)]
    + [dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=1, tally_mode=2),
       dict(waves_per_block=8, blocks_per_cu=1, tally_slots=8064, units_per_wave=1, tally_mode=2)]
    + [dict(waves_per_block=8, blocks_per_cu=2, tally_slots=3008, units_per_wave=u, tally_mode=1) for u in (2, 4)]
    # histories in start-position order (lanes of a wave start next to each other)
    + [dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=u, tally_mode=1, source_order=1)
       for u in (1, 2, 4)]
    + [dict(waves_per_block=16, blocks_per_cu=1, tally_slots=8064, units_per_wave=u, tally_mode=2, source_order=1)
       for u in (1, 2, 4, 8)]
)


def default_cache_path():
    return os.environ.get("FDC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "fdc_autotune.json"))


def signature(ctx, plans, flags, spots_per_plan, histories_per_plan):
    parts = [f"flags={flags}"]
    for p in plans:
        parts.append(f"{ctx.plans[p]}:{spots_per_plan[p]}:{histories_per_plan[p]}")
    return hashlib.sha1("|".join(parts).encode()).hexdigest()[:16]


def _device_key(ctx):
    try:
        import torch
        name = torch.cuda.get_device_name(ctx.device)
    except Exception:
        name = "unknown"
    return f"{name}|cus={ctx.device_cus()}"


def _time_run(ctx, plans, flags, reps):
    import torch
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.run_histories(plans, flags)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best


def tune(ctx, plans, flags=F.FDC_RUN_VARIANCE, spots_per_plan=None, histories_per_plan=None, reps=2,
         cache_path=None, use_cache=True, candidates=CANDIDATES, log=None):
    """Pick the fastest launch configuration for running `plans` with `flags`,
    apply it to ctx and return (config, timings).  The plans are rewound."""
    plans = [int(p) for p in plans]
    spots_per_plan = spots_per_plan or {p: -1 for p in plans}
    histories_per_plan = histories_per_plan or {p: -1 for p in plans}
    key = _device_key(ctx) + "|" + signature(ctx, plans, flags, spots_per_plan, histories_per_plan)
    path = cache_path or default_cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            cfg = cache[key]["config"]
            ctx.set_launch_config(**cfg)
            return cfg, cache[key].get("timings", {})
    timings = {}
    for cfg in candidates:
        try:
            ctx.set_launch_config(**cfg)
            for p in plans:                            # clear the tallies (histories keep counting), so
                ctx.reset_plan(p)                      # repeated runs of big plans cannot overflow them
            ctx.run_histories(plans, flags)            # warm-up (and first-touch of the tallies)
            t = _time_run(ctx, plans, flags, reps)
        except F.FdcError as e:                        # e.g. an LDS size that does not fit
            if log:
                log(f"autotune: skip {cfg}: {e}")
            continue
        timings[json.dumps(cfg, sort_keys=True)] = t
        if log:
            log(f"autotune: {cfg} {t * 1e3:.2f} ms")
    for p in plans:
        ctx.reset_plan(p, rewind=True)
    best = json.loads(min(timings, key=timings.get))
    ctx.set_launch_config(**best)
    cache[key] = {"config": best, "timings": timings}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(path + ".tmp", path)
    except OSError:
        pass
    return best, timings
