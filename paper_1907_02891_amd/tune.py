"""Autotuner for the specialised kernels of a plan.

For each stage (rows, columns) the library holds several compile-time
variants of the register-resident kernels for some lengths: different radix
orders, threads per transform, rows per workgroup, register budgets, one or
two tiles per workgroup.  `autotune` runs every variant of each stage on the
plan's own workspace and stream, times it with the library's HIP events
(lp_plan_timing / lp_plan_stage_ms), keeps the fastest, and caches the choice
in a JSON file keyed by the plan's shape (LP_TUNE_CACHE, default
~/.cache/lpfft/tune.json).  The stages are independent, so each is tuned with
the others at their current choice.
"""
from __future__ import annotations

import json
import os

from . import lp

STAGE_NAMES = {lp.STAGE_ROWS: "rows", lp.STAGE_COLUMNS: "columns"}


def cache_path():
    return os.environ.get("LP_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "lpfft",
                                                         "tune.json"))


def plan_key(plan):
    py, px = plan.padding
    return f"{plan.ny}x{plan.nx}/k{plan.ky}x{plan.kx}/p{py}x{px}/form{plan.form}"


def _load_cache():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save_cache(c):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(c, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _stage_time(plan, x, out, stage, reps, warmup, adjoint=False):
    run = plan.adjoint if adjoint else plan.convolve
    for _ in range(warmup):
        run(x, out=out)
    plan.timing(True)
    for _ in range(reps):
        run(x, out=out)
    ms, calls = plan.stage_ms()
    plan.timing(False)
    if stage == lp.STAGE_ROWS:
        return (ms[0] + ms[2]) / calls
    return ms[1] / calls


def autotune(plan, x=None, out=None, *, reps=20, warmup=3, use_cache=True, verbose=False):
    """Pick the fastest variant of each stage for this plan (bound, with its
    kernel spectrum).  Returns {stage name: {"variant", "ms", "all": [...]}}."""
    import torch
    if x is None:
        x = torch.rand(plan.ny, plan.nx, device=plan.workspace.device)
    if out is None:
        out = torch.empty_like(x)
    key = plan_key(plan)
    cache = _load_cache() if use_cache else {}
    report = {}
    for stage in (lp.STAGE_ROWS, lp.STAGE_COLUMNS):
        n = plan.variant_count(stage)
        name = STAGE_NAMES[stage]
        if n <= 1:
            report[name] = {"variant": 0 if n else None, "ms": None, "all": []}
            continue
        cached = cache.get(key, {}).get(name)
        if cached is not None and 0 <= cached < n:
            plan.set_variant(stage, cached)
            report[name] = {"variant": cached, "ms": None, "all": [], "cached": True}
            continue
        times = []
        for k in range(n):
            plan.set_variant(stage, k)
            t = _stage_time(plan, x, out, stage, reps, warmup)
            times.append(t)
            if verbose:
                print(f"tune {name} variant {k} {plan.variant_info(stage, k)}: {t * 1e3:.1f} us", flush=True)
        best = min(range(n), key=lambda k: times[k])
        plan.set_variant(stage, best)
        report[name] = {"variant": best, "ms": times[best], "all": times}
        cache.setdefault(key, {})[name] = best
    if use_cache:
        _save_cache(cache)
    return report
