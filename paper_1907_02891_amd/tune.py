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
    """Cache key: shape, padding, spectrum form, classes and precision (a
    split-precision plan numbers its variants among the matrix-core ones)."""
    py, px = plan.padding
    cls = f"/classes{plan.classes}" if plan.classes > 1 else ""
    prec = f"/precision{plan.precision}" if plan.precision else ""
    return f"{plan.ny}x{plan.nx}/k{plan.ky}x{plan.kx}/p{py}x{px}/form{plan.form}{cls}{prec}"


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


def _stage_times(plan, x, out, reps, warmup, adjoint=False):
    """Mean ms per call of (rows forward, columns, rows inverse)."""
    if plan.classes > 1:  # x: one map per class
        def run():
            plan.convolve_classes(x, out=out)
    else:
        f = plan.adjoint if adjoint else plan.convolve

        def run():
            f(x, out=out)
    for _ in range(warmup):
        run()
    plan.timing(True)
    for _ in range(reps):
        run()
    ms, calls = plan.stage_ms()
    plan.timing(False)
    return [m / calls for m in ms]


def autotune(plan, x=None, out=None, *, reps=20, warmup=3, use_cache=True, verbose=False):
    """Pick the fastest variant of each stage for this plan (bound, with its
    kernel spectra).  x: a map, or for a plan of several source classes a list
    of one map per class.  Returns {stage name: {"variant", "ms", "all":
    [...]}}."""
    import torch
    if x is None:
        x = [torch.rand(plan.ny, plan.nx, device=plan.workspace.device) for _ in range(plan.classes)]
        x = x[0] if plan.classes == 1 else x
    if out is None:
        out = torch.empty_like(x[0] if isinstance(x, (list, tuple)) else x)
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
            ci = cache.get(key, {}).get(name + "_inverse")
            if stage == lp.STAGE_ROWS and ci is not None and 0 <= ci < n:
                plan.set_variant(lp.STAGE_ROWS_INVERSE, ci)
                report[name]["variant_inverse"] = ci
            continue
        times, fwd, inv = [], [], []
        for k in range(n):
            plan.set_variant(stage, k)
            t = _stage_times(plan, x, out, reps, warmup)
            if stage == lp.STAGE_ROWS:
                fwd.append(t[0])
                inv.append(t[2])
                times.append(t[0] + t[2])
            else:
                times.append(t[1])
            if verbose:
                print(f"tune {name} variant {k} {plan.variant_info(stage, k)}: {times[-1] * 1e3:.1f} us", flush=True)
        best = min(range(n), key=lambda k: times[k])
        plan.set_variant(stage, best)
        report[name] = {"variant": best, "ms": times[best], "all": times}
        cache.setdefault(key, {})[name] = best
        if stage == lp.STAGE_ROWS:
            # the two row directions are separate kernels: pick each its own
            bf = min(range(n), key=lambda k: fwd[k])
            bi = min(range(n), key=lambda k: inv[k])
            plan.set_variant(lp.STAGE_ROWS, bf)
            plan.set_variant(lp.STAGE_ROWS_INVERSE, bi)
            report[name].update({"variant": bf, "variant_inverse": bi, "ms": fwd[bf] + inv[bi],
                                 "forward_ms": fwd, "inverse_ms": inv})
            cache[key][name] = bf
            cache[key][name + "_inverse"] = bi
    if use_cache:
        _save_cache(cache)
    return report


def _time_batch(b, xs, ys, reps, warmup):
    import torch
    for _ in range(warmup):
        b.convolve(xs, ys)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        b.convolve(xs, ys)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def length_sets(need_min, need_max, all_lengths):
    """Candidate restrictions of the padded-length set between the smallest
    length >= need_min and the smallest length >= need_max (which is always
    kept): the full range, every second / third length, the top few."""
    L = sorted(all_lengths)
    cap = min([x for x in L if x >= need_max] or [L[-1]])
    lo = min([x for x in L if x >= need_min] or [cap])
    L = [x for x in L if lo <= x <= cap]
    cands = [L]
    for step in (2, 3):
        for start in range(step):
            cands.append(sorted(set(L[start::step]) | {cap}))
    for k in (1, 2, 3):
        cands.append(L[-k:])
    out, seen = [], set()
    for c in cands:
        t = tuple(c)
        if t not in seen:
            seen.add(t)
            out.append(list(c))
    return out


def tune_batch_rows(b, maps, ys, reps=3, warmup=1, verbose=False):
    """Row variants of a bound batch, one choice per padded row length (all
    classes of that length together), timed on the whole batch.  Returns
    {row length: (chosen variant, ms per variant)}."""
    by_px = {}
    for g, info in enumerate(b.groups):
        by_px.setdefault(info["padding"][1], []).append(g)
    out = {}
    for px, gs in sorted(by_px.items()):
        n = b.groups[gs[0]]["row_variants"]
        if n < 2:
            continue
        times = []
        for k in range(n):
            for g in gs:
                b.set_variant(g, lp.STAGE_ROWS, k)
            times.append(_time_batch(b, maps, ys, reps, warmup))
        kbest = min(range(n), key=lambda k: times[k])
        for g in gs:
            b.set_variant(g, lp.STAGE_ROWS, kbest)
        out[str(px)] = (kbest, [round(t, 4) for t in times])
        if verbose:
            print(f"tune batch: rows {px}: variant {kbest} of {times}", flush=True)
    return out


def autotune_batch(shapes, psf_ids, psfs, maps, *, pitch_km=0.5, reps=3, warmup=1, verbose=False):
    """Choose the padding classes of a batch: try restricted length sets
    (fewer, larger classes versus more padding), time each batch on the
    given maps (device tensors); on the fastest, choose the row variants per
    padded row length and the graph branches; return (best Batch, report)."""
    import torch
    ly_all, lx_all = lp.spec_lengths()
    ky = [p.shape[0] for p in psfs]
    kx = [p.shape[1] for p in psfs]
    need = [(s[0] + ky[i] // 2, s[1] + kx[i] // 2) for s, i in zip(shapes, psf_ids)]
    sets_y = length_sets(min(n[0] for n in need), max(n[0] for n in need), ly_all)
    sets_x = length_sets(min(n[1] for n in need), max(n[1] for n in need), lx_all)
    ys = [torch.empty_like(m) for m in maps]
    best, report = None, []
    # the same thinning policy on both axes (the k-th candidate of each)
    for k in range(max(len(sets_y), len(sets_x))):
        sy, sx = sets_y[min(k, len(sets_y) - 1)], sets_x[min(k, len(sets_x) - 1)]
        try:
            b = lp.Batch(shapes, psf_ids, [p.shape for p in psfs], pitch_km, lengths=(sy, sx)).bind()
        except lp.LPError:
            continue
        b.set_kernels(psfs)
        ms = _time_batch(b, maps, ys, reps, warmup)
        report.append({"lengths_y": sy, "lengths_x": sx, "classes": len(b.groups), "ms": ms})
        if verbose:
            print(f"tune batch: {len(b.groups)} classes, {ms:.3f} ms  y={sy} x={sx}", flush=True)
        if best is None or ms < best[0]:
            if best is not None:
                best[1].close()
            best = (ms, b)
        else:
            b.close()
        torch.cuda.empty_cache()
    b = best[1]
    report.append({"row_variants": tune_batch_rows(b, maps, ys, reps, warmup, verbose)})
    # parallel class branches of the captured graph, on the chosen classes
    times = {}
    for n in (1, 2, 3, 4):
        b.set_graph_branches(n)
        times[n] = _time_batch(b, maps, ys, reps, warmup)
        if verbose:
            print(f"tune batch: {n} graph branches, {times[n]:.3f} ms", flush=True)
    n_best = min(times, key=times.get)
    b.set_graph_branches(n_best)
    report.append({"graph_branches_ms": {str(k): v for k, v in times.items()}, "graph_branches": n_best})
    return b, report
